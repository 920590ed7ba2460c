// k_sort.hip -- spatial order of the points for the BF16 step (gfx950).
//
// The BF16 form centres every 256-point block of points on a local reference
// so that the bf16 products stay accurate; that needs blocks that are compact
// in space.  Points are ordered by the Morton code of their quantized
// coordinates (D <= 4) with a stable LSD radix sort, deterministic (no
// floating-point atomics; ranks inside a block come from wave ballots in wave
// order).  The order only changes which points share a block: the update sums
// over all points whatever their order.

#include "fms_internal.h"

namespace fms {

namespace {

constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / 64;

// Per-dimension min/max of the packed points (first D of DP columns).
__global__ __launch_bounds__(256) void bounds_kernel(const float* __restrict__ Xp, int n, int DP,
                                                     int D, float* out /* 2*D, init +/-inf */) {
    __shared__ float smin[256], smax[256];
    for (int k = 0; k < D; ++k) {
        float lo = __builtin_inff(), hi = -__builtin_inff();
        for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
            const float v = Xp[(long long)i * DP + k];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        smin[threadIdx.x] = lo;
        smax[threadIdx.x] = hi;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
                smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + off]);
                smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + off]);
            }
            __syncthreads();
        }
        // per-block results go to a scratch row; the host-side launcher reduces
        // them in a second pass (see bounds_final_kernel)
        if (threadIdx.x == 0) {
            out[2 * D + (2 * blockIdx.x) * D + k] = smin[0];
            out[2 * D + (2 * blockIdx.x + 1) * D + k] = smax[0];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void bounds_final_kernel(float* out, int D, int blocks) {
    __shared__ float lo_s[256], hi_s[256];
    for (int k = 0; k < D; ++k) {
        float lo = __builtin_inff(), hi = -__builtin_inff();
        for (int b = threadIdx.x; b < blocks; b += 256) {
            lo = fminf(lo, out[2 * D + (2 * b) * D + k]);
            hi = fmaxf(hi, out[2 * D + (2 * b + 1) * D + k]);
        }
        lo_s[threadIdx.x] = lo;
        hi_s[threadIdx.x] = hi;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
                lo_s[threadIdx.x] = fminf(lo_s[threadIdx.x], lo_s[threadIdx.x + off]);
                hi_s[threadIdx.x] = fmaxf(hi_s[threadIdx.x], hi_s[threadIdx.x + off]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[2 * k] = lo_s[0];
            out[2 * k + 1] = hi_s[0];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ unsigned spread_bits(unsigned v, int D) {
    // interleave: bit b of v goes to bit b*D
    unsigned r = 0;
    for (int b = 0; b < 30 / D; ++b) r |= ((v >> b) & 1u) << (b * D);
    return r;
}

__global__ void morton_kernel(const float* __restrict__ Xp, int n, int DP, int D,
                              const float* __restrict__ bnd, unsigned* keys, int* vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int bits = 30 / D;
    const float cells = (float)(1u << bits);
    unsigned key = 0;
    for (int k = 0; k < D; ++k) {
        const float lo = bnd[2 * k], hi = bnd[2 * k + 1];
        const float span = hi - lo;
        float f = span > 0.0f ? (Xp[(long long)i * DP + k] - lo) / span * cells : 0.0f;
        int c = (int)f;
        c = c < 0 ? 0 : (c >= (int)cells ? (int)cells - 1 : c);
        key |= spread_bits((unsigned)c, D) << k;
    }
    keys[i] = key;
    vals[i] = i;
}

// Stable LSD radix sort, 8 bits per pass.
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const unsigned* __restrict__ keys,
                                                                  int n, int shift, int nblocks,
                                                                  int* hist) {
    __shared__ int h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    __syncthreads();
    if (threadIdx.x < 256) hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of hist (digit-major, 256 * nblocks entries) in one block:
// each thread scans a contiguous segment, one block-wide scan of the segment
// totals, then each segment adds its offset.
__global__ __launch_bounds__(1024) void radix_scan_kernel(int* hist, int total) {
    __shared__ int seg[1024];
    const int per = (total + 1023) / 1024;
    const int lo = threadIdx.x * per;
    const int hi = min(total, lo + per);
    int sum = 0;
    for (int e = lo; e < hi; ++e) sum += hist[e];
    seg[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int add = threadIdx.x >= off ? seg[threadIdx.x - off] : 0;
        __syncthreads();
        seg[threadIdx.x] += add;
        __syncthreads();
    }
    int run = seg[threadIdx.x] - sum;   // exclusive offset of this segment
    for (int e = lo; e < hi; ++e) {
        const int v = hist[e];
        hist[e] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const unsigned* __restrict__ kin, const int* __restrict__ vin, int n, int shift, int nblocks,
    const int* __restrict__ offs, unsigned* kout, int* vout) {
    __shared__ int wcount[kSortWaves][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < kSortWaves * 256; e += kSortThreads) (&wcount[0][0])[e] = 0;
    __syncthreads();
    const int i = blockIdx.x * kSortThreads + threadIdx.x;
    const bool live = i < n;
    const unsigned key = live ? kin[i] : 0u;
    const unsigned dig = (key >> shift) & 255u;
    // lanes of this wave with the same digit
    unsigned long long peers = __ballot(live);
    for (int b = 0; b < 8; ++b) {
        const unsigned long long bal = __ballot(live && ((dig >> b) & 1u));
        peers &= ((dig >> b) & 1u) ? bal : ~bal;
    }
    const int rank = __popcll(peers & ((1ull << lane) - 1ull));
    // the lowest peer lane records the wave's count for this digit
    if (live && rank == 0) wcount[wave][dig] = __popcll(peers);
    __syncthreads();
    // exclusive prefix over waves, per digit (wave order = index order)
    if (threadIdx.x < 256) {
        int s = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            const int c = wcount[w][threadIdx.x];
            wcount[w][threadIdx.x] = s;
            s += c;
        }
    }
    __syncthreads();
    if (live) {
        const int pos = offs[dig * nblocks + blockIdx.x] + wcount[wave][dig] + rank;
        kout[pos] = key;
        vout[pos] = vin[i];
    }
}

__global__ void gather_rows_kernel(const float* __restrict__ Xp, int DP, const int* __restrict__ perm,
                                   int n, float* Xs) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * DP) return;
    const int i = (int)(e / DP), k = (int)(e % DP);
    Xs[e] = Xp[(long long)perm[i] * DP + k];
}

// Per 256-point block of the sorted points: centre = midpoint of the bounding
// box, radius = max distance of a block point from the centre (FP32, rounded
// up slightly so that it bounds the FP32 distances the step computes).
// geom row (kGeomStride floats): centre[0..D), radius at [4].
__global__ __launch_bounds__(256) void block_geom_kernel(const float* __restrict__ Xs, int n, int DP,
                                                         int D, float* geom) {
    __shared__ float red[256];
    __shared__ float ctr[4];
    const int b = blockIdx.x;
    const int i = b * 256 + threadIdx.x;
    const bool live = i < n;
    for (int k = 0; k < D; ++k) {
        const float v = live ? Xs[(long long)i * DP + k] : 0.0f;
        red[threadIdx.x] = live ? v : __builtin_inff();
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] = fminf(red[threadIdx.x], red[threadIdx.x + off]);
            __syncthreads();
        }
        const float lo = red[0];
        __syncthreads();
        red[threadIdx.x] = live ? v : -__builtin_inff();
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
            __syncthreads();
        }
        if (threadIdx.x == 0) ctr[k] = 0.5f * (lo + red[0]);
        __syncthreads();
    }
    float r2 = 0.0f;
    if (live)
        for (int k = 0; k < D; ++k) {
            const float t = Xs[(long long)i * DP + k] - ctr[k];
            r2 = fmaf(t, t, r2);
        }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x < kGeomStride) {
        float* g = geom + (long long)b * kGeomStride;
        if (threadIdx.x < D) g[threadIdx.x] = ctr[threadIdx.x];
        else if (threadIdx.x == 4) g[threadIdx.x] = sqrtf(red[0]) * 1.0001f + 1e-30f;
        else g[threadIdx.x] = 0.0f;
    }
}

}  // namespace

size_t sort_workspace_bytes(int n) {
    const size_t nblocks = (n + kSortThreads - 1) / kSortThreads;
    // keys x2, vals x2, hist, bounds scratch (2*4 + 2*4*256 floats)
    return (size_t)n * 4 * 4 + nblocks * 256 * 4 + (8 + 2 * 4 * 256) * 4 + 1024;
}

// Packed points Xp (n x DP) -> sorted copy Xs, permutation perm (Xs[i] =
// Xp[perm[i]]) and per-256-block geometry (centre, radius).
hipError_t launch_spatial_sort(const float* Xp, int n, int DP, int D, float* Xs, int* perm,
                               float* geom, void* ws, hipStream_t s) {
    const int nblocks = (n + kSortThreads - 1) / kSortThreads;
    char* w = (char*)ws;
    unsigned* k0 = (unsigned*)w; w += (size_t)n * 4;
    unsigned* k1 = (unsigned*)w; w += (size_t)n * 4;
    int* v0 = (int*)w; w += (size_t)n * 4;
    int* v1 = perm;
    int* vtmp = (int*)w; w += (size_t)n * 4;
    int* hist = (int*)w; w += (size_t)nblocks * 256 * 4;
    float* bnd = (float*)w;
    const int bblocks = 256;
    hipLaunchKernelGGL(bounds_kernel, dim3(bblocks), dim3(256), 0, s, Xp, n, DP, D, bnd);
    hipLaunchKernelGGL(bounds_final_kernel, dim3(1), dim3(256), 0, s, bnd, D, bblocks);
    hipLaunchKernelGGL(morton_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Xp, n, DP, D, bnd, k0, v0);
    // 4 passes over 30-bit keys; the result lands in (k0, v0) after an even count
    unsigned* ka = k0; unsigned* kb = k1;
    int* va = v0; int* vb = vtmp;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = pass * 8;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, ka, n, shift,
                           nblocks, hist);
        hipLaunchKernelGGL(radix_scan_kernel, dim3(1), dim3(1024), 0, s, hist, 256 * nblocks);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, ka, va, n,
                           shift, nblocks, hist, kb, vb);
        unsigned* tk = ka; ka = kb; kb = tk;
        int* tv = va; va = vb; vb = tv;
    }
    hipError_t e = hipMemcpyAsync(v1, va, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)(((long long)n * DP + 255) / 256)), dim3(256),
                       0, s, Xp, DP, perm, n, Xs);
    hipLaunchKernelGGL(block_geom_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Xs, n, DP, D, geom);
    return hipGetLastError();
}

}  // namespace fms
