// k_fit_batched.hip -- the round epilogue and labelling of the whole method
// (Algorithm 2, seed pool of Section II-D) for many independent clouds at
// once: seed gather from each cloud's pool, pool coverage by each cloud's new
// modes, per-cloud stable pool compaction, and nearest-mode labels within a
// cloud.  The iterations themselves are the batched fused step
// (k_batched.hip); the draws, the greedy merge and the seed-count control run
// on the host between rounds.
//
// Layout: cloud c owns the points X[x_off[c], x_off[c+1]) and the pool slice
// pool[x_off[c], x_off[c] + pool_len[c]) of cloud-local point ids in
// ascending order; removed[] flags pool entries (by position) that leave the
// pool this round.

#include "fms_internal.h"

namespace fms {

namespace {

constexpr int kT = 256;

// Row widths with a register-resident form; other d take the generic loop (D = 0).
#define FMS_DSWITCH_ROWS(d_, CALL) \
    switch (d_) {                  \
        case 1: CALL(1); break;    \
        case 2: CALL(2); break;    \
        case 3: CALL(3); break;    \
        case 4: CALL(4); break;    \
        case 8: CALL(8); break;    \
        case 16: CALL(16); break;  \
        case 32: CALL(32); break;  \
        default: CALL(0); break;   \
    }

__device__ __forceinline__ int cloud_of(const long long* __restrict__ off, int ncl, long long v) {
    // the cloud c with off[c] <= v < off[c + 1] (off ascending; empty clouds skipped)
    int lo = 0, hi = ncl;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Initial pools: every point of its cloud, pool[e] = e - x_off[c].
__global__ void bf_iota_kernel(const long long* __restrict__ x_off, int ncl, int32_t* pool, long long n) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    pool[e] = (int32_t)(e - x_off[cloud_of(x_off, ncl, e)]);
}

// Seed g of the round belongs to cloud c (s_off[c] <= g < s_off[c+1]) and was
// drawn at pool position pos[g] of that cloud: seeds[g] = X[x_off[c] + id]
// with id = pool[x_off[c] + pos[g]], and the pool entry leaves the pool.
__global__ void bf_gather_kernel(const float* __restrict__ X, int d, const long long* __restrict__ x_off,
                                 const long long* __restrict__ s_off, int ncl, const int32_t* __restrict__ pos,
                                 const int32_t* __restrict__ pool, uint8_t* removed, float* seeds, int M) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M) return;
    const int c = cloud_of(s_off, ncl, g);
    const long long e = x_off[c] + pos[g];
    const long long row = x_off[c] + pool[e];
    removed[e] = 1;
    for (int k = 0; k < d; ++k) seeds[(long long)g * d + k] = X[row * d + k];
}

// Squared FP32 distance (direct differences, k ascending) of a point to row m:
// D > 0 with the point in registers, D = 0 for any d.
template <int D>
__device__ __forceinline__ float row_dist2(const float* __restrict__ x, const float (&xr)[D > 0 ? D : 1],
                                           const float* __restrict__ m, int d) {
    float q = 0.0f;
    if constexpr (D > 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float t = xr[k] - m[k];
            q = fmaf(t, t, q);
        }
    } else {
        for (int k = 0; k < d; ++k) {
            const float t = x[k] - m[k];
            q = fmaf(t, t, q);
        }
    }
    return q;
}

template <int D>
__device__ __forceinline__ void load_point(const float* __restrict__ x, float (&xr)[D > 0 ? D : 1]) {
    if constexpr (D > 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) xr[k] = x[k];
    }
}

// Pool coverage: every pool entry of cloud c still in the pool and within
// r2 (squared) of one of the cloud's new modes (rows m_off[c] .. m_off[c+1]
// of nm) leaves the pool.  FP32 direct differences.
template <int D>
__global__ void bf_cover_kernel(const float* __restrict__ X, int d, const long long* __restrict__ x_off,
                                int ncl, const int32_t* __restrict__ pool, const int32_t* __restrict__ pool_len,
                                const float* __restrict__ nm, const int32_t* __restrict__ m_off, float r2,
                                uint8_t* removed, long long n) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int c = cloud_of(x_off, ncl, e);
    if (e - x_off[c] >= pool_len[c] || removed[e]) return;
    const float* x = X + (x_off[c] + pool[e]) * d;
    float xr[D > 0 ? D : 1];
    load_point<D>(x, xr);
    for (int j = m_off[c]; j < m_off[c + 1]; ++j) {
        if (row_dist2<D>(x, xr, nm + (long long)j * d, d) <= r2) {
            removed[e] = 1;
            return;
        }
    }
}

// Stable compaction of each cloud's pool slice, one workgroup of kCT
// threads per cloud: entries not removed keep their order (the pool stays
// ascending); the removed flags of the slice are cleared for the next round.
constexpr int kCT = 1024;

__global__ __launch_bounds__(kCT) void bf_compact_kernel(const long long* __restrict__ x_off,
                                                        const int32_t* __restrict__ pool_in, uint8_t* removed,
                                                        int32_t* pool_len, int32_t* pool_out) {
    __shared__ int wsum[kCT / 64];
    const int c = blockIdx.x;
    const long long base = x_off[c];
    const int len = pool_len[c];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int carry = 0;
    for (int e0 = 0; e0 < len; e0 += kCT) {
        const int e = e0 + threadIdx.x;
        bool keep = false;
        int32_t v = 0;
        if (e < len) {
            keep = !removed[base + e];
            v = pool_in[base + e];
            removed[base + e] = 0;
        }
        const unsigned long long bal = __ballot(keep);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int before = carry, total = 0;
        for (int w = 0; w < kCT / 64; ++w) {
            if (w < wave) before += wsum[w];
            total += wsum[w];
        }
        if (keep) pool_out[base + before + __popcll(bal & ((1ull << lane) - 1ull))] = v;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) pool_len[c] = carry;
}

// Labels: point i of cloud c gets the index (within the cloud) of its nearest
// mode among rows m_off[c] .. m_off[c+1] of modes, ties to the lowest index
// (strict '<' in increasing order); FP32 direct differences.
template <int D>
__global__ void bf_assign_kernel(const float* __restrict__ X, int d, const long long* __restrict__ x_off,
                                 int ncl, const float* __restrict__ modes, const int32_t* __restrict__ m_off,
                                 int32_t* labels, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cloud_of(x_off, ncl, i);
    const float* x = X + i * d;
    float xr[D > 0 ? D : 1];
    load_point<D>(x, xr);
    float best = __builtin_inff();
    int arg = 0;
    for (int j = m_off[c]; j < m_off[c + 1]; ++j) {
        const float q = row_dist2<D>(x, xr, modes + (long long)j * d, d);
        if (q < best) {
            best = q;
            arg = j - m_off[c];
        }
    }
    labels[i] = arg;
}

}  // namespace

hipError_t launch_bf_iota(const long long* x_off, int ncl, int32_t* pool, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(bf_iota_kernel, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, x_off, ncl, pool, n);
    return hipGetLastError();
}

hipError_t launch_bf_gather(const float* X, int d, const long long* x_off, const long long* s_off, int ncl,
                            const int32_t* pos, const int32_t* pool, uint8_t* removed, float* seeds, int M,
                            hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(bf_gather_kernel, dim3((M + kT - 1) / kT), dim3(kT), 0, s, X, d, x_off, s_off, ncl, pos,
                       pool, removed, seeds, M);
    return hipGetLastError();
}

hipError_t launch_bf_cover(const float* X, int d, const long long* x_off, int ncl, const int32_t* pool,
                           const int32_t* pool_len, const float* nm, const int32_t* m_off, float r2,
                           uint8_t* removed, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define FMS_COVER(DD)                                                                                  \
    hipLaunchKernelGGL(bf_cover_kernel<DD>, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, X, d, x_off, \
                       ncl, pool, pool_len, nm, m_off, r2, removed, n)
    FMS_DSWITCH_ROWS(d, FMS_COVER);
#undef FMS_COVER
    return hipGetLastError();
}

hipError_t launch_bf_compact(const long long* x_off, int ncl, const int32_t* pool_in, uint8_t* removed,
                             int32_t* pool_len, int32_t* pool_out, hipStream_t s) {
    hipLaunchKernelGGL(bf_compact_kernel, dim3(ncl), dim3(kCT), 0, s, x_off, pool_in, removed, pool_len, pool_out);
    return hipGetLastError();
}

hipError_t launch_bf_assign(const float* X, int d, const long long* x_off, int ncl, const float* modes,
                            const int32_t* m_off, int32_t* labels, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define FMS_ASSIGN(DD)                                                                                 \
    hipLaunchKernelGGL(bf_assign_kernel<DD>, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, X, d, x_off, \
                       ncl, modes, m_off, labels, n)
    FMS_DSWITCH_ROWS(d, FMS_ASSIGN);
#undef FMS_ASSIGN
    return hipGetLastError();
}

}  // namespace fms
