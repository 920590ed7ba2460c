// k_fit_batched.hip -- the round epilogue and labelling of the whole method
// (Algorithm 2, seed pool of Section II-D) for many independent clouds at
// once: seed gather from each cloud's pool, pool coverage by each cloud's new
// modes, per-cloud stable pool compaction, and nearest-mode labels within a
// cloud.  The iterations themselves are the batched fused step
// (k_batched.hip); the greedy merge runs here too, in parallel decision passes
// per cloud; the draws and the seed-count control run on the host between
// rounds.
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
// r2 (squared) of one of the cloud's new modes (rows x_off[c] + k_old[c] ..
// x_off[c] + k_new[c] of the mode store) leaves the pool.  FP32 direct
// differences.
template <int D>
__global__ void bf_cover_kernel(const float* __restrict__ X, int d, const long long* __restrict__ x_off,
                                int ncl, const int32_t* __restrict__ pool, const int32_t* __restrict__ pool_len,
                                const float* __restrict__ mstore, const int32_t* __restrict__ k_old,
                                const int32_t* __restrict__ k_new, float r2, uint8_t* removed, long long n) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int c = cloud_of(x_off, ncl, e);
    if (e - x_off[c] >= pool_len[c] || removed[e]) return;
    const float* x = X + (x_off[c] + pool[e]) * d;
    float xr[D > 0 ? D : 1];
    load_point<D>(x, xr);
    const float* ms = mstore + x_off[c] * d;
    for (int j = k_old[c]; j < k_new[c]; ++j) {
        if (row_dist2<D>(x, xr, ms + (long long)j * d, d) <= r2) {
            removed[e] = 1;
            return;
        }
    }
}

// The greedy merge of a round (Algorithms 1-2, prune modes): cloud c's
// converged seeds [s_off[c], s_off[c+1]) in draw order, each joining the
// first mode within r -- the cloud's modes from earlier rounds (rows x_off[c]
// .. x_off[c] + k_cnt[c] of the mode store), then this round's founders in
// seed order -- or founding a new one.  Decided in parallel passes, one wave
// per seed: a seed is settled once an old mode is within r (first pass), or
// once the first earlier seed of its cloud that is a founder or undecided and
// within r is a founder (it joins), or there is none (it founds); a seed
// whose first such seed is undecided waits for a later pass.  The lowest
// undecided seed of a cloud is always settled, so the passes end.  A state
// read before another wave settles it reads as undecided, which only
// postpones a decision.  Distances are FP32 direct differences, k ascending,
// fused multiply-adds, compared with <= r2.
enum : int32_t { BF_SKIP = -3, BF_UNDECIDED = -2, BF_FOUNDER = -1, BF_JOINED = 0 };
constexpr int kDecideWaves = 4;
constexpr int kCTF = 1024;   // threads of the founders kernel

__device__ __forceinline__ float seed_dist2(const float* __restrict__ a, const float* __restrict__ b, int d) {
    float q = 0.0f;
    for (int k = 0; k < d; ++k) {
        const float t = a[k] - b[k];
        q = fmaf(t, t, q);
    }
    return q;
}

template <bool kFirst>
__global__ __launch_bounds__(64 * kDecideWaves) void bf_decide_kernel(
    const float* __restrict__ S, int d, const uint8_t* __restrict__ conv, const long long* __restrict__ s_off,
    int ncl, const float* __restrict__ mstore, const long long* __restrict__ x_off, const int32_t* __restrict__ k_cnt,
    float r2, int32_t* state, int32_t* und, int M) {
    const int g = blockIdx.x * kDecideWaves + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= M) return;
    if (kFirst && conv[g] != ST_CONVERGED) {
        if (lane == 0) __atomic_store_n(&state[g], (int32_t)BF_SKIP, __ATOMIC_RELAXED);
        return;
    }
    if (__atomic_load_n(&state[g], __ATOMIC_RELAXED) != BF_UNDECIDED) return;
    const int c = cloud_of(s_off, ncl, g);
    const float* sg = S + (long long)g * d;
    if (kFirst) {
        const float* ms = mstore + x_off[c] * d;
        const int K = k_cnt[c];
        for (int base = 0; base < K; base += 64) {
            const int j = base + lane;
            const bool hit = j < K && seed_dist2(sg, ms + (long long)j * d, d) <= r2;
            if (__ballot(hit)) {
                if (lane == 0) __atomic_store_n(&state[g], (int32_t)BF_JOINED, __ATOMIC_RELAXED);
                return;
            }
        }
    }
    int result = BF_FOUNDER;
    for (long long base = s_off[c]; base < g; base += 64) {
        const long long j = base + lane;
        int sj = BF_SKIP;
        bool hit = false;
        if (j < g) {
            sj = __atomic_load_n(&state[j], __ATOMIC_RELAXED);
            if (sj == BF_FOUNDER || sj == BF_UNDECIDED) hit = seed_dist2(sg, S + j * d, d) <= r2;
        }
        const unsigned long long bal = __ballot(hit);
        if (bal) {
            const int first = __ffsll((unsigned long long)bal) - 1;
            const int sf = __shfl(sj, first);
            result = sf == BF_FOUNDER ? BF_JOINED : BF_UNDECIDED;
            break;
        }
    }
    if (lane == 0) {
        if (result != BF_UNDECIDED) __atomic_store_n(&state[g], result, __ATOMIC_RELAXED);
        else atomicAdd(und, 1);
    }
}

// After the passes: cloud c's founders, in seed order, become its modes
// k_cnt[c], k_cnt[c] + 1, ... (rows of the mode store); k_old[c] keeps the
// count before the round.  One workgroup per cloud.
__global__ __launch_bounds__(kCTF) void bf_founders_kernel(const float* __restrict__ S, int d,
                                                          const long long* __restrict__ s_off,
                                                          const int32_t* __restrict__ state,
                                                          const long long* __restrict__ x_off, float* mstore,
                                                          int32_t* k_cnt, int32_t* k_old) {
    __shared__ int wsum[kCTF / 64];
    __shared__ long long rows[kCTF];
    const int c = blockIdx.x;
    const long long s0 = s_off[c], s1 = s_off[c + 1];
    const int K0 = k_cnt[c];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* ms = mstore + x_off[c] * d;
    int carry = 0;
    for (long long e0 = s0; e0 < s1; e0 += kCTF) {
        const long long g = e0 + threadIdx.x;
        const bool f = g < s1 && state[g] == BF_FOUNDER;
        const unsigned long long bal = __ballot(f);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kCTF / 64; ++w) {
            if (w < wave) before += wsum[w];
            total += wsum[w];
        }
        if (f) rows[before + __popcll(bal & ((1ull << lane) - 1ull))] = g;
        __syncthreads();
        // the founders' rows, contiguous in the store (a cloud's seeds are
        // distinct points of it, so its modes never outnumber its rows;
        // checked all the same)
        const long long cap = x_off[c + 1] - x_off[c];
        for (int e = threadIdx.x; e < total * d; e += kCTF) {
            const int r = e / d, k = e - r * d;
            if (K0 + carry + r < cap) ms[(long long)(K0 + carry + r) * d + k] = S[rows[r] * d + k];
        }
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        k_old[c] = K0;
        k_cnt[c] = K0 + carry;
    }
}

// The modes of every cloud, back to back (cloud c at rows k_off[c] ..): one
// workgroup per cloud.
__global__ void bf_modes_out_kernel(const float* __restrict__ mstore, int d, const long long* __restrict__ x_off,
                                    const int32_t* __restrict__ k_off, float* modes) {
    const int c = blockIdx.x;
    const float* ms = mstore + x_off[c] * d;
    float* out = modes + (long long)k_off[c] * d;
    const long long cnt = (long long)(k_off[c + 1] - k_off[c]) * d;
    for (long long e = threadIdx.x; e < cnt; e += blockDim.x) out[e] = ms[e];
}

__global__ void bf_fill_i32_kernel(int32_t* a, long long count, int32_t v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) a[i] = v;
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
                           const int32_t* pool_len, const float* mstore, const int32_t* k_old,
                           const int32_t* k_new, float r2, uint8_t* removed, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define FMS_COVER(DD)                                                                                  \
    hipLaunchKernelGGL(bf_cover_kernel<DD>, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, X, d, x_off, \
                       ncl, pool, pool_len, mstore, k_old, k_new, r2, removed, n)
    FMS_DSWITCH_ROWS(d, FMS_COVER);
#undef FMS_COVER
    return hipGetLastError();
}

hipError_t launch_bf_merge_init(int32_t* state, int M, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(bf_fill_i32_kernel, dim3((M + kT - 1) / kT), dim3(kT), 0, s, state, (long long)M,
                       (int32_t)BF_UNDECIDED);
    return hipGetLastError();
}

hipError_t launch_bf_decide_pass(const float* S, int d, const uint8_t* conv, const long long* s_off, int ncl,
                                 const float* mstore, const long long* x_off, const int32_t* k_cnt, float r2,
                                 int32_t* state, int32_t* und, int M, bool first, hipStream_t s) {
    hipLaunchKernelGGL(bf_fill_i32_kernel, dim3(1), dim3(64), 0, s, und, 1LL, 0);
    if (M <= 0) return hipGetLastError();
    const dim3 grid((M + kDecideWaves - 1) / kDecideWaves);
    if (first)
        hipLaunchKernelGGL(bf_decide_kernel<true>, grid, dim3(64 * kDecideWaves), 0, s, S, d, conv, s_off, ncl,
                           mstore, x_off, k_cnt, r2, state, und, M);
    else
        hipLaunchKernelGGL(bf_decide_kernel<false>, grid, dim3(64 * kDecideWaves), 0, s, S, d, conv, s_off, ncl,
                           mstore, x_off, k_cnt, r2, state, und, M);
    return hipGetLastError();
}

hipError_t launch_bf_founders(const float* S, int d, const long long* s_off, int ncl, const int32_t* state,
                              const long long* x_off, float* mstore, int32_t* k_cnt, int32_t* k_old, hipStream_t s) {
    hipLaunchKernelGGL(bf_founders_kernel, dim3(ncl), dim3(kCTF), 0, s, S, d, s_off, state, x_off, mstore, k_cnt,
                       k_old);
    return hipGetLastError();
}

hipError_t launch_bf_modes_out(const float* mstore, int d, const long long* x_off, int ncl, const int32_t* k_off,
                               float* modes, hipStream_t s) {
    hipLaunchKernelGGL(bf_modes_out_kernel, dim3(ncl), dim3(256), 0, s, mstore, d, x_off, k_off, modes);
    return hipGetLastError();
}

hipError_t launch_bf_fill_i32(int32_t* a, long long count, int32_t v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(bf_fill_i32_kernel, dim3((unsigned)((count + kT - 1) / kT)), dim3(kT), 0, s, a, count, v);
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
