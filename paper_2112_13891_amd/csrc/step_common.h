// step_common.h -- device code shared by the FP32 and BF16 fused steps:
// launch geometry, the early-stop count, the per-seed update and convergence
// test, tile finalize with ballot compaction, and the reduction kernel for
// chunk partials.  Included by the step translation units only.
#pragma once

#include "fms_internal.h"

namespace fms {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMinChunk = 256;   // points per (tile, chunk) work item, at least
constexpr int kMaxGrid = 2048;   // 8 workgroups of 4 waves on each of 256 CUs

__device__ __forceinline__ int chunks_for(int m, int TS, int n, int grid) {
    int tiles = (m + TS - 1) / TS;
    if (tiles >= grid) return 1;
    int c = grid / tiles;
    int cmax = (n + kMinChunk - 1) / kMinChunk;
    if (c > cmax) c = cmax;
    return c < 1 ? 1 : c;
}

__device__ __forceinline__ int active_count(const Ctl* ctl, int t) {
    // early stop (Section II-C): once `need` seeds converged, nothing is active
    int conv = 0;
    for (int u = 0; u < t; ++u) conv += ctl->conv_it[u];
    return (conv >= ctl->need) ? 0 : ctl->count[t % 3];
}

struct StepArgs {
    const float* Xp;
    int n, d;
    float* S;
    const int32_t* act_in;
    int32_t* act_out;
    uint8_t* status;
    int32_t* iters;
    float* shift2;
    float* part;
    Ctl* ctl;
    float h2, scale, inv_scale, thr2;
};

// Update and convergence test of one seed (slot of the active list) from its
// sums a[0..D) = sum w (x - s) (packed units) and a[D] = sum w.  Returns
// 1 if the seed stays active, 2 if it converged, 0 otherwise.
template <int D, int DP>
__device__ __forceinline__ int update_seed(const StepArgs& a, int slot, const float* v) {
    const int j = a.act_in[slot];
    const float W = v[D];
    if (!(W > 0.0f) || !isfinite(W)) {
        a.status[j] = ST_FAILED;
        return 0;
    }
    float sh2 = 0.0f;
    float* sj = a.S + (long long)j * DP;
    bool finite = true;
    const float inv = a.inv_scale / W;
    // padded coordinates (k >= d) carry exact zeros, so looping to D is exact
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float dk = v[k] * inv;
        finite = finite && isfinite(dk);
        sh2 = fmaf(dk, dk, sh2);
        sj[k] = sj[k] + dk;
    }
    a.iters[j] += 1;
    a.shift2[j] = sh2;
    if (!finite) {
        a.status[j] = ST_FAILED;
        return 0;
    }
    if (sh2 < a.thr2) {
        a.status[j] = ST_CONVERGED;
        return 2;
    }
    return 1;
}

// Finalize the seeds of one tile from sums[k * TS + pos] (one lane per seed).
template <int D, int DP, int R>
__device__ void finalize_tile(const StepArgs& a, int t, int m, int tile, const float* sums) {
    constexpr int TS = 64 * R;
    const int pos = threadIdx.x;
    const int slot = tile * TS + pos;
    int res = 0;
    if (pos < TS && slot < m) {
        float v[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) v[k] = sums[k * TS + pos];
        res = update_seed<D, DP>(a, slot, v);
    }
    const int lane = threadIdx.x & 63;
    const unsigned long long keep = __ballot(res == 1);
    const unsigned long long done = __ballot(res == 2);
    int base = 0;
    if (lane == 0) {
        if (keep) base = atomicAdd(&a.ctl->count[(t + 1) % 3], __popcll(keep));
        if (done) atomicAdd(&a.ctl->conv_it[t], __popcll(done));
    }
    base = __shfl(base, 0);
    if (res == 1) a.act_out[base + __popcll(keep & ((1ull << lane) - 1ull))] = a.act_in[slot];
}

// Reduction of the chunk partials and finalize (only when chunks > 1), in
// 1024-thread blocks.  Many chunks and few seeds: one wave per seed; its lanes
// add the partials lane-strided, then in a fixed butterfly, and the block's 16
// seeds are finalized by 16 lanes of wave 0 (one compaction atomic per block).
// Otherwise one lane per seed adds its partials in chunk order and each wave
// compacts its 64 seeds with one ballot and one atomic.
constexpr int kFinThreads = 1024;
constexpr int kFinWaves = kFinThreads / 64;

template <int D, int DP>
__device__ __forceinline__ void compact_wave(const StepArgs& a, int t, int slot, int res) {
    const int lane = threadIdx.x & 63;
    const unsigned long long keep = __ballot(res == 1);
    const unsigned long long done = __ballot(res == 2);
    int off = 0;
    if (lane == 0) {
        if (keep) off = atomicAdd(&a.ctl->count[(t + 1) % 3], __popcll(keep));
        if (done) atomicAdd(&a.ctl->conv_it[t], __popcll(done));
    }
    off = __shfl(off, 0);
    if (res == 1) a.act_out[off + __popcll(keep & ((1ull << lane) - 1ull))] = a.act_in[slot];
}

template <int D, int DP, int R>
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(StepArgs a, int t, int grid) {
    constexpr int TS = 64 * R;
    const int m = active_count(a.ctl, t);
    if (m == 0) return;
    const int chunks = chunks_for(m, TS, a.n, grid);
    if (chunks == 1) return;   // finalized inside the step kernel
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __shared__ float sums[kFinWaves][D + 1];
    if (chunks > 64 && m <= 8192) {
        for (int base = blockIdx.x * kFinWaves; base < m; base += gridDim.x * kFinWaves) {
            const int slot = base + wave;
            if (slot < m) {
                const int tile = slot / TS, pos = slot % TS;
                float v[D + 1];
#pragma unroll
                for (int k = 0; k <= D; ++k) v[k] = 0.0f;
                const float* src = a.part + ((long long)tile * chunks * TS + pos) * (D + 1);
                for (int c = lane; c < chunks; c += 64) {
                    const float* p = src + (long long)c * TS * (D + 1);
#pragma unroll
                    for (int k = 0; k <= D; ++k) v[k] += p[k];
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
                    for (int k = 0; k <= D; ++k) v[k] += __shfl_xor(v[k], off);
                if (lane == 0) {
#pragma unroll
                    for (int k = 0; k <= D; ++k) sums[wave][k] = v[k];
                }
            }
            __syncthreads();
            if (wave == 0) {
                const int my = base + lane;
                int res = 0;
                if (lane < kFinWaves && my < m) res = update_seed<D, DP>(a, my, sums[lane]);
                compact_wave<D, DP>(a, t, my, res);
            }
            __syncthreads();
        }
        return;
    }
    const int nwaves = gridDim.x * kFinWaves;
    for (int base = (blockIdx.x * kFinWaves + wave) * 64; base < m; base += nwaves * 64) {
        const int slot = base + lane;
        int res = 0;
        if (slot < m) {
            const int tile = slot / TS, pos = slot % TS;
            float v[D + 1];
#pragma unroll
            for (int k = 0; k <= D; ++k) v[k] = 0.0f;
            const float* src = a.part + ((long long)tile * chunks * TS + pos) * (D + 1);
            for (int c = 0; c < chunks; ++c) {
                const float* p = src + (long long)c * TS * (D + 1);
#pragma unroll
                for (int k = 0; k <= D; ++k) v[k] += p[k];
            }
            res = update_seed<D, DP>(a, slot, v);
        }
        compact_wave<D, DP>(a, t, slot, res);
    }
}

}  // namespace
}  // namespace fms
