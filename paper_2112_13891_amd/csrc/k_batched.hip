// k_batched.hip -- the fused mean-shift iteration (FP32 form) for many
// independent point clouds of uneven size in one launch per kernel.
//
// Cloud c owns the points Xp[x_off[c], x_off[c+1]) and the seeds
// [seg[c], seg[c+1]) of the batch; each seed is updated with the points of
// its own cloud only, exactly as a call per cloud would (Section II-B update,
// per-seed convergence of Algorithms 1-2).
//
// One iteration is three launches:
//   plan     one workgroup: from the per-cloud active counts, each cloud's
//            seed tiles (64R seeds) and point chunks (chunk_points points,
//            1024 unless the call or the tuner sets another),
//            the prefix of work items and of active slots, and for every
//            work item and active slot its cloud (one wave per cloud fills
//            the cloud's ranges);
//   step     a persistent grid over the work items (cloud, seed tile, point
//            chunk): with more items than workgroups every item comes from
//            a queue (one atomic per item, so that uneven items and
//            late-starting workgroups balance), else each its own; the
//            same pair loop as the single-cloud step, one (D+1)-vector
//            partial per seed and item, stored component-major within the
//            item (component k of the item's TS seeds contiguous) so that
//            the stores and the finalize's loads are coalesced;
//   finalize one lane per active seed: its chunk partials added in chunk
//            order, the update and convergence test, and the seed kept in
//            its cloud's next active list (per-cloud counter).
// The chunking depends only on the counts, never on the order of an active
// list, so results are deterministic; no floating-point atomics.

#include "step_common.h"

namespace fms {

namespace {

constexpr int kPlanThreads = 1024;

// Appends seed j to the active list of its cloud c (slots seg[c] + cnt[c]++)
// for every lane with keep set: the wave's seeds one cloud at a time, one
// atomic per cloud and wave, slots in lane order.  Every active lane of the
// wave must call it.
__device__ __forceinline__ void append_by_cloud(bool keep, int c, int j, int32_t* cnt, const int32_t* seg,
                                                int32_t* act) {
    unsigned long long pend = __ballot(keep);
    while (pend) {
        const int leader = __builtin_ctzll(pend);
        const int lc = __shfl(c, leader);
        const bool mine = keep && c == lc;
        const unsigned long long mask = __ballot(mine);
        int base = 0;
        if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(&cnt[lc], __popcll(mask));
        base = __shfl(base, leader);
        if (mine) {
            const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
            act[seg[c] + base + below] = j;
        }
        pend &= ~mask;
    }
}

// Inclusive block scan of one value per thread (kPlanThreads threads).
__device__ __forceinline__ int plan_scan(int v, int* wsum, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < kPlanThreads / 64; ++w) {
        if (w < wave) before += wsum[w];
        tot += wsum[w];
    }
    *total = tot;
    __syncthreads();
    return v + before;
}

constexpr int kMaxClouds = 8192;

__global__ __launch_bounds__(kPlanThreads) void bplan_kernel(BatchedArgs B, int t, int TS) {
    __shared__ int ipre[kMaxClouds + 1];
    __shared__ int spre[kMaxClouds + 1];
    __shared__ int wsum[kPlanThreads / 64];
    const int* cin = B.cnt + (t & 1) * B.ncl;
    int* cout = B.cnt + ((t + 1) & 1) * B.ncl;
    int icarry = 0, scarry = 0;
    for (int c0 = 0; c0 < B.ncl; c0 += kPlanThreads) {
        const int c = c0 + threadIdx.x;
        int items = 0, m = 0;
        if (c < B.ncl) {
            m = cin[c];
            const long long n = B.x_off[c + 1] - B.x_off[c];
            const int tl = (m + TS - 1) / TS;
            const int ch = m > 0 ? (int)((n + B.chunk_points - 1) / B.chunk_points) : 0;
            B.tiles[c] = tl;
            B.chunks[c] = ch;
            items = tl * ch;
            cout[c] = 0;   // filled by this iteration's finalize
        }
        int itot, stot;
        const int iinc = plan_scan(items, wsum, &itot);
        const int sinc = plan_scan(m, wsum, &stot);
        if (c < B.ncl) {
            ipre[c] = icarry + iinc - items;
            spre[c] = scarry + sinc - m;
        }
        icarry += itot;
        scarry += stot;
    }
    if (threadIdx.x == 0) {
        ipre[B.ncl] = icarry;
        spre[B.ncl] = scarry;
        *B.queue = 0;
    }
    __syncthreads();
    for (int c = threadIdx.x; c <= B.ncl; c += kPlanThreads) {
        B.item_pre[c] = ipre[c];
        B.slot_pre[c] = spre[c];
    }
    // a cloud's work items and active slots are contiguous ranges: one wave
    // per cloud writes them, 64 entries per store
    const int lane = threadIdx.x & 63;
    for (int c = threadIdx.x >> 6; c < B.ncl; c += kPlanThreads / 64) {
        for (int i = ipre[c] + lane; i < ipre[c + 1]; i += 64) B.item_cloud[i] = c;
        for (int g = spre[c] + lane; g < spre[c + 1]; g += 64) B.slot_cloud[g] = c;
    }
}

template <int D, int DP, int R, int KERN>
__global__ __launch_bounds__(kThreads) void bstep_kernel(StepArgs a, BatchedArgs B) {
    constexpr int TS = 64 * R;
    const int total = B.item_pre[B.ncl];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __shared__ float red[(kWaves - 1) * TS * (D + 1)];
    __shared__ int next_item;
    // with no more items than workgroups each takes its own; otherwise every
    // item comes from the queue (every thread has read the previous item --
    // the pair loop holds barriers -- before thread 0 writes the next one)
    const bool own = total <= (int)gridDim.x;
    int it = blockIdx.x;
    if (!own) {
        if (threadIdx.x == 0) next_item = atomicAdd(B.queue, 1);
        __syncthreads();
        it = next_item;
    }
    while (it < total) {
        const int c = B.item_cloud[it];
        const int local = it - B.item_pre[c];
        const int tiles = B.tiles[c], chunks = B.chunks[c];
        const int tile = local % tiles, chunk = local / tiles;
        const long long x0 = B.x_off[c];
        const long long n = B.x_off[c + 1] - x0;
        const int m = B.slot_pre[c + 1] - B.slot_pre[c];
        float acc[R][D + 1];
        tile_sums<D, DP, R, KERN>(a, a.Xp + x0 * DP, n * chunk / chunks, n * (chunk + 1) / chunks,
                                  a.act_in + B.seg[c], tile * TS, m, acc, red);
        if (wave == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float* dst = a.part + (long long)it * TS * (D + 1) + r * 64 + lane;
#pragma unroll
                for (int k = 0; k <= D; ++k) dst[k * TS] = acc[r][k];
            }
        }
        if (own) break;
        if (threadIdx.x == 0) next_item = atomicAdd(B.queue, 1);
        __syncthreads();
        it = next_item;
    }
}

template <int D, int DP, int R>
__global__ __launch_bounds__(kFinThreads) void bfinal_kernel(StepArgs a, BatchedArgs B, int t) {
    constexpr int TS = 64 * R;
    const int total = B.slot_pre[B.ncl];
    int* cout = B.cnt + ((t + 1) & 1) * B.ncl;
    for (int g = blockIdx.x * kFinThreads + threadIdx.x; g < total; g += gridDim.x * kFinThreads) {
        const int c = B.slot_cloud[g];
        const int q = g - B.slot_pre[c];
        const int tile = q / TS, pos = q % TS;
        const int tiles = B.tiles[c], chunks = B.chunks[c];
        const int ib = B.item_pre[c];
        float v[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) v[k] = 0.0f;
        // chunk order; the loads of four chunks in flight together
        constexpr int U = D <= 16 ? 4 : 1;
        int ch = 0;
        for (; ch + U <= chunks; ch += U) {
            float tmp[U][D + 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float* p = a.part + (long long)(ib + (ch + u) * tiles + tile) * TS * (D + 1) + pos;
#pragma unroll
                for (int k = 0; k <= D; ++k) tmp[u][k] = p[k * TS];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k <= D; ++k) v[k] += tmp[u][k];
        }
        for (; ch < chunks; ++ch) {
            const float* p = a.part + (long long)(ib + ch * tiles + tile) * TS * (D + 1) + pos;
#pragma unroll
            for (int k = 0; k <= D; ++k) v[k] += p[k * TS];
        }
        const int j = a.act_in[B.seg[c] + q];
        const bool keep = update_seed_id<D, DP>(a, j, v) == 1;
        append_by_cloud(keep, c, j, cout, B.seg, a.act_out);
    }
}

// Seeds of the batch: copy (d -> DP columns), status from the caller's flags,
// and every active seed into its cloud's first active list.
__global__ void bseed_init_kernel(const float* __restrict__ seeds, const uint8_t* __restrict__ conv_in,
                                  int d, int DP, int M, const int32_t* __restrict__ seg, int ncl,
                                  float* S, int32_t* act0, uint8_t* status, int32_t* iters, float* shift2,
                                  int32_t* cnt0) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    bool active = false;
    int c = 0;
    if (j < M) {
        for (int k = 0; k < DP; ++k) S[(long long)j * DP + k] = (k < d) ? seeds[(long long)j * d + k] : 0.0f;
        const uint8_t st = conv_in[j];
        status[j] = st;
        iters[j] = 0;
        shift2[j] = __builtin_nanf("");
        active = st == ST_ACTIVE;
        if (active) c = upper_cloud(seg, ncl, j);
    }
    append_by_cloud(active, c, j, cnt0, seg, act0);
}

__global__ void bzero_kernel(int32_t* a, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) a[i] = 0;
}

StepArgs batched_step_args(const Batch& b, const BatchedArgs& B, int t) {
    StepArgs a = {};
    a.Xp = b.Xp;
    a.n = b.n;
    a.d = b.d;
    a.min_chunk = B.chunk_points;
    a.S = b.S;
    a.act_in = b.act[t & 1];
    a.act_out = b.act[(t + 1) & 1];
    a.status = b.status;
    a.iters = b.iters;
    a.shift2 = b.shift2;
    a.part = b.part;
    a.ctl = b.ctl;
    a.h2 = b.h * b.h;
    a.scale = b.scale;
    a.inv_scale = b.inv_scale;
    a.thr2 = b.thr2;
    a.metric = b.metric;
    return a;
}

int batched_finalize_blocks(const Batch& b) {
    const int fblocks = (b.n_seeds + kFinThreads - 1) / kFinThreads;
    return fblocks < 1 ? 1 : (fblocks > 1024 ? 1024 : fblocks);
}

template <int D, int DP, int R>
hipError_t bstep_t(const Batch& b, const BatchedArgs& B, int t, hipStream_t s) {
    const StepArgs a = batched_step_args(b, B, t);
    hipLaunchKernelGGL(bplan_kernel, dim3(1), dim3(kPlanThreads), 0, s, B, t, 64 * R);
    // no more workgroups than the first iteration has work items (seeds only
    // ever leave the active lists)
    const int grid = std::max(1, std::min(B.grid_cap, b.grid));
    if (b.kernel == MS_KERNEL_GAUSSIAN)
        hipLaunchKernelGGL((bstep_kernel<D, DP, R, MS_KERNEL_GAUSSIAN>), dim3(grid), dim3(kThreads),
                           0, s, a, B);
    else
        hipLaunchKernelGGL((bstep_kernel<D, DP, R, MS_KERNEL_FLAT>), dim3(grid), dim3(kThreads), 0,
                           s, a, B);
    hipLaunchKernelGGL((bfinal_kernel<D, DP, R>), dim3(batched_finalize_blocks(b)), dim3(kFinThreads), 0, s, a, B,
                       t);
    return hipGetLastError();
}

// The BF16 form (Gaussian, D in {8, 16, 32}): the same plan over seed tiles
// of 128 and chunks of whole 256-point blocks of each cloud's sorted points,
// the compensated step per work item, the same finalize (two seeds' slots per
// lane: tiles of 128).
template <int D>
hipError_t bstep_bf16_t(const Batch& b, const BatchedArgs& B, int t, hipStream_t s) {
    static_assert(kBf16fTile == 128, "the finalize's tile");
    const StepArgs a = batched_step_args(b, B, t);
    hipLaunchKernelGGL(bplan_kernel, dim3(1), dim3(kPlanThreads), 0, s, B, t, kBf16fTile);
    const int grid = std::max(1, std::min(B.grid_cap, b.grid));
    hipError_t e = launch_bstep_bf16f(b, B, t, grid, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bfinal_kernel<D, D, 2>), dim3(batched_finalize_blocks(b)), dim3(kFinThreads), 0, s, a, B,
                       t);
    return hipGetLastError();
}

}  // namespace

int batched_max_clouds() { return kMaxClouds; }

// Work items of the first iteration (every seed active): the size of the
// partials and of the item map.
long long batched_max_items(const long long* x_off, const int32_t* seg, int ncl, int TS, int chunk_points) {
    long long items = 0;
    for (int c = 0; c < ncl; ++c) {
        const long long m = seg[c + 1] - seg[c];
        const long long n = x_off[c + 1] - x_off[c];
        if (m > 0) items += ((m + TS - 1) / TS) * ((n + chunk_points - 1) / chunk_points);
    }
    return items;
}

hipError_t launch_batched_init(const float* seeds, const uint8_t* conv_in, int d, int M,
                               const int32_t* seg_dev, int ncl, int32_t* cnt, Batch& b, hipStream_t s) {
    hipLaunchKernelGGL(bzero_kernel, dim3((2 * ncl + 255) / 256), dim3(256), 0, s, cnt, 2 * ncl);
    if (M > 0)
        hipLaunchKernelGGL(bseed_init_kernel, dim3((M + 255) / 256), dim3(256), 0, s, seeds, conv_in, d,
                           b.sh.DP, M, seg_dev, ncl, b.S, b.act[0], b.status, b.iters, b.shift2, cnt);
    return hipGetLastError();
}

hipError_t launch_batched_iteration(const Batch& b, const long long* x_off_dev, const int32_t* seg_dev,
                                    int ncl, int32_t* cnt, int32_t* plan, int32_t* item_cloud,
                                    int32_t* slot_cloud, int t, hipStream_t s) {
    BatchedArgs B;
    B.ncl = ncl;
    B.x_off = x_off_dev;
    B.seg = seg_dev;
    B.cnt = cnt;
    B.tiles = plan;
    B.chunks = plan + ncl;
    B.item_pre = plan + 2 * ncl;
    B.slot_pre = plan + 3 * ncl + 1;
    B.item_cloud = item_cloud;
    B.slot_cloud = slot_cloud;
    B.queue = plan + 4 * ncl + 2;
    B.chunk_points = b.chunk_points;
    B.grid_cap = b.grid_cap;
    B.boff = b.boff;
    const int D = b.sh.D, R = b.sh.R;
    if (b.prec == MS_PREC_BF16_REFINE) {
        if (!b.boff || b.chunk_points % 256 != 0) return hipErrorInvalidValue;
        switch (D) {
            case 8: return bstep_bf16_t<8>(b, B, t, s);
            case 16: return bstep_bf16_t<16>(b, B, t, s);
            case 32: return bstep_bf16_t<32>(b, B, t, s);
            default: return hipErrorInvalidValue;
        }
    }
#define FMS_BCASE(DD, DPP, RR) \
    if (D == DD && R == RR) return bstep_t<DD, DPP, RR>(b, B, t, s);
    FMS_BCASE(1, 4, 1) FMS_BCASE(1, 4, 2) FMS_BCASE(1, 4, 4)
    FMS_BCASE(2, 4, 1) FMS_BCASE(2, 4, 2) FMS_BCASE(2, 4, 4)
    FMS_BCASE(3, 4, 1) FMS_BCASE(3, 4, 2) FMS_BCASE(3, 4, 4)
    FMS_BCASE(4, 4, 1) FMS_BCASE(4, 4, 2) FMS_BCASE(4, 4, 4)
    FMS_BCASE(8, 8, 1) FMS_BCASE(8, 8, 2)
    FMS_BCASE(16, 16, 1) FMS_BCASE(16, 16, 2) FMS_BCASE(32, 32, 1) FMS_BCASE(64, 64, 1)
#undef FMS_BCASE
    return hipErrorInvalidValue;
}

}  // namespace fms
