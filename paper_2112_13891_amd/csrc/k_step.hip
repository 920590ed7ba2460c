// k_step.hip -- the fused mean-shift iteration (FP32 form) for gfx950: the
// pair work, the reduction, the update, the convergence test and the
// compaction of the active seeds, in one or two launches per iteration.
//
// One iteration updates every active seed s_j by the kernel-weighted mean of
// ALL n points (Section II-B; eq. (12)-(15) for the flat window):
//     s_j' = s_j + sum_i w_ij (x_i - s_j) / sum_i w_ij .
// The shift form is algebraically the plain m(s) = sum w x / sum w, but keeps
// the FP32 accumulation on small numbers.  No m x n weight matrix exists: a
// lane holds R seeds in registers, streams the points of its range through
// wave-uniform (scalar) loads and keeps the weights in registers.
//
// Work decomposition, from the device-side active count m only (so every
// seed's arithmetic depends on m alone and is bitwise reproducible, whatever
// order the active list has):
//   tiles  = ceil(m / TS), TS = 64 R seeds per tile;
//   chunks = point ranges per tile;
//   a workgroup (4 waves) takes one (tile, chunk); each wave a quarter of the
//   chunk; the wave sums are added in wave order into one chunk partial.
// Reduction without floating-point atomics or in-kernel cross-workgroup
// traffic (the L2s of the eight XCDs are not coherent with each other, so a
// device-scope fence inside a kernel costs an L2 write-back): when a tile has
// a single chunk, its workgroup finalizes it directly; otherwise each
// workgroup stores one (D+1)-vector partial per seed and a second kernel
// gives every seed one wave, whose lanes add the chunk partials in a fixed
// lane-strided order and then in a fixed shuffle tree.  Finalizing = the
// update, the convergence test (|shift|^2 < (tol h)^2, the "while not
// converge" of Algorithms 1-2) and the compaction of the seeds that stay
// active (wave64 ballot, one atomic per wave, or one per seed in the
// per-seed kernel).  The batch early-stop rule of Section II-C is applied at
// the start of each launch from per-iteration converged counters.
//
// Gaussian weights use packed coordinates pre-scaled by
// c = sqrt(log2(e) / (2 h^2)), so w = exp2(-|c x - c s|^2) is one v_exp_f32.

#include "step_common.h"

namespace fms {

namespace {

__global__ void pack_points_kernel(const float* __restrict__ X, int n, int d, int DP,
                                   float scale, float* __restrict__ Xp) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)n * DP;
    if (e >= total) return;
    int i = (int)(e / DP), k = (int)(e % DP);
    Xp[e] = (k < d) ? X[(long long)i * d + k] * scale : 0.0f;
}

// Cosine metric: each row divided by its length (FP32); a row without a
// finite nonzero length raises *bad.
__global__ void normalize_rows_kernel(const float* __restrict__ X, int n, int d, float* __restrict__ Xn,
                                      int32_t* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* x = X + (long long)i * d;
    float nn = 0.0f;
    for (int k = 0; k < d; ++k) nn = fmaf(x[k], x[k], nn);
    const float r = 1.0f / sqrtf(nn);
    if (!(nn > 0.0f) || !isfinite(r)) {
        if (bad) *bad = 1;
    }
    float* o = Xn + (long long)i * d;
    for (int k = 0; k < d; ++k) o[k] = x[k] * r;
}

__device__ void ctl_reset_body(Ctl* ctl, int B, int need, int max_iter) {
    for (int u = threadIdx.x; u <= max_iter; u += blockDim.x) ctl->conv_it[u] = 0;
    if (threadIdx.x < kMaxMergePasses) ctl->und[threadIdx.x] = 0;
    if (threadIdx.x < kRefinedSlots) ctl->refined[threadIdx.x * kRefinedStride] = 0;
    if (threadIdx.x == 0) {
        ctl->count[0] = B;
        ctl->count[1] = 0;
        ctl->count[2] = 0;
        ctl->conv_base[0] = 0;
        ctl->need = need;
        ctl->iters_run = 0;
        ctl->pool_len = 0;
        ctl->pairs = 0;
    }
}

__global__ void ctl_reset_kernel(Ctl* ctl, int B, int need, int max_iter) {
    ctl_reset_body(ctl, B, need, max_iter);
}

// Start of a fit round in one launch: the B drawn seeds (pool[pos[j]], or
// j itself when pos is NULL) leave the pool (removed flag), their positions
// become the batch's seeds, every seed starts active and undecided for the
// merge, and workgroup 0 resets the control block.
__global__ void round_init_kernel(const float* __restrict__ X, int d, int DP,
                                  const int32_t* __restrict__ pool, const int32_t* __restrict__ pos,
                                  int B, int32_t* ids, uint8_t* removed, int32_t* merge_state,
                                  float* S, int32_t* act0, uint8_t* status, int32_t* iters,
                                  float* shift2, Ctl* ctl, int need, int max_iter) {
    if (blockIdx.x == 0) ctl_reset_body(ctl, B, need, max_iter);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= B) return;
    int id = j;
    if (pos) {
        const int p = pos[j];
        id = pool[p];
        removed[p] = 1;
    }
    ids[j] = id;
    merge_state[j] = MG_UNDECIDED;
    const long long src = (long long)id * d;
    for (int k = 0; k < DP; ++k) S[(long long)j * DP + k] = (k < d) ? X[src + k] : 0.0f;
    act0[j] = j;
    status[j] = ST_ACTIVE;
    iters[j] = 0;
    shift2[j] = __builtin_nanf("");
}

__global__ void seed_init_array_kernel(const float* __restrict__ seeds,
                                       const uint8_t* __restrict__ conv_in, int d, int DP,
                                       int m, int unit, float* S, int32_t* act0, uint8_t* status,
                                       int32_t* iters, float* shift2, Ctl* ctl) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    bool live = false;
    if (j < m) {
        float r = 1.0f;   // cosine metric: seeds start as unit vectors
        if (unit) {
            float nn = 0.0f;
            for (int k = 0; k < d; ++k) nn = fmaf(seeds[(long long)j * d + k], seeds[(long long)j * d + k], nn);
            r = 1.0f / sqrtf(nn);
        }
        for (int k = 0; k < DP; ++k)
            S[(long long)j * DP + k] = (k < d) ? seeds[(long long)j * d + k] * r : 0.0f;
        uint8_t st = conv_in[j];
        status[j] = st;
        iters[j] = 0;
        shift2[j] = __builtin_nanf("");
        live = (st == ST_ACTIVE);
    }
    // wave64 ballot compaction of the seeds that start active
    unsigned long long mask = __ballot(live);
    int lane = threadIdx.x & 63;
    int rank = __popcll(mask & ((1ull << lane) - 1ull));
    int base = 0;
    if (lane == 0 && mask) base = atomicAdd(&ctl->count[0], __popcll(mask));
    base = __shfl(base, 0);
    if (live) act0[base + rank] = j;
}

// One iteration over the active seeds: pair work and chunk partials.
template <int D, int DP, int R, int KERN>
__global__ __launch_bounds__(kThreads) void step_kernel(StepArgs a, int t) {
    constexpr int TS = 64 * R;
    Ctl* ctl = a.ctl;
    const int n = a.n;
    const int m = active_count(ctl, t);
    step_prologue(a, t, m);
    if (m == 0) return;
    const int G = gridDim.x;
    const int tiles = (m + TS - 1) / TS;
    const int chunks = chunks_for(m, TS, n, G, a.min_chunk);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __shared__ float red[(kWaves - 1) * TS * (D + 1)];   // wave partials; then the tile sums

    for (int item = blockIdx.x; item < tiles * chunks; item += G) {
        const int tile = item % tiles;
        const int chunk = item / tiles;
        float acc[R][D + 1];
        tile_sums<D, DP, R, KERN>(a, a.Xp, (long long)n * chunk / chunks,
                                  (long long)n * (chunk + 1) / chunks, a.act_in, tile * TS, m, acc, red);

        if (chunks == 1) {
            // the chunk partial is the tile sum: finalize here
            if (wave == 0) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int k = 0; k <= D; ++k) red[k * TS + r * 64 + lane] = acc[r][k];
            }
            __syncthreads();
            finalize_tile<D, DP, R>(a, t, m, tile, red);
            __syncthreads();
        } else if (wave == 0) {
            // one (D+1)-vector per seed: part[(tile*chunks + chunk)*TS + pos][k]
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float* dst = a.part + (((long long)tile * chunks + chunk) * TS + r * 64 + lane) * (D + 1);
#pragma unroll
                for (int k = 0; k <= D; ++k) dst[k] = acc[r][k];
            }
        }
    }
}

__global__ void seed_export_kernel(const float* __restrict__ S, int DP, int d, int m,
                                   const uint8_t* __restrict__ status,
                                   const int32_t* __restrict__ it,
                                   const float* __restrict__ sh, float* seeds,
                                   uint8_t* conv, int32_t* iters, float* shift2) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    for (int k = 0; k < d; ++k) seeds[(long long)j * d + k] = S[(long long)j * DP + k];
    conv[j] = status[j];
    iters[j] = it[j];
    if (it[j] > 0) shift2[j] = sh[j];
}

template <int D, int DP, int R>
hipError_t launch_step_t(Batch& b, int t, hipStream_t s) {
    StepArgs a;
    a.Xp = b.Xp;
    a.n = b.n;
    a.d = b.d;
    a.min_chunk = b.sh.MC;
    a.S = b.S;
    a.act_in = b.act[t & 1];
    a.act_out = b.act[(t + 1) & 1];
    a.status = b.status;
    a.iters = b.iters;
    a.shift2 = b.shift2;
    a.part = b.part;
    a.red = b.part + step_red_offset(b.sh, b.n_seeds, b.grid);
    a.prog = b.prog;
    a.ctl = b.ctl;
    a.h2 = b.h * b.h;
    a.scale = b.scale;
    a.inv_scale = b.inv_scale;
    a.thr2 = b.thr2;
    a.metric = b.metric;
    if (b.kernel == MS_KERNEL_GAUSSIAN)
        hipLaunchKernelGGL((step_kernel<D, DP, R, MS_KERNEL_GAUSSIAN>), dim3(b.grid),
                           dim3(kThreads), 0, s, a, t);
    else
        hipLaunchKernelGGL((step_kernel<D, DP, R, MS_KERNEL_FLAT>), dim3(b.grid), dim3(kThreads),
                           0, s, a, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize<D, DP, R>(a, t, b.grid, b.n_seeds, s);
}

}  // namespace

// Points per point chunk, at least: smaller chunks spread a small batch of
// seeds over more workgroups (measured best at 256 for both forms).
constexpr int kStepMinChunk = 256;

StepShape step_shape(int d) {
    StepShape sh;
    if (d <= 4) sh.D = d;
    else if (d <= 8) sh.D = 8;
    else if (d <= 16) sh.D = 16;
    else if (d <= 32) sh.D = 32;
    else if (d <= 64) sh.D = 64;
    else if (d <= 128) sh.D = 128;
    else sh.D = 256;
    sh.DP = sh.D < 4 ? 4 : sh.D;
    sh.R = sh.D <= 4 ? 4 : (sh.D <= 8 ? 2 : 1);
    sh.TS = 64 * sh.R;
    sh.MC = kStepMinChunk;
    return sh;
}

StepShape step_shape_for(int d, int B) {
    StepShape sh = step_shape(d);
    // small batches: fewer seeds per lane keeps lanes busy
    while (sh.R > 1 && 64 * sh.R > B) sh.R /= 2;
    sh.TS = 64 * sh.R;
    return sh;
}

int step_grid(const StepShape& sh, int B, int n) {
    long long tiles = (B + sh.TS - 1) / sh.TS;
    long long chunks = (n + sh.MC - 1) / sh.MC;
    long long g = tiles * chunks;
    if (g > kMaxGrid) g = kMaxGrid;
    return (int)(g < 1 ? 1 : g);
}

long long step_red_offset(const StepShape& sh, int B, int grid) {
    // items = tiles * chunks <= max(tiles, grid) with chunks > 1 only when tiles < grid
    const long long tiles = (B + sh.TS - 1) / sh.TS;
    const long long items = tiles < grid ? grid : tiles;
    return items * sh.TS * (long long)(sh.D + 1);
}

long long step_part_floats(const StepShape& sh, int B, int grid) {
    // chunk partials, then one reduced (D+1)-vector per slot
    const long long tiles = (B + sh.TS - 1) / sh.TS;
    return step_red_offset(sh, B, grid) + tiles * sh.TS * (long long)(sh.D + 1);
}

hipError_t launch_normalize_rows(const float* X, int n, int d, float* Xn, int32_t* bad, hipStream_t s) {
    hipLaunchKernelGGL(normalize_rows_kernel, dim3((n + 255) / 256), dim3(256), 0, s, X, n, d, Xn, bad);
    return hipGetLastError();
}

hipError_t launch_pack_points(const float* X, int n, int d, int DP, float scale, float* Xp,
                              hipStream_t s) {
    long long total = (long long)n * DP;
    int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(pack_points_kernel, dim3(blocks), dim3(256), 0, s, X, n, d, DP, scale,
                       Xp);
    return hipGetLastError();
}

hipError_t launch_ctl_reset(Ctl* ctl, int B, int need, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(256), 0, s, ctl, B, need, max_iter);
    return hipGetLastError();
}

hipError_t launch_round_init(const float* X, int d, int DP, const int32_t* pool,
                             const int32_t* pos, int B, int32_t* ids, uint8_t* removed,
                             int32_t* merge_state, Batch& b, int need, int max_iter, hipStream_t s) {
    const int blocks = B > 0 ? (B + 255) / 256 : 1;
    hipLaunchKernelGGL(round_init_kernel, dim3(blocks), dim3(256), 0, s, X, d, DP, pool, pos, B,
                       ids, removed, merge_state, b.S, b.act[0], b.status, b.iters, b.shift2,
                       b.ctl, need, max_iter);
    return hipGetLastError();
}

hipError_t launch_seed_init_from_array(const float* seeds, const uint8_t* conv_in, int d,
                                       int m, Batch& b, hipStream_t s) {
    hipLaunchKernelGGL(seed_init_array_kernel, dim3((m + 255) / 256), dim3(256), 0, s, seeds,
                       conv_in, d, b.sh.DP, m, b.metric == MS_METRIC_COSINE ? 1 : 0, b.S, b.act[0],
                       b.status, b.iters, b.shift2, b.ctl);
    return hipGetLastError();
}

hipError_t launch_seed_export(const Batch& b, int m, float* seeds, uint8_t* conv,
                              int32_t* iters, float* shift2, hipStream_t s) {
    hipLaunchKernelGGL(seed_export_kernel, dim3((m + 255) / 256), dim3(256), 0, s, b.S,
                       b.sh.DP, b.d, m, b.status, b.iters, b.shift2, seeds, conv, iters,
                       shift2);
    return hipGetLastError();
}

// One iteration: the fused step (and the partial reduction when needed).
hipError_t launch_iteration(Batch& b, int t, hipStream_t s) {
    if (b.prec == MS_PREC_BF16_REFINE) return launch_iteration_bf16(b, t, s);
    if (b.Xs && b.geom) return launch_iteration_cull(b, t, s);
    if (b.sh.D > 64) return launch_iteration_wide(b, t, s);
    const int D = b.sh.D, R = b.sh.R;
#define FMS_CASE(DD, DPP, RR) \
    if (D == DD && R == RR) return launch_step_t<DD, DPP, RR>(b, t, s);
    FMS_CASE(1, 4, 1) FMS_CASE(1, 4, 2) FMS_CASE(1, 4, 4)
    FMS_CASE(2, 4, 1) FMS_CASE(2, 4, 2) FMS_CASE(2, 4, 4)
    FMS_CASE(3, 4, 1) FMS_CASE(3, 4, 2) FMS_CASE(3, 4, 4)
    FMS_CASE(4, 4, 1) FMS_CASE(4, 4, 2) FMS_CASE(4, 4, 4)
    FMS_CASE(8, 8, 1) FMS_CASE(8, 8, 2)
    FMS_CASE(16, 16, 1)
    FMS_CASE(32, 32, 1)
    FMS_CASE(64, 64, 1)
#undef FMS_CASE
    return hipErrorInvalidValue;
}

}  // namespace fms
