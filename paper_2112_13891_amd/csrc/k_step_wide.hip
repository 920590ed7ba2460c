// k_step_wide.hip -- the FP32 fused step for wide rows (padded D = 128, 256).
//
// Same update as the narrow step (Section II-B: every active seed moves to
// the kernel-weighted mean of all n points, eq. (12)-(15) for the flat
// window), for rows too wide for one lane to hold a seed and its D + 1 sums
// in registers.  The four waves of a workgroup hold the same 64 seeds (one
// per lane) but different quarters of the coordinates, Q = D / 4 each, and
// walk the same points in batches of P:
//   1. each wave computes, per point, the squared distance over its
//      coordinate quarter (wave-uniform scalar loads of that quarter);
//   2. the four partial distances meet in LDS and are added in wave order,
//      so every wave derives the same distance and weight for the pair;
//   3. each wave adds w (x - s) into its own coordinate quarter, and wave 0
//      adds w into the weight sum.
// A workgroup's sums are therefore complete for its (seed tile, point chunk)
// work item with no cross-wave reduction; they are stored as chunk partials
// and wide_finalize_kernel adds them in chunk order (also for one chunk per
// tile) and updates the seeds.
// No floating-point atomics, and every sum runs in a fixed order.

#include "step_common.h"

namespace fms {

namespace {

constexpr int kWideBatch = 32;   // points per batch

template <int D, int KERN>
__global__ __launch_bounds__(kThreads) void step_wide_kernel(StepArgs a, int t) {
    constexpr int TS = 64;
    constexpr int Q = D / kWaves;
    constexpr int P = kWideBatch;
    const int m = active_count(a.ctl, t);
    step_prologue(a, t, m);
    if (m == 0) return;
    const int n = a.n;
    const int G = gridDim.x;
    const int tiles = (m + TS - 1) / TS;
    const int chunks = chunks_for(m, TS, n, G, a.min_chunk);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q0 = wave * Q;
    __shared__ float qpart[kWaves][P][64];
    const const_f32_ptr xs = wave_uniform_const(a.Xp);

    for (int item = blockIdx.x; item < tiles * chunks; item += G) {
        const int tile = item % tiles;
        const int chunk = item / tiles;
        const int slot = tile * TS + lane;
        const int j = a.act_in[slot < m ? slot : tile * TS];
        float s[Q], acc[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            s[k] = a.S[(long long)j * D + q0 + k] * a.scale;
            acc[k] = 0.0f;
        }
        float accw = 0.0f;
        const int lo = __builtin_amdgcn_readfirstlane((int)((long long)n * chunk / chunks));
        const int hi = __builtin_amdgcn_readfirstlane((int)((long long)n * (chunk + 1) / chunks));
        for (int p0 = lo; p0 < hi; p0 += P) {
            const int cnt = __builtin_amdgcn_readfirstlane(min(P, hi - p0));
            // 1. partial squared distances over this wave's coordinates
#pragma unroll
            for (int p = 0; p < P; ++p) {
                float q = 0.0f;
                if (p < cnt) {
                    const const_f32_ptr row = xs + (long long)(p0 + p) * D + q0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        const float dk = row[k] - s[k];
                        q = fmaf(dk, dk, q);
                    }
                }
                qpart[wave][p][lane] = q;
            }
            __syncthreads();
            // 2. the whole distance, added in wave order, and the weight
            float w[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                float q = qpart[0][p][lane];
#pragma unroll
                for (int v = 1; v < kWaves; ++v) q += qpart[v][p][lane];
                float wp;
                if (KERN == MS_KERNEL_GAUSSIAN)
                    wp = __builtin_amdgcn_exp2f(-q);
                else
                    wp = (q <= a.h2) ? 1.0f : 0.0f;
                w[p] = p < cnt ? wp : 0.0f;
            }
            __syncthreads();   // qpart is rewritten by the next batch
            // 3. this wave's coordinates of sum w (x - s), and sum w
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (p < cnt) {
                    const const_f32_ptr row = xs + (long long)(p0 + p) * D + q0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) acc[k] = fmaf(w[p], row[k] - s[k], acc[k]);
                    accw += w[p];
                }
            }
        }
        float* dst = a.part + (((long long)tile * chunks + chunk) * TS + lane) * (D + 1);
#pragma unroll
        for (int k = 0; k < Q; ++k) dst[q0 + k] = acc[k];
        if (wave == 0) dst[D] = accw;
    }
}

// Sum over the 64 lanes by a fixed xor butterfly: every lane ends with the
// same value (each step adds two values that commute exactly).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Reduction and finalize of the wide step, one wave per active seed: lane l
// holds coordinates l, l + 64, ... of the seed's sums and adds them over the
// chunk partials in chunk order (lane 0 also the weight sum); then the
// update, the shift (fixed butterfly over the lanes) and the convergence test
// of Algorithms 1-2, as update_seed_id does for narrow rows.  A seed that
// stays active takes its slot of the next active list with one atomic (the
// results never depend on the order of that list).
template <int D>
__global__ __launch_bounds__(kThreads) void wide_finalize_kernel(StepArgs a, int t, int grid) {
    constexpr int TS = 64;
    constexpr int C = D / 64;
    const int m = active_count(a.ctl, t);
    if (m == 0) return;
    const int chunks = chunks_for(m, TS, a.n, grid, a.min_chunk);
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * kWaves;
    for (int slot = blockIdx.x * kWaves + (threadIdx.x >> 6); slot < m; slot += nw) {
        const int tile = slot / TS, pos = slot % TS;
        const float* src = a.part + ((long long)tile * chunks * TS + pos) * (D + 1);
        float v[C];
#pragma unroll
        for (int i = 0; i < C; ++i) v[i] = 0.0f;
        float W = 0.0f;
        for (int c = 0; c < chunks; ++c) {
            const float* p = src + (long long)c * TS * (D + 1);
#pragma unroll
            for (int i = 0; i < C; ++i) v[i] += p[lane + 64 * i];
            if (lane == 0) W += p[D];
        }
        W = __shfl(W, 0);
        const int j = a.act_in[slot];
        float* sj = a.S + (long long)j * D;
        int res = 0;
        if (!(W > 0.0f) || !isfinite(W)) {
            if (lane == 0) a.status[j] = ST_FAILED;
        } else {
            const float inv = a.inv_scale / W;
            float u[C];
            bool finite = true;
            float part2 = 0.0f;
            if (a.metric == MS_METRIC_COSINE) {
                float nn = 0.0f;
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    u[i] = sj[lane + 64 * i] + v[i] * inv;
                    nn = fmaf(u[i], u[i], nn);
                }
                nn = wave_sum(nn);
                const float rn = 1.0f / sqrtf(nn);
                finite = nn > 0.0f && isfinite(rn);
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    u[i] *= rn;
                    const float dk = u[i] - sj[lane + 64 * i];
                    finite = finite && isfinite(u[i]);
                    part2 = fmaf(dk, dk, part2);
                }
            } else {
#pragma unroll
                for (int i = 0; i < C; ++i) {
                    const float dk = v[i] * inv;
                    finite = finite && isfinite(dk);
                    part2 = fmaf(dk, dk, part2);
                    u[i] = sj[lane + 64 * i] + dk;
                }
            }
            const float sh2 = wave_sum(part2);
            finite = __ballot(!finite) == 0;
#pragma unroll
            for (int i = 0; i < C; ++i) sj[lane + 64 * i] = u[i];
            res = !finite ? 0 : (sh2 < a.thr2 ? 2 : 1);
            if (lane == 0) {
                a.iters[j] += 1;
                a.shift2[j] = sh2;
                if (!finite) a.status[j] = ST_FAILED;
                else if (res == 2) a.status[j] = ST_CONVERGED;
            }
        }
        if (lane == 0) {
            if (res == 1) a.act_out[atomicAdd(&a.ctl->count[(t + 1) % 3], 1)] = j;
            else if (res == 2) add_converged(a.ctl, t, 1);
        }
    }
}

template <int D>
hipError_t launch_wide_t(Batch& b, int t, hipStream_t s) {
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
        hipLaunchKernelGGL((step_wide_kernel<D, MS_KERNEL_GAUSSIAN>), dim3(b.grid), dim3(kThreads), 0, s, a, t);
    else
        hipLaunchKernelGGL((step_wide_kernel<D, MS_KERNEL_FLAT>), dim3(b.grid), dim3(kThreads), 0, s, a, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int fblocks = (b.n_seeds + kWaves - 1) / kWaves;
    if (fblocks > 4096) fblocks = 4096;
    hipLaunchKernelGGL((wide_finalize_kernel<D>), dim3(fblocks < 1 ? 1 : fblocks), dim3(kThreads), 0, s, a, t,
                       b.grid);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_iteration_wide(Batch& b, int t, hipStream_t s) {
    if (b.sh.R != 1 || b.sh.DP != b.sh.D) return hipErrorInvalidValue;
    if (b.sh.D == 128) return launch_wide_t<128>(b, t, s);
    if (b.sh.D == 256) return launch_wide_t<256>(b, t, s);
    return hipErrorInvalidValue;
}

}  // namespace fms
