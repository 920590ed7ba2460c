// k_step_cull.hip -- FP32 fused step over spatially ordered points (d <= 4:
// Morton order; D = 8, 16, 32: nearest-pivot order), skipping the point
// blocks whose weights are exactly zero for a whole wave.
//
// The update is the one of Section II-B (every seed against ALL n points,
// s' = s + sum w (x - s) / sum w).  The points are spatially ordered (Morton
// order for d <= 4; for D = 8, 16, 32 by nearest pivot, shifted by the frame
// midpoint, the seeds shifted alike) and cut into 256-point blocks, each
// with a centre c_b and a radius r_b (rounded up); the active seeds are in the
// same order, so the 64 R seeds of a wave are close to each other.  For a
// seed s, every point of block b lies at distance at least |s - c_b| - r_b.
// If that bound puts every pair of the block past
// the point where the weight is exactly zero in FP32 -- Gaussian:
// |c s - c x|^2 >= kCullGauss in exp2 units, so exp2(-q) underflows to +0;
// flat window: |s - x|^2 > h^2 with a relative margin far above the FP32
// rounding of the bound -- for all seeds of the wave, the wave skips the
// block.  The skipped pairs would add +0 to every sum, so the result is the
// one of evaluating all pairs, and it does not depend on which seeds share
// a wave.
//
// Work decomposition (from the active count m only, as in the plain step):
// tiles of TS = 64 R seeds, chunks of at least 2 whole blocks; a workgroup
// of 4 waves takes one (tile, chunk).  All four waves hold the tile's seeds,
// so they agree on which blocks are live; each live block is staged in LDS
// with one coalesced vector load per thread (the next live block's load is in
// flight while the current one computes), wave w takes its points
// [64 w, 64 w + 64) as broadcast reads (wide rows: straight from memory
// through scalar loads), and the four wave sums are added in wave order.
// Chunk partials are reduced as in the plain step.

#include <cmath>

#include "step_common.h"

namespace fms {

namespace {

constexpr int kCullBlk = 256;            // points per block of the geometry
constexpr float kCullGauss = 160.0f;     // exp2(-q) == +0 in FP32 for q >= 150
constexpr float kCullFlatMargin = 1.001f;
constexpr int kCullMinPoints = 16384;     // below this the sort costs more than it saves

// One point against the lane's R seeds: Gaussian exp2(-q) in packed units or
// the flat window, accumulated into sum w (x - s) and sum w.
template <int D, int R, int KERN>
__device__ __forceinline__ void pair_acc(const float* x, const float (&s)[R][D], float (&acc)[R][D + 1],
                                         float h2) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float dx[D];
        float q = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dx[k] = x[k] - s[r][k];
            q = fmaf(dx[k], dx[k], q);
        }
        float w;
        if (KERN == MS_KERNEL_GAUSSIAN)
            w = __builtin_amdgcn_exp2f(-q);
        else
            w = (q <= h2) ? 1.0f : 0.0f;
        acc[r][D] += w;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[r][k] = fmaf(w, dx[k], acc[r][k]);
    }
}

// Geometry row of a block: centre[0..D), radius at [4] (D <= 4, stride 8) or
// at [D] (stride D + 8).
template <int D>
struct CullGeom {
    static constexpr int kStride = D <= 4 ? kGeomStride : D + 8;
    static constexpr int kRadius = D <= 4 ? 4 : D;
};

// Next block at or after blk (below b1) that some seed of the wave may see
// with a nonzero weight; b1 if none.
template <int D, int R>
__device__ __forceinline__ int next_live_block(const_f32_ptr geom, int blk, int b1,
                                               const float (&s)[R][D], const bool (&live)[R],
                                               float qcull) {
    for (; blk < b1; ++blk) {
        // wave-uniform block geometry (scalar loads)
        const const_f32_ptr gm = geom + (long long)blk * CullGeom<D>::kStride;
        bool near = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float d2 = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const float u = s[r][k] - gm[k];
                d2 = fmaf(u, u, d2);
            }
            const float lb = sqrtf(d2) - gm[CullGeom<D>::kRadius];
            near = near || (live[r] && !(lb > 0.0f && lb * lb > qcull));
        }
        if (__ballot(near)) break;
    }
    return blk;
}

template <int D, int R, int KERN>
__global__ __launch_bounds__(kThreads) void step_cull_kernel(StepArgs a, const float* __restrict__ geom,
                                                             const float* __restrict__ shift, float qcull,
                                                             int t) {
    constexpr int TS = 64 * R;
    constexpr int DP = D <= 4 ? 4 : D;
    constexpr bool kStage = D <= 4;           // small rows: stage blocks in LDS
    constexpr int PWD = kCullBlk / kWaves;    // points of a block per wave
    Ctl* ctl = a.ctl;
    const int n = a.n;
    const int m = active_count(ctl, t);
    step_prologue(a, t, m);
    if (m == 0) return;
    const int G = gridDim.x;
    const int tiles = (m + TS - 1) / TS;
    const int chunks = chunks_for(m, TS, n, G, a.min_chunk);
    const int nblk = (n + kCullBlk - 1) / kCullBlk;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int V = TS * (D + 1);
    __shared__ float red[(kWaves - 1) * V];
    __shared__ float4 xs[kStage ? kCullBlk : 1];   // the staged block, one point per thread
    const float4* __restrict__ X4 = reinterpret_cast<const float4*>(a.Xp);
    const const_f32_ptr xq = wave_uniform_const(a.Xp);   // wide rows: scalar loads

    const const_f32_ptr gq = wave_uniform_const(geom);
    for (int item = blockIdx.x; item < tiles * chunks; item += G) {
        const int tile = item % tiles;
        const int chunk = item / tiles;
        // uniform over the workgroup (the compiler cannot see it: chunks
        // derives from the active count)
        const int b0 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * chunk / chunks));
        const int b1 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * (chunk + 1) / chunks));
        // every wave holds the same TS seeds, so every wave takes the same
        // culling decisions and the block loop below is uniform over the
        // workgroup
        float s[R][D], acc[R][D + 1];
        bool live[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int slot = tile * TS + r * 64 + lane;
            live[r] = slot < m;
            const int j = a.act_in[live[r] ? slot : tile * TS];
            // the sorted points of the wide form are shifted by the frame
            // midpoint; the seeds take the same shift
#pragma unroll
            for (int k = 0; k < D; ++k)
                s[r][k] = a.S[(long long)j * DP + k] * a.scale - (shift ? shift[k] : 0.0f);
#pragma unroll
            for (int k = 0; k <= D; ++k) acc[r][k] = 0.0f;
        }
        int blk = next_live_block<D, R>(gq, b0, b1, s, live, qcull);
        if constexpr (kStage) {
            // one point per thread; past the last point a clamped (valid) row is
            // loaded and replaced by zeros, so no address is ever selected
            auto load_pt = [&](int bb) -> float4 {
                const long long p = (long long)bb * kCullBlk + threadIdx.x;
                const float4 t = X4[p < n ? p : (long long)n - 1];
                return p < n ? t : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            };
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (blk < b1) v = load_pt(blk);
            while (blk < b1) {
                __syncthreads();   // the previous block is no longer read
                xs[threadIdx.x] = v;
                __syncthreads();
                const int nxt = next_live_block<D, R>(gq, blk + 1, b1, s, live, qcull);
                if (nxt < b1) v = load_pt(nxt);   // in flight while this block computes
                const int lo = wave * PWD;
                const int hi = min(lo + PWD, n - blk * kCullBlk);
#pragma unroll 4
                for (int p = lo; p < hi; ++p) {
                    const float4 xp = xs[p];   // same address in every lane: broadcast
                    const float x[4] = {xp.x, xp.y, xp.z, xp.w};
                    pair_acc<D, R, KERN>(x, s, acc, a.h2);
                }
                blk = nxt;
            }
        } else {
            // wide rows: each wave streams its 64 points of a live block
            // through scalar loads
            while (blk < b1) {
                const int p0 = blk * kCullBlk + wave * PWD;
                const int p1 = min(p0 + PWD, n);
                stream_rows<D, DP>(xq + (long long)p0 * DP, p1 - p0,
                                   [&](const float (&x)[D]) { pair_acc<D, R, KERN>(x, s, acc, a.h2); });
                blk = next_live_block<D, R>(gq, blk + 1, b1, s, live, qcull);
            }
        }
        // the four wave sums added in wave order
        if (wave > 0) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k <= D; ++k) red[(wave - 1) * V + k * TS + r * 64 + lane] = acc[r][k];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k <= D; ++k) {
                    float v = acc[r][k];
#pragma unroll
                    for (int w2 = 1; w2 < kWaves; ++w2) v += red[(w2 - 1) * V + k * TS + r * 64 + lane];
                    acc[r][k] = v;
                }
        }
        __syncthreads();
        if (chunks == 1) {
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
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float* dst = a.part + (((long long)tile * chunks + chunk) * TS + r * 64 + lane) * (D + 1);
#pragma unroll
                for (int k = 0; k <= D; ++k) dst[k] = acc[r][k];
            }
        }
    }
}

template <int D, int R>
hipError_t launch_cull_t(Batch& b, int t, hipStream_t s) {
    StepArgs a;
    a.Xp = b.Xs;
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
        hipLaunchKernelGGL((step_cull_kernel<D, R, MS_KERNEL_GAUSSIAN>), dim3(b.grid), dim3(kThreads), 0,
                           s, a, b.geom, b.shift, kCullGauss, t);
    else
        hipLaunchKernelGGL((step_cull_kernel<D, R, MS_KERNEL_FLAT>), dim3(b.grid), dim3(kThreads), 0, s,
                           a, b.geom, b.shift, a.h2 * kCullFlatMargin, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize<D, (D <= 4 ? 4 : D), R>(a, t, b.grid, b.n_seeds, s);
}

}  // namespace

bool cull_supported(int d, int n) {
    if (n < kCullMinPoints || d < 1 || d > 32) return false;
    const int D = step_shape(d).D;
    return D <= 4 || D == 8 || D == 16 || D == 32;
}

double cull_reach(int kernel, double h) {
    // the distance beyond which every pair of a block may be skipped: exp2
    // underflow of the Gaussian in packed units (q >= kCullGauss), or the
    // flat window with its margin
    if (kernel == MS_KERNEL_GAUSSIAN) return std::sqrt(2.0 * (double)kCullGauss / 1.4426950408889634) * h;
    return std::sqrt((double)kCullFlatMargin) * h;
}

StepShape step_shape_cull(int d, int B, int n) {
    StepShape sh = step_shape(d);
    sh.DP = sh.D <= 4 ? 4 : sh.D;
    sh.R = 1;
    sh.TS = 64 * sh.R;
    sh.MC = 2 * kCullBlk;   // whole blocks per chunk, at least two
    (void)B;
    (void)n;
    return sh;
}

hipError_t launch_iteration_cull(Batch& b, int t, hipStream_t s) {
    const int D = b.sh.D, R = b.sh.R;
#define FMS_CASE(DD, RR) \
    if (D == DD && R == RR) return launch_cull_t<DD, RR>(b, t, s);
    FMS_CASE(1, 1) FMS_CASE(2, 1) FMS_CASE(3, 1) FMS_CASE(4, 1)
    FMS_CASE(8, 1) FMS_CASE(16, 1) FMS_CASE(32, 1)
#undef FMS_CASE
    return hipErrorInvalidValue;
}

}  // namespace fms
