// k_step_bf16w.hip -- the fused mean-shift iteration in the BF16 form for
// 8 <= D <= 32 (gfx950): every seed-point product on MFMA in bf16 with FP32
// accumulation, used to screen the pairs; every pair whose weight may be
// above the FP32 underflow (2^-127, Gaussian) or inside the window (flat) is
// then computed exactly in FP32 -- distance, weight and accumulation, as the
// FP32 step does it.  Pairs below the screen contribute nothing.
//
// Points are sorted by nearest pivot and shifted by the bounding-box
// midpoint; for a block of 256 of them with centre c and radius R, and a
// seed s (packed units, same frame), x~ = x - c and
//   E = 2 x~.s - (|x~|^2 + 2 x~.c) - |s - c|^2  (= -|x - s|^2).
// One v_mfma_f32_32x32x16_bf16 per 16 slots of K = [x~ | p_hi | p_lo | 0..]
// x [2s | 1 | 1 | 0..] with p = -(|x~|^2 + 2 x~.c) in hi/lo bf16 parts, and
// -|s - c|^2 (FP32) as the accumulator's start value.  The seed operand does
// not depend on the block.  With u = 2^-8 (bf16 rounding) the estimate is
// off by at most
//   eps = 2 (2u + u^2) R |s| + 2^-14 (R^2 + 2 R |c| + |s - c|^2),
// the first term from the rounded products (Cauchy-Schwarz), the second
// bounding the hi/lo and FP32 rounding of the other terms and of the MFMA
// accumulation; a 32 x 32 tile with some E + eps >= the threshold recomputes
// its rows exactly, and each pair keeps its exact weight if and only if its
// own bound passes, so that a pair's result never depends on its tile mates.
// MFMA layouts as in the D <= 4 form: A lane l holds row (point) l%32 and
// k = (l/32)*8..+8; B lane l holds k = (l/32)*8..+8 and column (seed) l%32;
// C lane l holds column l%32 and rows 8(v/4) + 4(l/32) + v%4.

#include "step_common.h"

namespace fms {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kWThreads = 256;     // 4 waves x 32 seeds
constexpr int kWSeeds = 128;       // seeds per tile
constexpr int kWBlk = 256;         // points per staged block

template <int D>
struct WShape {
    static constexpr int KP = ((D + 2 + 15) / 16) * 16;   // K padded to the MFMA depth
    static constexpr int KB = KP / 16;                    // MFMAs per 32 x 32 tile
    static constexpr int PF_BYTES = (kWBlk / 32) * KB * 512 * 2;
    static constexpr int XS_BYTES = kWBlk * D * 4;
    static_assert(PF_BYTES % (16 * kWThreads) == 0 && XS_BYTES % (16 * kWThreads) == 0,
                  "stage layout");
};

struct Bf16wArgs {
    StepArgs base;
    const float* Xs;        // sorted, shifted points (n x D, packed units)
    const float* geom;      // per block: centre[D], radius, |centre|
    int gs;                 // geometry row stride
    const __bf16* pf;       // point operand, [tile][kb][half][point][8]
    const float* shift;     // frame shift (D floats)
    float e_thr;            // screen threshold on E (packed units)
};

__device__ __forceinline__ float bfr(float x) { return (float)(__bf16)x; }

// Point operand of one point: slots [0, D) x~, D and D+1 the hi/lo parts of
// p = -(|x~|^2 + 2 x~.c), the rest 0; padding points carry p = -inf.
template <int D>
__global__ void bf16w_features_kernel(const float* __restrict__ Xs, int n, int npad,
                                      const float* __restrict__ geom, int gs, __bf16* pf) {
    using Sh = WShape<D>;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    const bool live = i < n;
    const float* g = geom + (long long)(i / kWBlk) * gs;
    float xt[D];
    float nx = 0.0f, xc = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xt[k] = live ? Xs[(long long)i * D + k] - g[k] : 0.0f;
        nx = fmaf(xt[k], xt[k], nx);
        xc = fmaf(xt[k], g[k], xc);
    }
    const float p = -(nx + 2.0f * xc);
    const float ph = live ? bfr(p) : -__builtin_inff();
    const float pl = live ? bfr(p - ph) : 0.0f;
    __bf16* out = pf + (long long)(i >> 5) * (Sh::KB * 512) + (i & 31) * 8;
#pragma unroll
    for (int s = 0; s < Sh::KP; ++s) {
        float v = 0.0f;
        if (s < D) v = xt[s];
        else if (s == D) v = ph;
        else if (s == D + 1) v = pl;
        out[(s >> 4) * 512 + ((s >> 3) & 1) * 256 + (s & 7)] = (__bf16)v;
    }
}

template <int D, int KERN>
__global__ __launch_bounds__(kWThreads) void step_bf16w_kernel(Bf16wArgs A, int t) {
    using Sh = WShape<D>;
    constexpr int TS = kWSeeds;
    constexpr int KB = Sh::KB;
    constexpr bool kGauss = KERN == MS_KERNEL_GAUSSIAN;
    const StepArgs& a = A.base;
    Ctl* ctl = a.ctl;
    const int n = a.n;
    const int m = active_count(ctl, t);
    step_prologue(a, t, m);
    if (m == 0) return;
    const int G = gridDim.x;
    const int tiles = (m + TS - 1) / TS;
    const int chunks = chunks_for(m, TS, n, G, a.min_chunk);
    const int nblk = (n + kWBlk - 1) / kWBlk;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int col = lane & 31, hf = lane >> 5;

    __shared__ __attribute__((aligned(16))) char stage[Sh::PF_BYTES + Sh::XS_BYTES];
    __shared__ float fin[(D + 1) * TS];
    const __bf16* spf = reinterpret_cast<const __bf16*>(stage);
    const float* sxs = reinterpret_cast<const float*>(stage + Sh::PF_BYTES);
    unsigned long long refined = 0;   // wave-uniform: counted from ballots

    const const_f32_ptr gq = wave_uniform_const(A.geom);   // block geometry: scalar loads
    for (int item = blockIdx.x; item < tiles * chunks; item += G) {
        const int tile = item % tiles;
        const int chunk = item / tiles;
        const int b0 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * chunk / chunks));
        const int b1 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * (chunk + 1) / chunks));
        const int slot = tile * TS + wave * 32 + col;
        const bool live = slot < m;
        const unsigned long long lmask = __ballot(live);   // lanes holding a seed
        const int j = a.act_in[live ? slot : 0];
        float shat[D], aex[D];
        float wex = 0.0f, ns2 = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            shat[k] = a.S[(long long)j * D + k] * a.scale - A.shift[k];
            ns2 = fmaf(shat[k], shat[k], ns2);
            aex[k] = 0.0f;
        }
        const float ns = sqrtf(ns2) * 1.0001f;
        // seed operand [2s | 1 | 1 | 0..]: this lane's 8 K slots of each MFMA
        bf16x8 sfrag[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int sl = kb * 16 + e;   // the slot for hf = 0; hf = 1 adds 8
                const float v0 = sl < D ? 2.0f * shat[sl < D ? sl : 0]
                                        : ((sl == D || sl == D + 1) ? 1.0f : 0.0f);
                const int sh = sl + 8;
                const float v1 = sh < D ? 2.0f * shat[sh < D ? sh : 0]
                                        : ((sh == D || sh == D + 1) ? 1.0f : 0.0f);
                sfrag[kb][e] = (__bf16)(hf ? v1 : v0);
            }
        }

        // the point operand of the chunk's first block travels in registers,
        // up to six 16-byte vectors per thread held in separate variables (an
        // array would be placed in scratch memory and its loads waited on)
        constexpr int NV = Sh::PF_BYTES / 16 / kWThreads;
        static_assert(NV >= 1 && NV <= 6, "operand vectors per thread");
        uint4 v0 = {}, v1 = {}, v2 = {}, v3 = {}, v4 = {}, v5 = {};
#define FMS_PF_LOAD(blk_)                                                                          \
    do {                                                                                           \
        const uint4* g_ = reinterpret_cast<const uint4*>(A.pf + (long long)(blk_) * (Sh::PF_BYTES / 2)); \
        v0 = g_[threadIdx.x];                                                                      \
        if constexpr (NV > 1) v1 = g_[kWThreads + threadIdx.x];                                    \
        if constexpr (NV > 2) v2 = g_[2 * kWThreads + threadIdx.x];                                \
        if constexpr (NV > 3) v3 = g_[3 * kWThreads + threadIdx.x];                                \
        if constexpr (NV > 4) v4 = g_[4 * kWThreads + threadIdx.x];                                \
        if constexpr (NV > 5) v5 = g_[5 * kWThreads + threadIdx.x];                                \
    } while (0)
        FMS_PF_LOAD(b0);
        for (int blk = b0; blk < b1; ++blk) {
            __syncthreads();   // the previous block's operands are no longer read
            {
                uint4* l_ = reinterpret_cast<uint4*>(stage);
                l_[threadIdx.x] = v0;
                if constexpr (NV > 1) l_[kWThreads + threadIdx.x] = v1;
                if constexpr (NV > 2) l_[2 * kWThreads + threadIdx.x] = v2;
                if constexpr (NV > 3) l_[3 * kWThreads + threadIdx.x] = v3;
                if constexpr (NV > 4) l_[4 * kWThreads + threadIdx.x] = v4;
                if constexpr (NV > 5) l_[5 * kWThreads + threadIdx.x] = v5;
            }
            if (blk + 1 < b1) FMS_PF_LOAD(blk + 1);   // travels while this block computes
#undef FMS_PF_LOAD
            const const_f32_ptr gm = gq + (long long)blk * A.gs;
            const float R = gm[D], cn = gm[D + 1];
            float st2 = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const float dk = shat[k] - gm[k];
                st2 = fmaf(dk, dk, st2);
            }
            const float eps = 0.016f * R * ns + (1.0f / 16384.0f) * (R * R + 2.0f * R * cn + st2);
            // The FP32 points are needed only by a pair that passes the screen:
            // E + eps >= thr implies -|x - s|^2 >= thr - 2 eps, and
            // |x - s| >= |s - c| - R for every point of the block, so a seed
            // for which (|s - c| - R)^2 > 2 eps - thr has no such pair here.
            const float lower = sqrtf(st2) * (1.0f - 1e-5f) - R;
            const bool maybe = live && (lower <= 0.0f ||
                                        lower * lower <= (2.0f * eps - A.e_thr) * 1.001f + 1e-6f);
            if (__syncthreads_or(maybe)) {   // (also the barrier for the operand above)
                const uint4* xsg = reinterpret_cast<const uint4*>(A.Xs + (long long)blk * kWBlk * D);
                const long long xs_vecs = ((long long)n * D - (long long)blk * kWBlk * D) / 4;
                uint4* sx = reinterpret_cast<uint4*>(stage + Sh::PF_BYTES);
#pragma unroll
                for (int q = 0; q < Sh::XS_BYTES / 16 / kWThreads; ++q) {
                    const int f = q * kWThreads + threadIdx.x;
                    sx[f] = f < xs_vecs ? xsg[f] : uint4{};
                }
                __syncthreads();
            }
#pragma unroll 1
            for (int tt = 0; tt < kWBlk / 32; ++tt) {
                f32x16 E;
#pragma unroll
                for (int v = 0; v < 16; ++v) E[v] = -st2;
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const bf16x8 afrag = *reinterpret_cast<const bf16x8*>(
                        spf + (tt * KB + kb) * 512 + hf * 256 + col * 8);
                    E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afrag, sfrag[kb], E, 0, 0, 0);
                }
                const float m0 = fmaxf(fmaxf(E[0], E[1]), E[2]);
                const float m1 = fmaxf(fmaxf(E[3], E[4]), E[5]);
                const float m2 = fmaxf(fmaxf(E[6], E[7]), E[8]);
                const float m3 = fmaxf(fmaxf(E[9], E[10]), E[11]);
                const float m4 = fmaxf(fmaxf(E[12], E[13]), E[14]);
                const float emax = fmaxf(fmaxf(fmaxf(m0, m1), m2), fmaxf(fmaxf(m3, m4), E[15]));
                // only lanes holding a seed: the FP32 points of this block
                // are in LDS only if one of them may need them (a lane past
                // the active count would read what an earlier block or
                // kernel left there, and even at weight 0 a NaN there
                // spreads into the sums)
                if (!__ballot(live && emax + eps >= A.e_thr)) continue;
                unsigned long long nref = 0;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const bool need = live && E[v] + eps >= A.e_thr;
                    const float* xr = sxs + (tt * 32 + 8 * (v >> 2) + 4 * hf + (v & 3)) * D;
                    // differences computed twice (distance, then accumulation)
                    // rather than held: the registers matter more than the
                    // subtractions on the few pairs that pass the screen
                    float q2 = 0.0f;
#pragma unroll
                    for (int k4 = 0; k4 < D; k4 += 4) {
                        const float4 x4 = *reinterpret_cast<const float4*>(xr + k4);
                        const float d0 = x4.x - shat[k4], d1 = x4.y - shat[k4 + 1];
                        const float d2 = x4.z - shat[k4 + 2], d3 = x4.w - shat[k4 + 3];
                        q2 = fmaf(d0, d0, q2);
                        q2 = fmaf(d1, d1, q2);
                        q2 = fmaf(d2, d2, q2);
                        q2 = fmaf(d3, d3, q2);
                    }
                    float we = kGauss ? __builtin_amdgcn_exp2f(-q2) : (q2 <= a.h2 ? 1.0f : 0.0f);
                    we = need ? we : 0.0f;
                    wex += we;
#pragma unroll
                    for (int k4 = 0; k4 < D; k4 += 4) {
                        const float4 x4 = *reinterpret_cast<const float4*>(xr + k4);
                        aex[k4] = fmaf(we, x4.x - shat[k4], aex[k4]);
                        aex[k4 + 1] = fmaf(we, x4.y - shat[k4 + 1], aex[k4 + 1]);
                        aex[k4 + 2] = fmaf(we, x4.z - shat[k4 + 2], aex[k4 + 2]);
                        aex[k4 + 3] = fmaf(we, x4.w - shat[k4 + 3], aex[k4 + 3]);
                    }
                    nref += __popcll(__ballot(need) & lmask);   // scalar unit
                }
                refined += nref;
            }
        }

        // chunk partial: the two lane halves saw different points of the seed
#pragma unroll
        for (int k = 0; k < D; ++k) aex[k] += __shfl_xor(aex[k], 32);
        wex += __shfl_xor(wex, 32);
        const int pos = wave * 32 + col;
        if (chunks == 1) {
            if (hf == 0) {
#pragma unroll
                for (int k = 0; k < D; ++k) fin[k * TS + pos] = aex[k];
                fin[D * TS + pos] = wex;
            }
            __syncthreads();
            finalize_tile<D, D, 2>(a, t, m, tile, fin);
            __syncthreads();
        } else if (hf == 0) {
            float* dst = a.part + (((long long)tile * chunks + chunk) * TS + pos) * (D + 1);
#pragma unroll
            for (int k = 0; k < D; ++k) dst[k] = aex[k];
            dst[D] = wex;
        }
    }
    // refined pairs: wave counts summed per workgroup, one atomic per
    // workgroup on one of the spread counters
    __shared__ unsigned long long wref[kWaves];
    if (lane == 0) wref[threadIdx.x >> 6] = refined;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = 0;
        for (int w = 0; w < kWaves; ++w) r += wref[w];
        if (r) atomicAdd((unsigned long long*)&ctl->refined[(blockIdx.x % kRefinedSlots) * kRefinedStride], r);
    }
}

template <int D>
hipError_t launch_bf16w_t(Batch& b, int t, hipStream_t s) {
    Bf16wArgs A;
    StepArgs& a = A.base;
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
    A.Xs = b.Xs;
    A.geom = b.geom;
    A.gs = geom_stride(D);
    A.pf = (const __bf16*)b.pf;
    A.shift = b.shift;
    A.e_thr = b.e_thr;
    if (b.kernel == MS_KERNEL_GAUSSIAN)
        hipLaunchKernelGGL((step_bf16w_kernel<D, MS_KERNEL_GAUSSIAN>), dim3(b.grid), dim3(kWThreads), 0,
                           s, A, t);
    else
        hipLaunchKernelGGL((step_bf16w_kernel<D, MS_KERNEL_FLAT>), dim3(b.grid), dim3(kWThreads), 0, s,
                           A, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize<D, D, 2>(a, t, b.grid, b.n_seeds, s);
}

}  // namespace

bool bf16w_dims(int D) { return D == 8 || D == 16 || D == 32; }

hipError_t launch_iteration_bf16w(Batch& b, int t, hipStream_t s) {
    switch (b.sh.D) {
        case 8: return launch_bf16w_t<8>(b, t, s);
        case 16: return launch_bf16w_t<16>(b, t, s);
        case 32: return launch_bf16w_t<32>(b, t, s);
        default: return hipErrorInvalidValue;
    }
}

size_t bf16w_feature_bytes(int n, int D) {
    const size_t npad = (size_t)((n + kWBlk - 1) / kWBlk) * kWBlk;
    const int KP = ((D + 2 + 15) / 16) * 16;
    return npad * KP * 2;
}

hipError_t launch_bf16w_features(const float* Xs, int n, int D, const float* geom, void* feat,
                                 hipStream_t s) {
    const int npad = (n + kWBlk - 1) / kWBlk * kWBlk;
    __bf16* pf = (__bf16*)feat;
    const int gs = geom_stride(D);
    switch (D) {
        case 8:
            hipLaunchKernelGGL(bf16w_features_kernel<8>, dim3((npad + 255) / 256), dim3(256), 0, s, Xs, n,
                               npad, geom, gs, pf);
            break;
        case 16:
            hipLaunchKernelGGL(bf16w_features_kernel<16>, dim3((npad + 255) / 256), dim3(256), 0, s, Xs, n,
                               npad, geom, gs, pf);
            break;
        case 32:
            hipLaunchKernelGGL(bf16w_features_kernel<32>, dim3((npad + 255) / 256), dim3(256), 0, s, Xs, n,
                               npad, geom, gs, pf);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fms
