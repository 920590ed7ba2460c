// k_step_bf16.hip -- the fused mean-shift iteration in the BF16+refine form
// for gfx950 (D <= 4): the seed-point products on MFMA in bf16 with FP32
// accumulation, an exact FP32 recompute for every pair that may lie within
// refine_radius * h, and the weighted sums on MFMA as well.
//
// Same result as the FP32 step (the kernel-weighted mean over all n points,
// Section II-B), computed as follows for a wave of 32 seeds and a block of 256
// points (points in Morton order, centred on the block's reference c):
//   E   = 2 x~.s~ - |x~|^2 - |s~|^2   (= -|x - s|^2 in packed units; x~ = x-c)
//        one v_mfma_f32_32x32x16_bf16 per 32 points, the products split into
//        bf16 hi/lo parts (x~h s~h + x~h s~l + x~l s~h) and the norms hi/lo;
//   the estimate is off by at most kappa (R + |s~|)^2 (R = block radius), so
//   every pair with E + kappa (R + |s~|)^2 >= -(refine_radius h)^2 (packed
//   units) -- every pair that may lie within refine_radius * h -- is
//   recomputed exactly as the FP32 step does it: direct-difference distance,
//   FP32 weight, FP32 accumulation of w (x - s) and w.  When the block's
//   bound (its radius and the seed's distance to its centre) admits such a
//   pair for some seed of the wave, the wave computes every pair of its half
//   block that way and no product at all (the live blocks near the seeds are
//   mostly within the radius anyway); otherwise no pair of the block can
//   need it and the products alone are used;
//   the remaining (far) pairs take their weight from the estimate (Gaussian;
//   zero for the flat window), packed to bf16, and  sum_p w [x~h | x~l | 1]
//   is accumulated by two more MFMAs per 32 points in FP32.
// MFMA layouts (one wave): A (32x16) lane l holds row l%32, k = (l/32)*8..+8;
// B (16x32) lane l holds k = (l/32)*8..+8, column l%32; C (32x32) lane l holds
// column l%32 and rows 8(v/4) + 4(l/32) + v%4, v = 0..15.  The first product
// puts points on rows and seeds on columns, so each lane already owns one
// seed's weights for 16 points; using those 16 points, in that order, as the
// K dimension of the second product needs no transpose: the point-side
// operand of the second product is stored with the same K order.

#include "step_common.h"

namespace fms {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kB16Threads = 256;    // 4 waves x 32 seeds
constexpr int kB16Seeds = 128;      // seeds per tile of the finalize for D > 4
constexpr int kBlk = 256;           // points per staged block (one centre)

struct Bf16Args {
    StepArgs base;
    const float* Xs;        // points in Morton order (n x 4, packed units)
    const float* geom;      // per block: centre[4], radius
    const __bf16* pf;       // per padded point: 16 first-product features
    const __bf16* xv;       // per 32-point tile: second-product operand, K order
    float e_thr;            // refine when E + eps >= e_thr
    float kappa;            // error bound coefficient
};

__device__ __forceinline__ float bf(float x) { return (float)(__bf16)x; }

// Point-side operands, built once per fit from the sorted points and the
// block centres.  Feature slots s of point i: s in [0,D) x~h, [D,2D) x~h,
// [2D,3D) x~l, 3D: -|x~|^2 hi, 3D+1: -|x~|^2 lo, 3D+2 and 3D+3: 1 (padding
// points carry -inf so that their weight is 0), stored as
// pf[tile][s / 8][i % 32][s % 8] for the 32-point tile of i, so that the
// 64 lanes of a wave read 1 KB contiguously (no LDS bank conflicts).
// xv[tile][kb][hh][c][e]: column c of [x~h | x~l | 1] for the point
// 16 kb + 8 (e/4) + 4 hh + e%4 of the tile.
template <int D>
__global__ void bf16_features_kernel(const float* __restrict__ Xs, int n, int npad,
                                     const float* __restrict__ geom, __bf16* pf, __bf16* xv) {
    constexpr int NCOL = 2 * D + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    const bool live = i < n;
    const float* g = geom + (long long)(i / kBlk) * kGeomStride;
    float xt[D], xh[D], xl[D], nx = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xt[k] = live ? Xs[(long long)i * 4 + k] - g[k] : 0.0f;
        xh[k] = bf(xt[k]);
        xl[k] = bf(xt[k] - xh[k]);
        nx = fmaf(xt[k], xt[k], nx);
    }
    const float nxh = bf(nx), nxl = bf(nx - nxh);
    __bf16* out = pf + (long long)(i >> 5) * 512 + (i & 31) * 8;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        float v = 0.0f;
        if (s < D) v = xh[s];
        else if (s < 2 * D) v = xh[s - D];
        else if (s < 3 * D) v = xl[s - 2 * D];
        else if (s == 3 * D) v = live ? -nxh : -__builtin_inff();
        else if (s == 3 * D + 1) v = live ? -nxl : 0.0f;
        else if (s < 3 * D + 4) v = 1.0f;
        out[(s >> 3) * 256 + (s & 7)] = (__bf16)v;
    }
    const int tile = i >> 5, p = i & 31;
    const int kb = p >> 4, r = p & 15, hh = (r >> 2) & 1, e = ((r >> 3) << 2) | (r & 3);
    __bf16* o2 = xv + (long long)tile * 512 + ((kb * 2 + hh) * 16) * 8 + e;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        float v = 0.0f;
        if (c < D) v = xh[c];
        else if (c < 2 * D) v = xl[c - D];
        else if (c < NCOL) v = live ? 1.0f : 0.0f;
        o2[c * 8] = (__bf16)v;
    }
}

// Seed features of the first product relative to a block centre.
template <int D>
__device__ __forceinline__ bf16x8 seed_frag(const float* st, float ns, int hf) {
    float sh[D], sl[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        sh[k] = bf(st[k]);
        sl[k] = bf(st[k] - sh[k]);
    }
    const float nsh = bf(ns), nsl = bf(ns - nsh);
    auto slot_val = [&](const int s2) -> float {
        if (s2 < D) return 2.0f * sh[s2 < D ? s2 : 0];
        if (s2 < 2 * D) return 2.0f * sl[s2 - D < D ? s2 - D : 0];
        if (s2 < 3 * D) return 2.0f * sh[s2 - 2 * D < D ? s2 - 2 * D : 0];
        if (s2 < 3 * D + 2) return 1.0f;
        if (s2 == 3 * D + 2) return -nsh;
        if (s2 == 3 * D + 3) return -nsl;
        return 0.0f;
    };
    bf16x8 f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float lo = slot_val(q), hi = slot_val(8 + q);
        f[q] = (__bf16)(hf ? hi : lo);
    }
    return f;
}

// Block culling.  For a seed s~ (packed units) and block b (centre c, radius
// R_b), every point lies at squared distance q >= lb^2, lb = |s~ - c| - R_b,
// and the estimate satisfies E <= -q + eps (eps = kappa (R_b + |s~ - c|)^2,
// the same bound the refine test uses).  When lb^2 exceeds both -e_thr + 2 eps
// and (Gaussian) 127 + eps, no pair of the block can pass the refine test or
// the far test, so the tile loop would add nothing for this seed: a group of
// 32 seeds skips the block when all of its seeds are that far, and the wave
// skips the block when both groups do.  The result is the one of the unculled
// loop.  Every wave of a workgroup holds the same seeds, so every wave takes
// the same decisions.
template <int D, int R, bool kGauss>
__device__ __forceinline__ bool bf16_block_near(const_f32_ptr gm, const float (&shat)[R][D],
                                                const bool (&live)[R], float kappa, float e_thr,
                                                bool (&gnear)[R]) {
    bool any = false;
#pragma unroll
    for (int g = 0; g < R; ++g) {
        float ns = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float u = shat[g][k] - gm[k];
            ns = fmaf(u, u, ns);
        }
        const float dist = sqrtf(ns);
        const float rr = gm[4] + dist;
        const float ep = kappa * rr * rr;
        float need = -e_thr + 2.0f * ep;
        if (kGauss) need = fmaxf(need, 127.0f + ep);
        need = need * 1.001f + 1e-3f;
        const float lb = dist - gm[4];
        const bool nl = live[g] && !(lb > 0.0f && lb * lb > need);
        gnear[g] = __ballot(nl) != 0ull;
        any = any || gnear[g];
    }
    return any;
}

// One iteration of the BF16 form.  A workgroup takes a tile of 64 seeds (two
// groups of 32) and a chunk of whole blocks.  Wave w holds group w / 2 and
// computes the 32-point tiles 4 (w % 2) .. 4 (w % 2) + 3 (points
// [128 (w % 2), 128 (w % 2) + 128)) of every block of the chunk that some seed
// of its group may see, with no barrier across waves: the first- and
// second-product operands come from global memory straight into the MFMA
// registers (one tile ahead), the wave's 128 FP32 points for the exact path
// through a wave-private LDS slice.  The two half-block sums of a seed are
// added in wave order.
constexpr int kTilesPerWave = kBlk / 32 / 2;   // 32-point MFMA tiles per wave and block
constexpr int kPtsPerWave = kBlk / 2;

template <int D, int KERN, int R>
__global__ __launch_bounds__(kB16Threads) void step_bf16_kernel(Bf16Args A, int t) {
    constexpr int TS = 64;
    constexpr int NCOL = 2 * D + 1;
    constexpr bool kGauss = KERN == MS_KERNEL_GAUSSIAN;
    static_assert(R == 1, "one group of 32 seeds per wave");
    const StepArgs& a = A.base;
    Ctl* ctl = a.ctl;
    const int n = a.n;
    const int m = active_count(ctl, t);
    step_prologue(a, t, m);
    if (m == 0) return;
    const int G = gridDim.x;
    const int tiles = (m + TS - 1) / TS;
    const int chunks = chunks_for(m, TS, n, G, a.min_chunk);
    const int nblk = (n + kBlk - 1) / kBlk;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = wave >> 1, half = wave & 1;
    const int lane = threadIdx.x & 63;
    const int col = lane & 31, hf = lane >> 5;

    __shared__ float4 sxs_all[kWaves][kPtsPerWave];
    __shared__ float tr[kWaves][NCOL][33];   // per-wave transpose (padded)
    __shared__ float red[kWaves][D + 1][32]; // per-wave seed sums
    float4* sxs = sxs_all[wave];
    const float4* __restrict__ xsg = reinterpret_cast<const float4*>(A.Xs);
    unsigned long long refined = 0;   // wave-uniform: counted from ballots

    const const_f32_ptr gq = wave_uniform_const(A.geom);
    for (int item = blockIdx.x; item < tiles * chunks; item += G) {
        const int tile = item % tiles;
        const int chunk = item / tiles;
        const int b0 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * chunk / chunks));
        const int b1 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * (chunk + 1) / chunks));
        float shat[1][D], arun[D], aex[D], wrun = 0.0f, wex = 0.0f;
        bool live[1];
        {
            const int slot = tile * TS + grp * 32 + col;
            live[0] = slot < m;
            const int j = a.act_in[live[0] ? slot : tile * TS];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                shat[0][k] = a.S[(long long)j * 4 + k] * a.scale;
                arun[k] = aex[k] = 0.0f;
            }
        }
        const unsigned long long lmask = __ballot(live[0]);   // lanes holding a seed
        bool gn[1];
        int blk = b0;
        while (blk < b1 && !bf16_block_near<D, 1, kGauss>(gq + (long long)blk * kGeomStride, shat, live,
                                                           A.kappa, A.e_thr, gn))
            ++blk;
        float4 p0 = {}, p1 = {};
        auto fetch_pts = [&](int bb) {
            const long long p = (long long)bb * kBlk + half * kPtsPerWave + lane;
            p0 = p < n ? xsg[p] : float4{};
            p1 = p + 64 < n ? xsg[p + 64] : float4{};
        };
        if (blk < b1) fetch_pts(blk);

        while (blk < b1) {
            // the previous block's points are no longer read (LDS operations
            // of one wave complete in order)
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            sxs[lane] = p0;
            sxs[64 + lane] = p1;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            int nxt = blk + 1;
            while (nxt < b1 && !bf16_block_near<D, 1, kGauss>(gq + (long long)nxt * kGeomStride, shat,
                                                               live, A.kappa, A.e_thr, gn))
                ++nxt;
            if (nxt < b1) fetch_pts(nxt);   // next live block's points travel while this one computes

            const const_f32_ptr gm = gq + (long long)blk * kGeomStride;
            float st[D];
            float ns = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                st[k] = shat[0][k] - gm[k];
                ns = fmaf(st[k], st[k], ns);
            }
            const float rr = gm[4] + sqrtf(ns);
            const float eps = A.kappa * rr * rr;
            {
                // some seed of the wave may have a pair of this block within
                // the refine radius (its bound admits E + eps >= e_thr): the
                // wave computes its half block exactly in FP32 (points from
                // LDS), every pair of every seed, with no products -- the live
                // blocks near the seeds mostly lie within the radius anyway.
                // Otherwise no pair of the block can need the recompute and
                // the products below serve.  A seed's result thus depends on
                // its wave mates; the finalize of this form compacts the
                // active list in list order (StepArgs::ordered), so the
                // grouping, and the result, are the same on every run
                const float lbk = sqrtf(ns) - gm[4];
                const bool may = live[0] && !(lbk > 0.0f && lbk * lbk > -A.e_thr + 2.0f * eps);
                if (__ballot(may)) {
                    const long long pb = (long long)blk * kBlk + half * kPtsPerWave;
                    unsigned long long nex = 0;
#pragma unroll 1
                    for (int tt = 0; tt < kTilesPerWave; ++tt) {
                        const float4* xr = sxs + tt * 32 + 4 * hf;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            float4 x4[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) x4[u] = xr[8 * q + u];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const bool valid = pb + tt * 32 + 8 * q + 4 * hf + u < n;
                                const float xv[4] = {x4[u].x, x4[u].y, x4[u].z, x4[u].w};
                                float dx[D], q2 = 0.0f;
#pragma unroll
                                for (int k = 0; k < D; ++k) {
                                    dx[k] = xv[k] - shat[0][k];
                                    q2 = fmaf(dx[k], dx[k], q2);
                                }
                                float we = kGauss ? __builtin_amdgcn_exp2f(-q2) : (q2 <= a.h2 ? 1.0f : 0.0f);
                                we = valid ? we : 0.0f;
                                wex += we;
#pragma unroll
                                for (int k = 0; k < D; ++k) aex[k] = fmaf(we, dx[k], aex[k]);
                                nex += __popcll(__ballot(valid) & lmask);
                            }
                        }
                    }
                    refined += nex;
                    blk = nxt;
                    continue;
                }
            }
            const bf16x8 sfrag = seed_frag<D>(st, ns, hf);
            f32x16 out = f32x16{};
            bool used = false;
            const long long tt0 = (long long)blk * (kBlk / 32) + half * kTilesPerWave;
            const __bf16* pfb = A.pf + tt0 * 512 + hf * 256 + col * 8;
            const __bf16* xvb = A.xv + tt0 * 512 + (hf * 16 + col) * 8;
            bf16x8 anext = *reinterpret_cast<const bf16x8*>(pfb);
#pragma unroll 1
            for (int tt = 0; tt < kTilesPerWave; ++tt) {
                const bf16x8 afrag = anext;
                if (tt + 1 < kTilesPerWave) anext = *reinterpret_cast<const bf16x8*>(pfb + (tt + 1) * 512);
                bf16x8 x0 = {}, x1 = {};
                if (kGauss && col < NCOL) {
                    x0 = *reinterpret_cast<const bf16x8*>(xvb + tt * 512);
                    x1 = *reinterpret_cast<const bf16x8*>(xvb + tt * 512 + 2 * 16 * 8);
                }
                f32x16 E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afrag, sfrag, f32x16{}, 0, 0, 0);
                // tree of maxima (depth 3 instead of a chain of 8)
                const float m0 = fmaxf(fmaxf(E[0], E[1]), E[2]);
                const float m1 = fmaxf(fmaxf(E[3], E[4]), E[5]);
                const float m2 = fmaxf(fmaxf(E[6], E[7]), E[8]);
                const float m3 = fmaxf(fmaxf(E[9], E[10]), E[11]);
                const float m4 = fmaxf(fmaxf(E[12], E[13]), E[14]);
                const float emax = fmaxf(fmaxf(fmaxf(m0, m1), m2), fmaxf(fmaxf(m3, m4), E[15]));
                const bool ref = __ballot(emax + eps >= A.e_thr);
                if (ref) {
                    // some pair of this 32 x 32 tile may lie within the refine
                    // radius: every row of the lane is recomputed exactly in
                    // FP32 (points from LDS), and each pair keeps the exact
                    // weight if and only if its own bound flags it (its
                    // estimate is then replaced by -inf, weight 0 in the bf16
                    // sums), so the result of a pair never depends on its
                    // tile mates
                    const float4* xr = sxs + tt * 32 + 4 * hf;
                    unsigned long long nref = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float4 x4[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) x4[u] = xr[8 * q + u];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int v = 4 * q + u;
                            const bool need = E[v] + eps >= A.e_thr;
                            const float xv[4] = {x4[u].x, x4[u].y, x4[u].z, x4[u].w};
                            float dx[D], q2 = 0.0f;
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                dx[k] = xv[k] - shat[0][k];
                                q2 = fmaf(dx[k], dx[k], q2);
                            }
                            float we = kGauss ? __builtin_amdgcn_exp2f(-q2) : (q2 <= a.h2 ? 1.0f : 0.0f);
                            we = need ? we : 0.0f;
                            wex += we;
#pragma unroll
                            for (int k = 0; k < D; ++k) aex[k] = fmaf(we, dx[k], aex[k]);
                            nref += __popcll(__ballot(need) & lmask);   // scalar unit
                            E[v] = need ? -__builtin_inff() : E[v];
                        }
                    }
                    refined += nref;
                }
                // far pairs (Gaussian only): weights from the estimate, unless
                // every weight of the wave left to them underflows (2^-127;
                // the refined pairs now carry -inf)
                float fmax = emax;
                if (ref) {
                    const float r0 = fmaxf(fmaxf(E[0], E[1]), E[2]);
                    const float r1 = fmaxf(fmaxf(E[3], E[4]), E[5]);
                    const float r2 = fmaxf(fmaxf(E[6], E[7]), E[8]);
                    const float r3 = fmaxf(fmaxf(E[9], E[10]), E[11]);
                    const float r4 = fmaxf(fmaxf(E[12], E[13]), E[14]);
                    fmax = fmaxf(fmaxf(fmaxf(r0, r1), r2), fmaxf(fmaxf(r3, r4), E[15]));
                }
                if (kGauss && __ballot(fmax >= -127.0f)) {
                    bf16x8 w0, w1;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        w0[q] = (__bf16)__builtin_amdgcn_exp2f(E[q]);
                        w1[q] = (__bf16)__builtin_amdgcn_exp2f(E[8 + q]);
                    }
                    out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, x0, out, 0, 0, 0);
                    out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, x1, out, 0, 0, 0);
                    used = true;
                }
            }
            // ---- out[seed row][col] -> per-seed sums through a wave-local
            // transpose (LDS operations of one wave complete in order)
            if (__ballot(used)) {
                if (col < NCOL) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) tr[wave][col][8 * (v >> 2) + 4 * hf + (v & 3)] = out[v];
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                const float Wb = tr[wave][2 * D][col];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float sx = tr[wave][k][col] + tr[wave][D + k][col];
                    // sum w (x~ - s~) = sum w (x - s): the block centre cancels
                    arun[k] += sx - st[k] * Wb;
                }
                wrun += Wb;
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
            blk = nxt;
        }

        // ---- this wave's sums per seed: the two lane halves saw different
        // points of the same seed
#pragma unroll
        for (int k = 0; k < D; ++k) {
            aex[k] += __shfl_xor(aex[k], 32);
            arun[k] += aex[k];
        }
        wex += __shfl_xor(wex, 32);
        wrun += wex;
        if (hf == 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) red[wave][k][col] = arun[k];
            red[wave][D][col] = wrun;
        }
        __syncthreads();
        // the two half-block sums of seed pos = 32 g + c, first half first
        float v[D + 1];
        const int pos = threadIdx.x;
        if (pos < TS) {
            const int g = pos >> 5, c = pos & 31;
#pragma unroll
            for (int k = 0; k <= D; ++k) v[k] = red[2 * g][k][c] + red[2 * g + 1][k][c];
        }
        __syncthreads();
        if (chunks == 1 && !a.ordered) {
            float* sums = &red[0][0][0];   // (D + 1) x 64 floats: sums[k * TS + pos]
            if (pos < TS) {
#pragma unroll
                for (int k = 0; k <= D; ++k) sums[k * TS + pos] = v[k];
            }
            __syncthreads();
            finalize_tile<D, 4, 1>(a, t, m, tile, sums);
            __syncthreads();
        } else if (pos < TS) {
            float* dst = a.part + (((long long)tile * chunks + chunk) * TS + pos) * (D + 1);
#pragma unroll
            for (int k = 0; k <= D; ++k) dst[k] = v[k];
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

template <int D, int R>
hipError_t launch_bf16_t(Batch& b, int t, hipStream_t s) {
    Bf16Args A;
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
    a.ordered = 1;
    A.Xs = b.Xs;
    A.geom = b.geom;
    A.pf = (const __bf16*)b.pf;
    A.xv = (const __bf16*)b.xv;
    A.e_thr = b.e_thr;
    A.kappa = b.kappa;
    if (b.kernel == MS_KERNEL_GAUSSIAN)
        hipLaunchKernelGGL((step_bf16_kernel<D, MS_KERNEL_GAUSSIAN, R>), dim3(b.grid),
                           dim3(kB16Threads), 0, s, A, t);
    else
        hipLaunchKernelGGL((step_bf16_kernel<D, MS_KERNEL_FLAT, R>), dim3(b.grid), dim3(kB16Threads),
                           0, s, A, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize<D, 4, 1>(a, t, b.grid, b.n_seeds, s);
}

}  // namespace

StepShape step_shape_bf16(int d, int B) {
    StepShape sh = step_shape(d);
    sh.MC = 256;           // one staged block per point chunk, at least
    if (sh.D > 4) {        // 4 waves x 32 seeds
        sh.R = 2;
        sh.TS = kB16Seeds;
        return sh;
    }
    // a tile of 64 seeds (two groups of 32) held by all four waves, chunks
    // of at least two blocks
    sh.R = 1;              // the finalize geometry: TS = 64 * R
    sh.TS = 64;
    sh.MC = 2 * kBlk;
    (void)B;
    return sh;
}

bool bf16_supported(int d) { return d >= 1 && (d <= 4 || (d <= 32 && bf16w_dims(step_shape(d).D))); }

hipError_t launch_iteration_bf16(Batch& b, int t, hipStream_t s) {
    if (b.sh.D > 4)
        return b.kernel == MS_KERNEL_GAUSSIAN ? launch_iteration_bf16f(b, t, s) : launch_iteration_bf16w(b, t, s);
    switch (b.sh.D) {
        case 1: return launch_bf16_t<1, 1>(b, t, s);
        case 2: return launch_bf16_t<2, 1>(b, t, s);
        case 3: return launch_bf16_t<3, 1>(b, t, s);
        case 4: return launch_bf16_t<4, 1>(b, t, s);
        default: return hipErrorInvalidValue;
    }
}

size_t bf16_feature_bytes(int n) {
    const size_t npad = (size_t)((n + kBlk - 1) / kBlk) * kBlk;
    return npad * 16 * 2 + npad * 16 * 2;   // pf + xv (16 bf16 per point each)
}

hipError_t launch_bf16_features(const float* Xs, int n, int d, const float* geom, void* feat,
                                hipStream_t s) {
    const int npad = (n + kBlk - 1) / kBlk * kBlk;
    __bf16* pf = (__bf16*)feat;
    __bf16* xv = pf + (size_t)npad * 16;
    switch (step_shape(d).D) {
#define FMS_CASE(DD)                                                                              \
    case DD:                                                                                       \
        hipLaunchKernelGGL(bf16_features_kernel<DD>, dim3((npad + 255) / 256), dim3(256), 0, s, Xs, \
                           n, npad, geom, pf, xv);                                                 \
        break;
        FMS_CASE(1)
        FMS_CASE(2)
        FMS_CASE(3)
        FMS_CASE(4)
#undef FMS_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fms
