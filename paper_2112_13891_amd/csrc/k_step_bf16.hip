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
//   FP32 weight, FP32 accumulation of w (x - s) and w;
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
constexpr int kB16Seeds = 128;      // seeds per tile
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

// Bytes staged per 256-point block: first-product features 256 x 32 B,
// second-product operand 8 tiles x 512 B, FP32 points 256 x 16 B.
constexpr int kPfBytes = kBlk * 16 * 2;
constexpr int kXvBytes = (kBlk / 32) * 512 * 2;
constexpr int kXsBytes = kBlk * 16;
constexpr int kStageVecs = (kPfBytes + kXvBytes + kXsBytes) / 16 / kB16Threads;   // per thread

template <int D, int KERN, int R>
__global__ __launch_bounds__(kB16Threads) void step_bf16_kernel(Bf16Args A, int t) {
    constexpr int TS = kB16Seeds * R;   // 4 waves x R groups x 32 seeds
    constexpr int NCOL = 2 * D + 1;     // [x~h | x~l | 1]
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
    const int nblk = (n + kBlk - 1) / kBlk;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int col = lane & 31, hf = lane >> 5;

    __shared__ __attribute__((aligned(16))) char stage[kPfBytes + kXvBytes + kXsBytes];
    __shared__ float tr[kB16Threads / 64][NCOL][33];   // per-wave transpose (padded)
    __shared__ float fin[(D + 1) * TS];
    const __bf16* spf = reinterpret_cast<const __bf16*>(stage);
    const __bf16* sxv = reinterpret_cast<const __bf16*>(stage + kPfBytes);
    const float4* sxs = reinterpret_cast<const float4*>(stage + kPfBytes + kXvBytes);
    unsigned refined = 0;

    static_assert(kStageVecs == 5 && kPfBytes / 16 == 2 * kB16Threads &&
                  kXvBytes / 16 == 2 * kB16Threads && kXsBytes / 16 == kB16Threads,
                  "stage layout");
    for (int item = blockIdx.x; item < tiles * chunks; item += G) {
        const int tile = item % tiles;
        const int chunk = item / tiles;
        const int b0 = (int)((long long)nblk * chunk / chunks);
        const int b1 = (int)((long long)nblk * (chunk + 1) / chunks);
        float shat[R][D], arun[R][D], aex[R][D], wrun[R], wex[R];
        bool live[R];
#pragma unroll
        for (int g = 0; g < R; ++g) {
            const int slot = tile * TS + (wave * R + g) * 32 + col;
            live[g] = slot < m;
            const int j = a.act_in[live[g] ? slot : 0];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                shat[g][k] = a.S[(long long)j * 4 + k] * a.scale;
                arun[g][k] = aex[g][k] = 0.0f;
            }
            wrun[g] = wex[g] = 0.0f;
        }
        // operands of the first block of the chunk, five 16-byte vectors per
        // thread: two of features, two of the second operand, one of points
        uint4 n0, n1, n2, n3, n4;
        {
            const uint4* pfg = reinterpret_cast<const uint4*>(A.pf + (long long)b0 * kBlk * 16);
            const uint4* xvg = reinterpret_cast<const uint4*>(A.xv + (long long)b0 * (kBlk / 32) * 512);
            const uint4* xsg = reinterpret_cast<const uint4*>(A.Xs) + (long long)b0 * kBlk;
            n0 = pfg[threadIdx.x];
            n1 = pfg[kB16Threads + threadIdx.x];
            n2 = xvg[threadIdx.x];
            n3 = xvg[kB16Threads + threadIdx.x];
            n4 = (long long)b0 * kBlk + threadIdx.x < n ? xsg[threadIdx.x] : uint4{};
        }

        for (int blk = b0; blk < b1; ++blk) {
            __syncthreads();   // the previous block's operands are no longer read
            reinterpret_cast<uint4*>(stage)[threadIdx.x] = n0;
            reinterpret_cast<uint4*>(stage)[kB16Threads + threadIdx.x] = n1;
            reinterpret_cast<uint4*>(stage)[2 * kB16Threads + threadIdx.x] = n2;
            reinterpret_cast<uint4*>(stage)[3 * kB16Threads + threadIdx.x] = n3;
            reinterpret_cast<uint4*>(stage)[4 * kB16Threads + threadIdx.x] = n4;
            __syncthreads();
            if (blk + 1 < b1) {   // next block's operands travel while this one computes
                const uint4* pfg = reinterpret_cast<const uint4*>(A.pf + (long long)(blk + 1) * kBlk * 16);
                const uint4* xvg = reinterpret_cast<const uint4*>(A.xv + (long long)(blk + 1) * (kBlk / 32) * 512);
                const uint4* xsg = reinterpret_cast<const uint4*>(A.Xs) + (long long)(blk + 1) * kBlk;
                n0 = pfg[threadIdx.x];
                n1 = pfg[kB16Threads + threadIdx.x];
                n2 = xvg[threadIdx.x];
                n3 = xvg[kB16Threads + threadIdx.x];
                n4 = (long long)(blk + 1) * kBlk + threadIdx.x < n ? xsg[threadIdx.x] : uint4{};
            }
            const float* gm = A.geom + (long long)blk * kGeomStride;
            float st[R][D], eps[R];
            bf16x8 sfrag[R];
#pragma unroll
            for (int g = 0; g < R; ++g) {
                float ns = 0.0f;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    st[g][k] = shat[g][k] - gm[k];
                    ns = fmaf(st[g][k], st[g][k], ns);
                }
                const float rr = gm[4] + sqrtf(ns);
                eps[g] = A.kappa * rr * rr;
                sfrag[g] = seed_frag<D>(st[g], ns, hf);
            }
            f32x16 out[R];
            bool used[R];
#pragma unroll
            for (int g = 0; g < R; ++g) {
                out[g] = f32x16{};
                used[g] = false;
            }
#pragma unroll 1
            for (int tt = 0; tt < kBlk / 32; ++tt) {
                const bf16x8 afrag = *reinterpret_cast<const bf16x8*>(spf + tt * 512 + hf * 256 + col * 8);
                // both groups' products first, so that one hides the other's latency
                f32x16 E[R];
                float emax[R];
#pragma unroll
                for (int g = 0; g < R; ++g)
                    E[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afrag, sfrag[g], f32x16{}, 0, 0, 0);
#pragma unroll
                for (int g = 0; g < R; ++g) {
                    // tree of maxima (depth 3 instead of a chain of 8)
                    const float m0 = fmaxf(fmaxf(E[g][0], E[g][1]), E[g][2]);
                    const float m1 = fmaxf(fmaxf(E[g][3], E[g][4]), E[g][5]);
                    const float m2 = fmaxf(fmaxf(E[g][6], E[g][7]), E[g][8]);
                    const float m3 = fmaxf(fmaxf(E[g][9], E[g][10]), E[g][11]);
                    const float m4 = fmaxf(fmaxf(E[g][12], E[g][13]), E[g][14]);
                    emax[g] = fmaxf(fmaxf(fmaxf(m0, m1), m2), fmaxf(fmaxf(m3, m4), E[g][15]));
                }
#pragma unroll
                for (int g = 0; g < R; ++g) {
                    const bool ref = __ballot(emax[g] + eps[g] >= A.e_thr);
                    if (ref) {
                        // some pair of this 32 x 32 tile may lie within the refine
                        // radius: every row of the lane is recomputed exactly in
                        // FP32 (points from LDS), and each pair keeps the exact
                        // weight if and only if its own bound flags it (its
                        // estimate is then replaced by -inf, weight 0 in the bf16
                        // sums), so the result of a pair never depends on its
                        // tile mates
                        const float4* xr = sxs + tt * 32 + 4 * hf;
                        unsigned nref = 0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            float4 x4[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) x4[u] = xr[8 * q + u];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int v = 4 * q + u;
                                const bool need = E[g][v] + eps[g] >= A.e_thr;
                                const float xv[4] = {x4[u].x, x4[u].y, x4[u].z, x4[u].w};
                                float dx[D], q2 = 0.0f;
#pragma unroll
                                for (int k = 0; k < D; ++k) {
                                    dx[k] = xv[k] - shat[g][k];
                                    q2 = fmaf(dx[k], dx[k], q2);
                                }
                                float we = kGauss ? __builtin_amdgcn_exp2f(-q2)
                                                  : (q2 <= a.h2 ? 1.0f : 0.0f);
                                we = need ? we : 0.0f;
                                wex[g] += we;
#pragma unroll
                                for (int k = 0; k < D; ++k) aex[g][k] = fmaf(we, dx[k], aex[g][k]);
                                nref += need ? 1u : 0u;
                                E[g][v] = need ? -__builtin_inff() : E[g][v];
                            }
                        }
                        refined += live[g] ? nref : 0u;
                    }
                    // far pairs (Gaussian only): weights from the estimate, unless
                    // every weight of the wave underflows (2^-127)
                    if (kGauss && (ref || __ballot(emax[g] >= -127.0f))) {
                        bf16x8 w0, w1;
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            w0[q] = (__bf16)__builtin_amdgcn_exp2f(E[g][q]);
                            w1[q] = (__bf16)__builtin_amdgcn_exp2f(E[g][8 + q]);
                        }
                        bf16x8 x0 = {}, x1 = {};
                        if (col < NCOL) {
                            x0 = *reinterpret_cast<const bf16x8*>(sxv + tt * 512 + ((0 * 2 + hf) * 16 + col) * 8);
                            x1 = *reinterpret_cast<const bf16x8*>(sxv + tt * 512 + ((1 * 2 + hf) * 16 + col) * 8);
                        }
                        out[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, x0, out[g], 0, 0, 0);
                        out[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, x1, out[g], 0, 0, 0);
                        used[g] = true;
                    }
                }
            }
            // ---- out[seed row][col] -> per-seed sums through a wave-local
            // transpose (LDS operations of one wave complete in order)
#pragma unroll
            for (int g = 0; g < R; ++g) {
                if (!__ballot(used[g])) continue;
                if (col < NCOL) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) tr[wave][col][8 * (v >> 2) + 4 * hf + (v & 3)] = out[g][v];
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                const float Wb = tr[wave][2 * D][col];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float sx = tr[wave][k][col] + tr[wave][D + k][col];
                    // sum w (x~ - s~) = sum w (x - s): the block centre cancels
                    arun[g][k] += sx - st[g][k] * Wb;
                }
                wrun[g] += Wb;
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }

        // ---- chunk partials (one (D+1)-vector per seed): the two lane halves
        // saw different points of the same seed
#pragma unroll
        for (int g = 0; g < R; ++g) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                aex[g][k] += __shfl_xor(aex[g][k], 32);
                arun[g][k] += aex[g][k];
            }
            wex[g] += __shfl_xor(wex[g], 32);
            wrun[g] += wex[g];
        }
        if (chunks == 1) {
            if (hf == 0) {
#pragma unroll
                for (int g = 0; g < R; ++g) {
                    const int pos = (wave * R + g) * 32 + col;
#pragma unroll
                    for (int k = 0; k < D; ++k) fin[k * TS + pos] = arun[g][k];
                    fin[D * TS + pos] = wrun[g];
                }
            }
            __syncthreads();
            finalize_tile<D, 4, R * 2>(a, t, m, tile, fin);
            __syncthreads();
        } else if (hf == 0) {
#pragma unroll
            for (int g = 0; g < R; ++g) {
                const int pos = (wave * R + g) * 32 + col;
                float* dst = a.part + (((long long)tile * chunks + chunk) * TS + pos) * (D + 1);
#pragma unroll
                for (int k = 0; k < D; ++k) dst[k] = arun[g][k];
                dst[D] = wrun[g];
            }
        }
    }
    // refined pairs: lane counts summed per wave, one atomic per wave
    for (int off = 32; off >= 1; off >>= 1) refined += __shfl_xor(refined, off);
    if (lane == 0 && refined)
        atomicAdd((unsigned long long*)&ctl->refined, (unsigned long long)refined);
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
    return launch_finalize<D, 4, 2 * R>(a, t, b.grid, b.n_seeds, s);
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
    // 4 waves x R groups of 32 seeds.  Two groups share each staged block and
    // pay off for mid-sized batches; one group needs fewer registers (4 waves
    // per SIMD instead of 2), which wins for small and for large batches.
    const int groups = (B >= 2 * kB16Seeds && B <= 1024) ? 2 : 1;
    sh.R = 2 * groups;     // the finalize geometry: TS = 64 * R
    sh.TS = kB16Seeds * groups;
    return sh;
}

bool bf16_supported(int d) { return d >= 1 && (d <= 4 || (d <= 32 && bf16w_dims(step_shape(d).D))); }

hipError_t launch_iteration_bf16(Batch& b, int t, hipStream_t s) {
    if (b.sh.D > 4) return launch_iteration_bf16w(b, t, s);
    const bool two = b.sh.TS == 2 * kB16Seeds;
    switch (b.sh.D) {
        case 1: return two ? launch_bf16_t<1, 2>(b, t, s) : launch_bf16_t<1, 1>(b, t, s);
        case 2: return two ? launch_bf16_t<2, 2>(b, t, s) : launch_bf16_t<2, 1>(b, t, s);
        case 3: return two ? launch_bf16_t<3, 2>(b, t, s) : launch_bf16_t<3, 1>(b, t, s);
        case 4: return two ? launch_bf16_t<4, 2>(b, t, s) : launch_bf16_t<4, 1>(b, t, s);
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
