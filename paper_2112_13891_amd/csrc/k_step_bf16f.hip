// k_step_bf16f.hip -- the fused mean-shift iteration in the BF16 form for the
// Gaussian kernel at 8 <= D <= 32 (gfx950), in the style of flash attention:
// the seed-point products on MFMA in bf16 with FP32 accumulation, the
// weights made in registers, and W.X accumulated on MFMA in FP32.
//
// Points are sorted by nearest pivot and shifted by the bounding-box
// midpoint.  Each block of 256 of them is centred on c, the coordinate-wise
// median of its points (robust to the few far points that end a pivot run),
// and for a seed s (packed units, where w = exp2(-|x - s|^2)) both sides are
// taken relative to it: x~ = x - c, s~ = s - c, and
//     E = 2 x~.s~ - |x~|^2 - |s~|^2  (= -|x - s|^2),
// each operand split into three bf16 parts (x~ = hi + mid + lo leaves a
// relative error of u^3, u = 2^-8), with K slots
// [x~ | -|x~|^2 hi, mid, lo | 0..] against [2 s~ | 1 | 1 | 1 | 0..] and
// -|s~|^2 (FP32) as the accumulator's start value.  The error of E for a
// pair grows with (|x~| + |s~|)^2, so a point farther than kInlierR from its
// block's centre is an outlier of the block (a bit per point); R is the
// radius of all the block's points, Rin that of the others.  Per block:
//   1. cull: a seed whose distance bound |s~| - R puts every pair of the
//      block beyond the FP32 underflow of the weight (2^-127) has nothing
//      there; the workgroup skips a block no seed of it can see;
//   2. screen: one product of the hi parts, whose error is at most
//      eps = 2 (2u + u^2) R |s~| + 2^-14 (R + |s~|)^2 (Cauchy-Schwarz on the
//      rounded products, plus the rounding of the norm and of the FP32
//      accumulation); a 32 x 32 tile whose every E + eps < -127 has weights
//      exactly 0 in FP32 and is skipped;
//   3. a live tile completes E with the products hi.mid, mid.hi, hi.lo,
//      lo.hi and mid.mid, whose remaining error is of order u^3 R |s~| plus
//      the FP32 accumulation of terms of size (R + |s~|)^2;
//   4. pairs for which that is not accurate enough are computed in FP32 by
//      direct differences (distance, weight and w (x - s), as the FP32 step
//      does): an outlier point whose compensated E, with its own small bound,
//      can still give a nonzero weight; and every point of the block for a
//      seed with (Rin + |s~|)^2 > 64 that can still have a weight of 2^-9 or
//      more there.  (The MFMA aligns the products of an output to its
//      largest term and truncates a few bits below that term's ulp: an
//      outlier's large x~ in W.X~, or |E|-sized partial sums, would swamp
//      the small products; the compensation products and each tile's W.X~
//      therefore start from a zero accumulator and are added in FP32);
//   5. the other weights w = exp2(E) are made in registers, split into three
//      bf16 parts, and W.X~ accumulates as the six products of order up to
//      u^2 on MFMA, the weight sum alongside in FP32;
//   6. the block centre comes back per block: sum w (x - s) =
//      sum w x~ - (s - c) sum w.
// Every decision is per pair or per seed, or skips pairs whose weight is
// exactly 0, so a seed's result never depends on the other seeds of its wave.
// MFMA layouts (v_mfma_f32_32x32x16_bf16): A lane l holds row l%32 and
// k = 8 (l/32) .. + 8; B lane l holds k = 8 (l/32) .. + 8 and column l%32; the
// accumulator lane l holds column l%32 and rows 8 (v/4) + 4 (l/32) + v%4.
// For W.X the weights of a lane (its column's seed, its 16 rows) are the A
// operand as they stand; the point order of K follows that register order.

#include "step_common.h"

namespace fms {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kFThreads = 256;   // 4 waves x 32 seeds
constexpr int kFSeeds = 128;     // seeds per tile
constexpr int kFBlk = 256;       // points per block
constexpr float kPadNorm = -1e30f;   // padding points: finite, weight 0
// Points farther than this (packed units) from their block's centre are the
// block's outliers: their pairs are recomputed exactly when they can matter.
constexpr float kInlierR = 4.0f;
// (Rin + |s~|)^2 above which a seed's distances to a block are recomputed in
// FP32 (packed units), unless every weight it can have there is below
// 2^-(3^2): the expanded form's terms are then too large for its FP32
// accumulation
constexpr float kExpandedMax = 64.0f;
constexpr float kFarLower = 3.0f;

template <int D>
struct FShape {
    static constexpr int KBH = (D + 3 + 15) / 16;   // K steps of the hi operand (with the norm)
    static constexpr int KBL = (D + 15) / 16;       // K steps of the mid and lo operands
    static constexpr int HI_BYTES = (kFBlk / 32) * KBH * 512 * 2;   // per block
    static constexpr int LO_BYTES = (kFBlk / 32) * KBL * 512 * 2;   // each of mid and lo
    static constexpr int STAGE = HI_BYTES + 2 * LO_BYTES;
    static constexpr int FIN = (D + 1) * kFSeeds * 4;
    static constexpr int TR = 4 * 32 * 33 * 4;
    static constexpr int SMEM = STAGE > FIN ? (STAGE > TR ? STAGE : TR) : (FIN > TR ? FIN : TR);
    // per-block row of the centring: centre[D], R, Rin, Ro, the block's
    // first row and live count (int32 bit patterns), 3 unused, the outlier
    // bits of the 8 tiles (a uint32 each, bit p = point p of the tile), then
    // the outliers' own centre[D] (Ro < 0: no outliers)
    static constexpr int INFO = 2 * D + 16;
    static_assert(STAGE % (16 * kFThreads) == 0, "stage layout");
};

struct Bf16fArgs {
    StepArgs base;
    const float* info;     // per block: centre, R, Rin, Ro, outlier bits, outlier centre (FShape::INFO floats)
    const __bf16* fhi;     // [tile][kb][half][point][8]: x~hi | -|x~|^2 hi, mid, lo
    const __bf16* fmid;    // [tile][kb][half][point][8]: x~mid
    const __bf16* flo;     // [tile][kb][half][point][8]: x~lo
    const float* Xs;       // sorted, shifted points (n x D, packed units)
    const float* shift;    // frame shift (D floats)
};

__device__ __forceinline__ float bfr(float x) { return (float)(__bf16)x; }

// Centring and operands of the points, built once per fit from the sorted
// points, one workgroup per block: the block's median centre (per
// coordinate, the live point of rank (nl - 1) / 2, ties broken by index),
// its radii, the outlier bits, the outliers' own ball (bounding-box
// midpoint and radius: where two pivot runs meet, the block's other run) and
// the three bf16 parts.
// With boff set (many clouds), block b belongs to the cloud c with boff[c] <=
// b < boff[c + 1] and holds the sorted rows x_off[c] + 256 (b - boff[c]) ..,
// at most 256 and within the cloud; otherwise block b holds rows 256 b .. of
// the n.  The first row and the live count go into the info row.
template <int D>
__global__ __launch_bounds__(kFBlk) void bf16f_features_kernel(const float* __restrict__ Xs, int n,
                                                               __bf16* fhi, __bf16* fmid, __bf16* flo,
                                                               float* info, const long long* __restrict__ x_off,
                                                               const int32_t* __restrict__ boff, int ncl) {
    using Sh = FShape<D>;
    constexpr int kW = kFBlk / 64;
    __shared__ float srt[kW][64];   // each wave's values of one coordinate, ascending
    __shared__ float ctr[D];
    __shared__ float rmax[3][kFBlk / 64];
    __shared__ float omin[kFBlk / 64][D], omax[kFBlk / 64][D], oc[D];
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    long long row0 = (long long)blk * kFBlk, rend = n;
    if (boff) {
        const int c = upper_cloud(boff, ncl, blk);
        row0 = x_off[c] + (long long)(blk - boff[c]) * kFBlk;
        rend = x_off[c + 1];
    }
    const long long row = row0 + tid;                 // this thread's point
    const long long i = (long long)blk * kFBlk + tid;   // its slot in the operands
    const int nl = (int)min((long long)kFBlk, rend - row0);   // live points of the block (>= 1)
    const bool live = tid < nl;
    const int mid = (nl - 1) / 2;
    float x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = live ? Xs[row * D + k] : 0.0f;
    if (tid < D) ctr[tid] = Xs[row0 * D + tid];   // stands in if ranks tie oddly (NaN)
    // per coordinate, the value of rank mid among the live points (padding
    // lanes hold +inf and sort last): each wave sorts its 64 values by a
    // bitonic network over lane shuffles, and the value at position p of
    // wave w has rank p + (values of the earlier waves <= it) + (values of
    // the later waves < it) -- a permutation of 0..255, so exactly one lane
    // holds rank mid, and its value is the coordinate's median
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll 1
    for (int k = 0; k < D; ++k) {
        float v = live ? x[k] : __builtin_inff();
#pragma unroll
        for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const float y = __shfl_xor(v, j);
                const bool keep_min = ((lane & kk) == 0) == ((lane & j) == 0);
                v = keep_min ? fminf(v, y) : fmaxf(v, y);
            }
        }
        srt[wv][lane] = v;
        __syncthreads();
        int rank = lane;
#pragma unroll
        for (int w = 0; w < kW; ++w) {
            if (w == wv) continue;
            // values of wave w below v (w > wv) or not above v (w < wv)
            int lo = 0, hi = 64;
            while (lo < hi) {
                const int md = (lo + hi) >> 1;
                const float u = srt[w][md];
                if (w < wv ? (u <= v) : (u < v)) lo = md + 1;
                else hi = md;
            }
            rank += lo;
        }
        if (rank == mid) ctr[k] = v;
        __syncthreads();   // srt is rewritten for the next coordinate
    }
    float xt[D];
    float nx = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xt[k] = live ? x[k] - ctr[k] : 0.0f;
        nx = fmaf(xt[k], xt[k], nx);
    }
    const bool outl = live && nx > kInlierR * kInlierR;
    float ra = live ? nx : 0.0f, ri = (live && !outl) ? nx : 0.0f;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        ra = fmaxf(ra, __shfl_xor(ra, off));
        ri = fmaxf(ri, __shfl_xor(ri, off));
    }
    const unsigned long long om = __ballot(outl);
    const int wave = tid >> 6;
    // the outliers' bounding box, per wave, then over the waves
#pragma unroll 1
    for (int k = 0; k < D; ++k) {
        float lo = outl ? x[k] : __builtin_inff(), hi = outl ? x[k] : -__builtin_inff();
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            lo = fminf(lo, __shfl_xor(lo, off));
            hi = fmaxf(hi, __shfl_xor(hi, off));
        }
        if ((tid & 63) == 0) {
            omin[wave][k] = lo;
            omax[wave][k] = hi;
        }
    }
    __syncthreads();
    if (tid < D) {
        float lo = omin[0][tid], hi = omax[0][tid];
        for (int w = 1; w < kFBlk / 64; ++w) {
            lo = fminf(lo, omin[w][tid]);
            hi = fmaxf(hi, omax[w][tid]);
        }
        oc[tid] = lo <= hi ? 0.5f * (lo + hi) : 0.0f;
    }
    __syncthreads();
    float ro = -1.0f;
    if (outl) {
        ro = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float t = x[k] - oc[k];
            ro = fmaf(t, t, ro);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ro = fmaxf(ro, __shfl_xor(ro, off));
    float* g = info + (long long)blk * Sh::INFO;
    if ((tid & 63) == 0) {
        rmax[0][wave] = ra;
        rmax[1][wave] = ri;
        rmax[2][wave] = ro;
        // tile 2 wave + h holds points 64 wave + 32 h ..: the ballot's halves
        unsigned* bits = reinterpret_cast<unsigned*>(g + D + 8);
        bits[2 * wave] = (unsigned)om;
        bits[2 * wave + 1] = (unsigned)(om >> 32);
    }
    __syncthreads();
    if (tid < D) {
        g[tid] = ctr[tid];
        g[D + 16 + tid] = oc[tid];
    }
    if (tid == 0) {
        g[D + 3] = __int_as_float((int)row0);
        g[D + 4] = __int_as_float(nl);
        float a = 0.0f, b = 0.0f, c = -1.0f;
        for (int w = 0; w < kFBlk / 64; ++w) {
            a = fmaxf(a, rmax[0][w]);
            b = fmaxf(b, rmax[1][w]);
            c = fmaxf(c, rmax[2][w]);
        }
        // rounded up slightly, so that they bound the FP32 distances
        g[D] = sqrtf(a) * 1.0001f + 1e-30f;
        g[D + 1] = sqrtf(b) * 1.0001f + 1e-30f;
        g[D + 2] = c < 0.0f ? -1.0f : sqrtf(c) * 1.0001f + 1e-30f;
    }
    const float ph = live ? bfr(-nx) : kPadNorm;
    const float pm = live ? bfr(-nx - ph) : 0.0f;
    const float pl = live ? bfr((-nx - ph) - pm) : 0.0f;
    __bf16* oh = fhi + (long long)(i >> 5) * (Sh::KBH * 512) + (i & 31) * 8;
#pragma unroll
    for (int s = 0; s < Sh::KBH * 16; ++s) {
        float v = 0.0f;
        if (s < D) v = bfr(xt[s]);
        else if (s == D) v = ph;
        else if (s == D + 1) v = pm;
        else if (s == D + 2) v = pl;
        oh[(s >> 4) * 512 + ((s >> 3) & 1) * 256 + (s & 7)] = (__bf16)v;
    }
    __bf16* om2 = fmid + (long long)(i >> 5) * (Sh::KBL * 512) + (i & 31) * 8;
    __bf16* ol = flo + (long long)(i >> 5) * (Sh::KBL * 512) + (i & 31) * 8;
#pragma unroll
    for (int s = 0; s < Sh::KBL * 16; ++s) {
        float vm = 0.0f, vl = 0.0f;
        if (s < D) {
            const float h = bfr(xt[s]);
            vm = bfr(xt[s] - h);
            vl = bfr((xt[s] - h) - vm);
        }
        const int o = (s >> 4) * 512 + ((s >> 3) & 1) * 256 + (s & 7);
        om2[o] = (__bf16)vm;
        ol[o] = (__bf16)vl;
    }
}

// One bf16 of coordinate c of staged point p (tile tt) from an operand stored
// [tile][kb][half][point][8] with `kbs` K steps per tile.
__device__ __forceinline__ __bf16 staged_coord(const __bf16* base, int kbs, int tt, int p, int c) {
    return base[((tt * kbs + (c >> 4)) * 2 + ((c >> 3) & 1)) * 256 + p * 8 + (c & 7)];
}

// The step kernel, in two launch forms.  One cloud (MANY = false): the work
// items (seed tile of 128, chunk of the blocks) of the iteration's active
// list, in a grid-stride loop, a chunk's partials finalized in place when the
// tile has one chunk.  Many clouds (MANY = true): a persistent grid over the
// work items (cloud, seed tile of 128, chunk of the cloud's blocks) of the
// batched plan, taken as the FP32 batched step takes them (from the queue
// when they outnumber the workgroups), each storing one partial per seed,
// component-major within the item, for the batched finalize.  Either way a
// lane holds one seed (the two halves of a wave the same 32 seeds, each half
// its own points of every tile).
// Many clouds at D <= 16: three waves per SIMD (168 VGPRs, some spilled):
// the batched workload's clusters lie within the weights' reach, so about
// half of the tiles pass the screen and the kernel waits on latency more
// than it computes (2.43 -> 2.15 ms per iteration on 512 uneven clouds at
// D = 16).  Four waves spill too much.
template <int D, bool MANY>
__global__ __launch_bounds__(kFThreads, (MANY && D <= 16) ? 3 : 2) void step_bf16f_kernel(Bf16fArgs A, int t,
                                                                                        BatchedArgs B) {
    using Sh = FShape<D>;
    constexpr int TS = kFSeeds;
    constexpr int KBH = Sh::KBH, KBL = Sh::KBL;
    const StepArgs& a = A.base;
    Ctl* ctl = a.ctl;
    int m = 0, tiles = 1, chunks = 1, nblk = 0, total = 0;
    if constexpr (MANY) {
        total = B.item_pre[B.ncl];
    } else {
        m = active_count(ctl, t);
        step_prologue(a, t, m);
        if (m == 0) return;
        tiles = (m + TS - 1) / TS;
        chunks = chunks_for(m, TS, a.n, gridDim.x, a.min_chunk);
        nblk = (a.n + kFBlk - 1) / kFBlk;
        total = tiles * chunks;
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int col = lane & 31, hf = lane >> 5;

    __shared__ __attribute__((aligned(16))) char smem[Sh::SMEM];
    __shared__ int next_item;
    const __bf16* shi = reinterpret_cast<const __bf16*>(smem);
    const __bf16* smid = reinterpret_cast<const __bf16*>(smem + Sh::HI_BYTES);
    const __bf16* slo = reinterpret_cast<const __bf16*>(smem + Sh::HI_BYTES + Sh::LO_BYTES);
    unsigned long long live_pairs = 0;   // wave-uniform: pairs of the live tiles

    // many clouds: with no more items than workgroups each takes its own;
    // otherwise every item comes from the queue (every thread has read the
    // previous item -- the transposition below holds barriers -- before
    // thread 0 writes the next one)
    const bool own = !MANY || total <= (int)gridDim.x;
    int item = blockIdx.x;
    if (!own) {
        if (threadIdx.x == 0) next_item = atomicAdd(B.queue, 1);
        __syncthreads();
        item = __builtin_amdgcn_readfirstlane(next_item);
    }
    const const_f32_ptr gq = wave_uniform_const(A.info);   // block centring: scalar loads
    while (item < total) {
        int tile, chunk, b0, b1, slot0;
        if constexpr (MANY) {
            const int c = __builtin_amdgcn_readfirstlane(B.item_cloud[item]);
            const int local = item - B.item_pre[c];
            tiles = B.tiles[c];
            chunks = B.chunks[c];
            tile = local % tiles;
            chunk = local / tiles;
            const int bc = B.boff[c];
            const int nb = B.boff[c + 1] - bc;
            b0 = __builtin_amdgcn_readfirstlane(bc + (int)((long long)nb * chunk / chunks));
            b1 = __builtin_amdgcn_readfirstlane(bc + (int)((long long)nb * (chunk + 1) / chunks));
            m = B.slot_pre[c + 1] - B.slot_pre[c];
            slot0 = B.seg[c];
        } else {
            tile = item % tiles;
            chunk = item / tiles;
            b0 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * chunk / chunks));
            b1 = __builtin_amdgcn_readfirstlane((int)((long long)nblk * (chunk + 1) / chunks));
            slot0 = 0;
        }
        const int slot = tile * TS + wave * 32 + col;
        const bool live = slot < m;
        const unsigned long long lmask = __ballot(live);   // lanes holding a seed
        const int j = a.act_in[slot0 + (live ? slot : 0)];
        float shat[D], aex[D];
        float wsum = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            shat[k] = a.S[(long long)j * D + k] * a.scale - A.shift[k];
            aex[k] = 0.0f;
        }
        f32x16 acc = f32x16{};   // sum of w x~ over the chunk: column = coordinate, rows = seeds

        for (int blk = b0; blk < b1; ++blk) {
            const const_f32_ptr gm = gq + (long long)blk * Sh::INFO;
            const float R = gm[D];
            const float Rin = gm[D + 1];
            float st[D];
            float ns = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                st[k] = shat[k] - gm[k];
                ns = fmaf(st[k], st[k], ns);
            }
            const float dist = sqrtf(ns);
            const float eps = 0.016f * R * dist + (1.0f / 16384.0f) * (R + dist) * (R + dist);
            // 1. no pair of the block can reach the screen: E + eps >= -127
            //    needs |x - s|^2 <= 127 + 2 eps, and |x - s| >= |s~| - Rin for
            //    the inliers, |s - co| - Ro for the outliers
            const float reach = (127.0f + 2.0f * eps) * 1.001f + 1e-6f;
            const float li = dist * (1.0f - 1e-5f) - Rin;
            bool maybe = !(li > 0.0f && li * li > reach);
            const float Ro = gm[D + 2];
            if (!maybe && Ro >= 0.0f) {
                float no = 0.0f;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float u = shat[k] - gm[D + 16 + k];
                    no = fmaf(u, u, no);
                }
                const float lo = sqrtf(no) * (1.0f - 1e-5f) - Ro;
                maybe = !(lo > 0.0f && lo * lo > reach);
            }
            maybe = maybe && live;
            if (!__syncthreads_or(maybe)) continue;   // (also: the previous block's stage is free)
            constexpr int NH = Sh::HI_BYTES / 16, NL = Sh::LO_BYTES / 16;
            // the hi operand first: the screen needs nothing else
            {
                const uint4* gh = reinterpret_cast<const uint4*>(A.fhi + (long long)blk * (Sh::HI_BYTES / 2));
                uint4* sm = reinterpret_cast<uint4*>(smem);
                uint4 v[NH / kFThreads];
#pragma unroll
                for (int q = 0; q < NH / kFThreads; ++q) v[q] = gh[q * kFThreads + threadIdx.x];
#pragma unroll
                for (int q = 0; q < NH / kFThreads; ++q) sm[q * kFThreads + threadIdx.x] = v[q];
            }
            __syncthreads();
            // seed operands of this block: [2 s~hi | 1 | 1 | 1 | 0..], [2 s~mid | 0..], [2 s~lo | 0..]
            bf16x8 bh[KBH], bm[KBL], bl[KBL];
            unsigned tmask = 0u;   // this wave's tiles that pass the screen
            if (__ballot(maybe)) {
#pragma unroll
                for (int kb = 0; kb < KBH; ++kb) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        // the slot for hf = 0 is s0, for hf = 1 it is s0 + 8
                        const int s0 = kb * 16 + e, s1 = s0 + 8;
                        const float c0 = s0 < D ? 2.0f * st[s0 < D ? s0 : 0] : 0.0f;
                        const float c1 = s1 < D ? 2.0f * st[s1 < D ? s1 : 0] : 0.0f;
                        const float one0 = (s0 >= D && s0 <= D + 2) ? 1.0f : 0.0f;
                        const float one1 = (s1 >= D && s1 <= D + 2) ? 1.0f : 0.0f;
                        const float c = hf ? c1 : c0;
                        const float vh = bfr(c);
                        const float vm = bfr(c - vh);
                        bh[kb][e] = (__bf16)(vh + (hf ? one1 : one0));
                        if (kb < KBL) {
                            bm[kb][e] = (__bf16)vm;
                            bl[kb][e] = (__bf16)bfr((c - vh) - vm);
                        }
                    }
                }
                // 2. the screen, on the hi products alone: a 32 x 32 tile whose
                //    every E + eps < -127 has weights exactly 0 in FP32
#pragma unroll 1
                for (int tt = 0; tt < kFBlk / 32; ++tt) {
                    f32x16 E;
#pragma unroll
                    for (int v = 0; v < 16; ++v) E[v] = -ns;
#pragma unroll
                    for (int kb = 0; kb < KBH; ++kb) {
                        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(shi + (tt * KBH + kb) * 512 + hf * 256 + col * 8);
                        E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[kb], E, 0, 0, 0);
                    }
                    const float m0 = fmaxf(fmaxf(E[0], E[1]), E[2]);
                    const float m1 = fmaxf(fmaxf(E[3], E[4]), E[5]);
                    const float m2 = fmaxf(fmaxf(E[6], E[7]), E[8]);
                    const float m3 = fmaxf(fmaxf(E[9], E[10]), E[11]);
                    const float m4 = fmaxf(fmaxf(E[12], E[13]), E[14]);
                    const float emax = fmaxf(fmaxf(fmaxf(m0, m1), m2), fmaxf(fmaxf(m3, m4), E[15]));
                    if (__ballot(live && emax + eps >= -127.0f)) tmask |= 1u << tt;
                }
            }
            // the mid and lo operands only for a block with a tile that passed
            // (a block no wave needs further ends here: its weights are all 0)
            if (!__syncthreads_or(tmask != 0u)) continue;
            {
                const uint4* gm2 = reinterpret_cast<const uint4*>(A.fmid + (long long)blk * (Sh::LO_BYTES / 2));
                const uint4* gl = reinterpret_cast<const uint4*>(A.flo + (long long)blk * (Sh::LO_BYTES / 2));
                uint4* sm = reinterpret_cast<uint4*>(smem);
                uint4 v[2 * NL / kFThreads];
#pragma unroll
                for (int q = 0; q < 2 * NL / kFThreads; ++q) {
                    const int f = q * kFThreads + threadIdx.x;
                    v[q] = f < NL ? gm2[f] : gl[f - NL];
                }
#pragma unroll
                for (int q = 0; q < 2 * NL / kFThreads; ++q) sm[NH + q * kFThreads + threadIdx.x] = v[q];
            }
            __syncthreads();
            if (tmask != 0u) {
                // the expanded form's terms are too large for its FP32
                // accumulation and the weights can be sizeable: this seed's
                // distances to the block are recomputed exactly
                const bool exact_seed = live && (Rin + dist) * (Rin + dist) > kExpandedMax &&
                                        dist * (1.0f - 1e-5f) - Rin < kFarLower;
                // the compensated E's bound for the outliers (R their radius)
                const float eps3 = 1.2e-6f * R * dist + 1e-6f * (R + dist) * (R + dist);
                float wb = 0.0f;   // this lane's weight sum over the block
                unsigned long long nlive = 0;
#pragma unroll 1
                for (int tt = 0; tt < kFBlk / 32; ++tt) {
                    if (!((tmask >> tt) & 1u)) continue;
                    // the hi products again (the same values as the screen's)
                    f32x16 E;
#pragma unroll
                    for (int v = 0; v < 16; ++v) E[v] = -ns;
#pragma unroll
                    for (int kb = 0; kb < KBH; ++kb) {
                        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(shi + (tt * KBH + kb) * 512 + hf * 256 + col * 8);
                        E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[kb], E, 0, 0, 0);
                    }
                    nlive += (unsigned long long)__popcll(lmask) * 16;
                    // 3. the compensated products, in an accumulator of their
                    //    own (their sizes are u and u^2 of the hi products)
                    {
                        f32x16 Ec = f32x16{};
#pragma unroll
                        for (int kb = 0; kb < KBL; ++kb) {
                            const int o = (tt * KBL + kb) * 512 + hf * 256 + col * 8;
                            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(shi + (tt * KBH + kb) * 512 + hf * 256 + col * 8);
                            const bf16x8 am = *reinterpret_cast<const bf16x8*>(smid + o);
                            const bf16x8 al = *reinterpret_cast<const bf16x8*>(slo + o);
                            Ec = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm[kb], Ec, 0, 0, 0);
                            Ec = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh[kb], Ec, 0, 0, 0);
                            Ec = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[kb], Ec, 0, 0, 0);
                            Ec = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[kb], Ec, 0, 0, 0);
                            Ec = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm[kb], Ec, 0, 0, 0);
                        }
#pragma unroll
                        for (int v = 0; v < 16; ++v) E[v] += Ec[v];
                    }
                    // 4. the pairs that are computed in FP32 by direct
                    //    differences, as the FP32 step does: distance, weight,
                    //    and w (x - s) into the seed's own sums; the MFMA sees
                    //    weight 0 for them (its products would be truncated
                    //    against the large x~ of an outlier)
                    const unsigned obits = __float_as_uint(gm[D + 8 + tt]);
                    if (obits != 0u || __ballot(exact_seed)) {
                        // the block's first row and live count
                        const long long r0 = (long long)__float_as_int(gm[D + 3]) + tt * 32;
                        const int nl = __float_as_int(gm[D + 4]) - tt * 32;
                        // pair v of this lane in FP32 (every lane of the wave
                        // calls it for the same v)
                        auto exact_pair = [&](int v, bool need) {
                            const int p = 8 * (v >> 2) + 4 * hf + (v & 3);
                            if (need && p < nl) {
                                const float4* xr = reinterpret_cast<const float4*>(A.Xs + (r0 + p) * D);
                                float q2 = 0.0f;
#pragma unroll
                                for (int k4 = 0; k4 < D; k4 += 4) {
                                    const float4 x4 = xr[k4 / 4];
                                    const float d0 = x4.x - shat[k4], d1 = x4.y - shat[k4 + 1];
                                    const float d2 = x4.z - shat[k4 + 2], d3 = x4.w - shat[k4 + 3];
                                    q2 = fmaf(d0, d0, q2);
                                    q2 = fmaf(d1, d1, q2);
                                    q2 = fmaf(d2, d2, q2);
                                    q2 = fmaf(d3, d3, q2);
                                }
                                const float we = __builtin_amdgcn_exp2f(-q2);
                                wsum += we;
#pragma unroll
                                for (int k4 = 0; k4 < D; k4 += 4) {
                                    const float4 x4 = xr[k4 / 4];
                                    aex[k4] = fmaf(we, x4.x - shat[k4], aex[k4]);
                                    aex[k4 + 1] = fmaf(we, x4.y - shat[k4 + 1], aex[k4 + 1]);
                                    aex[k4 + 2] = fmaf(we, x4.z - shat[k4 + 2], aex[k4 + 2]);
                                    aex[k4 + 3] = fmaf(we, x4.w - shat[k4 + 3], aex[k4 + 3]);
                                }
                            }
                            if (need) E[v] = kPadNorm;
                        };
                        auto needs = [&](int v) {
                            const int p = 8 * (v >> 2) + 4 * hf + (v & 3);
                            return exact_seed || (live && ((obits >> p) & 1u) && E[v] + eps3 >= -127.0f);
                        };
                        if constexpr (D <= 16) {
                            // this lane's pairs first, then one ballot for the
                            // common case of none in the wave
                            unsigned nm = 0u;
#pragma unroll
                            for (int v = 0; v < 16; ++v)
                                if (needs(v)) nm |= 1u << v;
                            if (__ballot(nm != 0u)) {
#pragma unroll
                                for (int v = 0; v < 16; ++v) {
                                    const bool need = (nm >> v) & 1u;
                                    if (__ballot(need)) exact_pair(v, need);
                                }
                            }
                        } else {
                            // (at D = 32 the mask costs more registers than it saves)
#pragma unroll
                            for (int v = 0; v < 16; ++v) {
                                const bool need = needs(v);
                                if (__ballot(need)) exact_pair(v, need);
                            }
                        }
                    }
                    // 5. weights and W.X~
                    bf16x8 wh[2], wm[2], wl[2];
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const float w = live ? __builtin_amdgcn_exp2f(E[v]) : 0.0f;
                        const float h = bfr(w);
                        const float mm = bfr(w - h);
                        const float l = bfr((w - h) - mm);
                        wb += w;
                        wh[v >> 3][v & 7] = (__bf16)h;
                        wm[v >> 3][v & 7] = (__bf16)mm;
                        wl[v >> 3][v & 7] = (__bf16)l;
                    }
                    // the tile's W.X~ in a fresh accumulator, added to the
                    // chunk's sums in FP32 (the MFMA would truncate the
                    // tile's products against the running sums)
                    f32x16 tw = f32x16{};
#pragma unroll
                    for (int ks = 0; ks < 2; ++ks) {
                        // this lane's column c = col of X~: the 8 points of K step ks
                        // w x~ = (wh + wm + wl)(xh + xm + xl) to a relative
                        // u^3: the six products of order up to u^2
                        bf16x8 xh, xm, xl;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int p = 16 * ks + 8 * (e >> 2) + 4 * hf + (e & 3);
                            xh[e] = col < D ? staged_coord(shi, KBH, tt, p, col) : (__bf16)0.0f;
                            xm[e] = col < D ? staged_coord(smid, KBL, tt, p, col) : (__bf16)0.0f;
                            xl[e] = col < D ? staged_coord(slo, KBL, tt, p, col) : (__bf16)0.0f;
                        }
                        tw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh[ks], xh, tw, 0, 0, 0);
                        tw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh[ks], xm, tw, 0, 0, 0);
                        tw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wm[ks], xh, tw, 0, 0, 0);
                        tw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh[ks], xl, tw, 0, 0, 0);
                        tw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl[ks], xh, tw, 0, 0, 0);
                        tw = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wm[ks], xm, tw, 0, 0, 0);
                    }
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[v] += tw[v];
                }
                // 6. sum w (x - s) = sum w x~ - (s - c) sum w, this block's part
                // (s~ recomputed from the scalar geometry row: not kept live
                // through the tiles)
#pragma unroll
                for (int k = 0; k < D; ++k) aex[k] = fmaf(-wb, shat[k] - gm[k], aex[k]);
                wsum += wb;
                live_pairs += nlive;
            }
        }

        // the chunk's sum w x~ (column = coordinate, rows = seeds) into the
        // seed lanes through LDS; the two lane halves saw different points
        __syncthreads();   // the stage is free
        float* tr = reinterpret_cast<float*>(smem) + wave * 32 * 33;
#pragma unroll
        for (int v = 0; v < 16; ++v) tr[(8 * (v >> 2) + 4 * hf + (v & 3)) * 33 + col] = acc[v];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < D; ++k) aex[k] += __shfl_xor(aex[k], 32);
        wsum += __shfl_xor(wsum, 32);
#pragma unroll
        for (int k = 0; k < D; ++k) aex[k] += tr[col * 33 + k];
        __syncthreads();   // tr is read before smem is reused
        const int pos = wave * 32 + col;
        if constexpr (MANY) {
            if (hf == 0) {
                float* dst = a.part + (long long)item * TS * (D + 1) + pos;
#pragma unroll
                for (int k = 0; k < D; ++k) dst[k * TS] = aex[k];
                dst[D * TS] = wsum;
            }
            if (own) break;
            if (threadIdx.x == 0) next_item = atomicAdd(B.queue, 1);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(next_item);
        } else {
            if (chunks == 1) {
                float* fin = reinterpret_cast<float*>(smem);
                if (hf == 0) {
#pragma unroll
                    for (int k = 0; k < D; ++k) fin[k * TS + pos] = aex[k];
                    fin[D * TS + pos] = wsum;
                }
                __syncthreads();
                finalize_tile<D, D, 2>(a, t, m, tile, fin);
                __syncthreads();
            } else if (hf == 0) {
                float* dst = a.part + (((long long)tile * chunks + chunk) * TS + pos) * (D + 1);
#pragma unroll
                for (int k = 0; k < D; ++k) dst[k] = aex[k];
                dst[D] = wsum;
            }
            item += gridDim.x;
        }
    }
    if constexpr (!MANY) {
        // pairs of the live tiles: wave counts summed per workgroup, one
        // atomic per workgroup on one of the spread counters
        __shared__ unsigned long long wref[kWaves];
        if (lane == 0) wref[threadIdx.x >> 6] = live_pairs;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long r = 0;
            for (int w = 0; w < kWaves; ++w) r += wref[w];
            if (r) atomicAdd((unsigned long long*)&ctl->refined[(blockIdx.x % kRefinedSlots) * kRefinedStride], r);
        }
    }
}

template <int D>
hipError_t launch_bf16f_t(Batch& b, int t, hipStream_t s) {
    using Sh = FShape<D>;
    Bf16fArgs A;
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
    const int npad = (b.n + kFBlk - 1) / kFBlk * kFBlk;
    A.fhi = (const __bf16*)b.pf;
    A.fmid = A.fhi + (size_t)npad / 32 * Sh::KBH * 512;
    A.flo = A.fmid + (size_t)npad / 32 * Sh::KBL * 512;
    A.info = reinterpret_cast<const float*>(A.flo + (size_t)npad / 32 * Sh::KBL * 512);
    A.Xs = b.Xs;
    A.shift = b.shift;
    hipLaunchKernelGGL((step_bf16f_kernel<D, false>), dim3(b.grid), dim3(kFThreads), 0, s, A, t, BatchedArgs{});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalize<D, D, 2>(a, t, b.grid, b.n_seeds, s);
}

template <int D>
size_t bf16f_bytes_blocks_t(long long blocks) {
    using Sh = FShape<D>;
    return (size_t)blocks * (kFBlk / 32) * (Sh::KBH + 2 * Sh::KBL) * 512 * 2 + (size_t)blocks * Sh::INFO * 4;
}

template <int D>
size_t bf16f_bytes_t(int n) {
    return bf16f_bytes_blocks_t<D>((n + kFBlk - 1) / kFBlk);
}

template <int D>
void bf16f_operands(Bf16fArgs& A, const void* feat, long long nblk) {
    using Sh = FShape<D>;
    const size_t npad = (size_t)nblk * kFBlk;
    A.fhi = (const __bf16*)feat;
    A.fmid = A.fhi + npad / 32 * Sh::KBH * 512;
    A.flo = A.fmid + npad / 32 * Sh::KBL * 512;
    A.info = reinterpret_cast<const float*>(A.flo + npad / 32 * Sh::KBL * 512);
}

template <int D>
hipError_t launch_bstep_bf16f_t(const Batch& b, const BatchedArgs& B, int t, int grid, hipStream_t s) {
    Bf16fArgs A = {};
    StepArgs& a = A.base;
    a.Xp = b.Xp;
    a.n = b.n;
    a.d = b.d;
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
    bf16f_operands<D>(A, b.pf, b.feat_blocks);
    A.Xs = b.Xs;
    A.shift = b.shift;
    hipLaunchKernelGGL((step_bf16f_kernel<D, true>), dim3(grid), dim3(kFThreads), 0, s, A, t, B);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_iteration_bf16f(Batch& b, int t, hipStream_t s) {
    switch (b.sh.D) {
        case 8: return launch_bf16f_t<8>(b, t, s);
        case 16: return launch_bf16f_t<16>(b, t, s);
        case 32: return launch_bf16f_t<32>(b, t, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bstep_bf16f(const Batch& b, const BatchedArgs& B, int t, int grid, hipStream_t s) {
    switch (b.sh.D) {
        case 8: return launch_bstep_bf16f_t<8>(b, B, t, grid, s);
        case 16: return launch_bstep_bf16f_t<16>(b, B, t, grid, s);
        case 32: return launch_bstep_bf16f_t<32>(b, B, t, grid, s);
        default: return hipErrorInvalidValue;
    }
}

size_t bf16f_feature_bytes_blocks(long long nblk, int D) {
    switch (D) {
        case 8: return bf16f_bytes_blocks_t<8>(nblk);
        case 16: return bf16f_bytes_blocks_t<16>(nblk);
        case 32: return bf16f_bytes_blocks_t<32>(nblk);
        default: return 0;
    }
}

hipError_t launch_bf16f_features_batched(const float* Xs, int D, const long long* x_off, const int32_t* boff,
                                         int ncl, int nblk, void* feat, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    Bf16fArgs A = {};
#define FMS_BFEAT(DD)                                                                                     \
    case DD: {                                                                                            \
        bf16f_operands<DD>(A, feat, nblk);                                                                \
        hipLaunchKernelGGL(bf16f_features_kernel<DD>, dim3(nblk), dim3(kFBlk), 0, s, Xs, 0,              \
                           (__bf16*)A.fhi, (__bf16*)A.fmid, (__bf16*)A.flo, (float*)A.info, x_off, boff,  \
                           ncl);                                                                          \
        break;                                                                                            \
    }
    switch (D) {
        FMS_BFEAT(8)
        FMS_BFEAT(16)
        FMS_BFEAT(32)
        default:
            return hipErrorInvalidValue;
    }
#undef FMS_BFEAT
    return hipGetLastError();
}

size_t bf16f_feature_bytes(int n, int D) {
    switch (D) {
        case 8: return bf16f_bytes_t<8>(n);
        case 16: return bf16f_bytes_t<16>(n);
        case 32: return bf16f_bytes_t<32>(n);
        default: return 0;
    }
}

// (geom, the shared block geometry, is not used: this form centres its blocks
// itself)
hipError_t launch_bf16f_features(const float* Xs, int n, int D, const float* /*geom*/, void* feat,
                                 hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nblk = (n + kFBlk - 1) / kFBlk;
    const int npad = nblk * kFBlk;
    __bf16* fhi = (__bf16*)feat;
#define FMS_FEAT(DD)                                                                                      \
    case DD: {                                                                                            \
        __bf16* fmid = fhi + (size_t)npad / 32 * FShape<DD>::KBH * 512;                                   \
        __bf16* flo = fmid + (size_t)npad / 32 * FShape<DD>::KBL * 512;                                   \
        float* info = reinterpret_cast<float*>(flo + (size_t)npad / 32 * FShape<DD>::KBL * 512);          \
        hipLaunchKernelGGL(bf16f_features_kernel<DD>, dim3(nblk), dim3(kFBlk), 0, s, Xs, n, fhi, fmid,   \
                           flo, info, nullptr, nullptr, 0);                                               \
        break;                                                                                            \
    }
    switch (D) {
        FMS_FEAT(8)
        FMS_FEAT(16)
        FMS_FEAT(32)
        default:
            return hipErrorInvalidValue;
    }
#undef FMS_FEAT
    return hipGetLastError();
}

}  // namespace fms
