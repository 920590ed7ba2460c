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
constexpr int kMaxGrid = 2048;   // 8 workgroups of 4 waves on each of 256 CUs

// Point chunks per seed tile for m active seeds: the grid split over the
// tiles, with at least min_chunk points per chunk.  A function of (m, grid)
// only, so every kernel of an iteration agrees and the result does not depend
// on the order of the active list.
__device__ __forceinline__ int chunks_for(int m, int TS, int n, int grid, int min_chunk) {
    int tiles = (m + TS - 1) / TS;
    if (tiles >= grid) return 1;
    int c = grid / tiles;
    int cmax = (n + min_chunk - 1) / min_chunk;
    if (c > cmax) c = cmax;
    return c < 1 ? 1 : c;
}

__device__ __forceinline__ int active_count(const Ctl* ctl, int t) {
    // early stop (Section II-C): once `need` seeds converged, nothing is active
    return (ctl->conv_base[t % 3] >= ctl->need) ? 0 : ctl->count[t % 3];
}

// Seeds that converged at iteration t: per-iteration count and the running
// total that iteration t + 1 starts from.
__device__ __forceinline__ void add_converged(Ctl* ctl, int t, int c) {
    atomicAdd(&ctl->conv_it[t], c);
    atomicAdd(&ctl->conv_base[(t + 1) % 3], c);
}

struct StepArgs {
    const float* Xp;
    int n, d;
    int min_chunk;     // points per point chunk, at least
    float* S;
    const int32_t* act_in;
    int32_t* act_out;
    uint8_t* status;
    int32_t* iters;
    float* shift2;
    float* part;
    float* red;        // per-slot sums reduced from many chunk partials
    unsigned long long* prog;   // host-mapped progress word, or NULL
    Ctl* ctl;
    float h2, scale, inv_scale, thr2;
    int metric = MS_METRIC_EUCLIDEAN;   // cosine: the updated seed is renormalized
    // 1: the finalize compacts in list order (each 64-slot run's kept ids and
    // count go to the run's own rows of `red`, and ordered_compact_kernel
    // places the runs one after the other), so the grouping of seeds into
    // waves is the same on every run; 0: one atomic per wave (run order is
    // the order of the atomics)
    int ordered = 0;
};

// Done once per iteration by thread 0 of workgroup 0 of the step kernel:
// reset the count of the iteration after next, carry the converged total
// into the slot of the next iteration, account the pairs, and
// publish (t, m) to the host-mapped progress word so that the host can stop
// enqueueing iterations once m reaches 0 (system-scope vector store).
__device__ __forceinline__ void step_prologue(const StepArgs& a, int t, int m) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    Ctl* ctl = a.ctl;
    ctl->count[(t + 2) % 3] = 0;
    ctl->conv_base[(t + 1) % 3] = ctl->conv_base[t % 3];   // finalize of t adds to it
    if (m > 0) {
        ctl->pairs += (long long)m * a.n;
        ctl->iters_run = t + 1;
    }
    if (a.prog)
        __hip_atomic_store(a.prog, ((unsigned long long)(unsigned)t << 32) | (unsigned)m,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Update and convergence test of seed j from its sums v[0..D) = sum w (x - s)
// (packed units) and v[D] = sum w.  Returns 1 if the seed stays active, 2 if
// it converged, 0 otherwise.  update_seed takes a slot of the active list.
template <int D, int DP>
__device__ __forceinline__ int update_seed_id(const StepArgs& a, int j, const float* v) {
    const float W = v[D];
    if (!(W > 0.0f) || !isfinite(W)) {
        a.status[j] = ST_FAILED;
        return 0;
    }
    float sh2 = 0.0f;
    float* sj = a.S + (long long)j * DP;
    bool finite = true;
    const float inv = a.inv_scale / W;
    if (a.metric == MS_METRIC_COSINE) {
        // the weighted mean direction: s' = (s + shift) / |s + shift|, and the
        // shift that counts is the one to the renormalized seed
        // (the unnormalized coordinates are recomputed in the second pass, not
        // kept, so wide seeds need no extra registers)
        float nn = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float t = sj[k] + v[k] * inv;
            nn = fmaf(t, t, nn);
        }
        const float rn = 1.0f / sqrtf(nn);
        finite = nn > 0.0f && isfinite(rn);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float uk = (sj[k] + v[k] * inv) * rn;
            const float dk = uk - sj[k];
            finite = finite && isfinite(uk);
            sh2 = fmaf(dk, dk, sh2);
            sj[k] = uk;
        }
    } else {
        // padded coordinates (k >= d) carry exact zeros, so looping to D is exact
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float dk = v[k] * inv;
            finite = finite && isfinite(dk);
            sh2 = fmaf(dk, dk, sh2);
            sj[k] = sj[k] + dk;
        }
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

template <int D, int DP>
__device__ __forceinline__ int update_seed(const StepArgs& a, int slot, const float* v) {
    return update_seed_id<D, DP>(a, a.act_in[slot], v);
}

// Sums of one work item of the FP32 step: the seeds act[slot0 .. slot0+TS)
// (slots >= m padded with the first seed, their sums unused) over the points
// Xp[lo, hi) (packed, stride DP).  The four waves take consecutive quarters of
// the points, each lane R seeds; the wave sums are added in wave order and
// wave 0 returns them in acc.  `red` is LDS of (kWaves - 1) * TS * (D + 1)
// floats.  All threads of the workgroup must call it.
// A value every lane of the wave holds, moved to scalar registers (so that
// addresses built from it give scalar loads).
__device__ __forceinline__ long long wave_uniform(long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffll));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Read-only data at a wave-uniform address, seen through the constant
// address space: loads from it are scalar (s_load) and shared by the wave.
// Only for data no kernel of the launch writes.
typedef const __attribute__((address_space(4))) float* const_f32_ptr;

__device__ __forceinline__ const_f32_ptr wave_uniform_const(const float* p) {
    return (const_f32_ptr)(uintptr_t)wave_uniform((long long)reinterpret_cast<uintptr_t>(p));
}

// Calls f(x) for the rows xrow[0 .. count) in order (row stride DP, the first
// D entries of each), the rows being wave-uniform: scalar loads, in groups of
// U rows (32 floats), the next group's loads issued before the current group
// is used.  With few waves per SIMD nothing else hides their latency.
// Rows wider than 32 floats are loaded one at a time.
template <int D, int DP, typename F>
__device__ __forceinline__ void stream_rows(const_f32_ptr xrow, int count, F&& f) {
    constexpr int kGroup = DP <= 4 ? 8 : (DP <= 8 ? 4 : (DP <= 16 ? 2 : (DP <= 32 ? 1 : 0)));
    constexpr int U = kGroup > 0 ? kGroup : 1;
    int p = 0;
    if (kGroup > 0 && count >= U) {
        float xn[U][D];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < D; ++k) xn[u][k] = xrow[u * DP + k];
        xrow += U * DP;
        for (; p + 2 * U <= count; p += U, xrow += U * DP) {
            float xc[U][D];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < D; ++k) xc[u][k] = xn[u][k];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < D; ++k) xn[u][k] = xrow[u * DP + k];
#pragma unroll
            for (int u = 0; u < U; ++u) f(xc[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) f(xn[u]);
        p += U;
    }
    for (; p < count; ++p, xrow += DP) {
        float x[D];
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = xrow[k];
        f(x);
    }
}

template <int D, int DP, int R, int KERN>
__device__ __forceinline__ void tile_sums(const StepArgs& a, const float* __restrict__ Xp, long long lo,
                                          long long hi, const int32_t* __restrict__ act, int slot0, int m,
                                          float (&acc)[R][D + 1], float* red) {
    constexpr int TS = 64 * R;
    constexpr int V = TS * (D + 1);
    // the wave index is uniform across a wave; saying so lets the point
    // stream use scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the bounds and the base are the same in every lane (they derive from
    // the active count and the work item, which the compiler cannot see)
    const long long len = hi - lo;
    const int p0 = __builtin_amdgcn_readfirstlane((int)(lo + len * wave / kWaves));
    const int p1 = __builtin_amdgcn_readfirstlane((int)(lo + len * (wave + 1) / kWaves));
    const const_f32_ptr xs = wave_uniform_const(Xp);
    float s[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int slot = slot0 + r * 64 + lane;
        const int j = act[slot < m ? slot : slot0];
#pragma unroll
        for (int k = 0; k < D; ++k) s[r][k] = a.S[(long long)j * DP + k] * a.scale;
#pragma unroll
        for (int k = 0; k <= D; ++k) acc[r][k] = 0.0f;
    }
    // one point's contribution to every seed of the lane
    auto pair = [&](const float (&x)[D]) {
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
                w = (q <= a.h2) ? 1.0f : 0.0f;
            acc[r][D] += w;
#pragma unroll
            for (int k = 0; k < D; ++k) acc[r][k] = fmaf(w, dx[k], acc[r][k]);
        }
    };
    stream_rows<D, DP>(xs + (long long)p0 * DP, p1 - p0, pair);
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
        if (done) add_converged(a.ctl, t, __popcll(done));
    }
    base = __shfl(base, 0);
    if (res == 1) a.act_out[base + __popcll(keep & ((1ull << lane) - 1ull))] = a.act_in[slot];
}

// Reduction of the chunk partials and finalize (only when chunks > 1).
// Few chunks (many seeds): finalize_kernel reads the partials itself, one lane
// per seed, adding them in chunk order (all loads in flight at once).  Many chunks (few seeds): reduce_kernel
// first spreads the sums over the whole chip -- each workgroup takes a group of
// SG seeds (a power of two <= 16, <= 8 for D >= 32, chosen from m and the grid), its 1024 threads
// add the partials of chunk lanes c = cl, cl + 1024/SG, ... in fixed order,
// then a fixed butterfly inside each wave and a fixed-order sum over the 16
// waves -- and writes one (D+1)-vector per slot to `red`; finalize_kernel then
// reads those.  Either way each wave compacts its 64 consecutive slots with one
// ballot and one atomic, so the active list keeps 64-slot runs in order.
constexpr int kFinThreads = 1024;
constexpr int kFinWaves = kFinThreads / 64;
constexpr int kDirectChunks = 16;   // one round of loads per seed in the finalize
constexpr int kRedThreads = 1024;

// Rows of `red` that hold the kept ids (64) and their count (at 64) of the
// 64-slot run starting at slot `base` in the ordered compaction: the run's
// own 64 x (D+1) floats, which the finalize has read before it writes them.
template <int D>
__device__ __forceinline__ int32_t* run_rows(const StepArgs& a, int base) {
    static_assert(64 * (D + 1) >= 65, "a run's rows hold its ids and count");
    return reinterpret_cast<int32_t*>(a.red + (long long)base * (D + 1));
}

template <int D, int DP>
__device__ __forceinline__ void compact_wave(const StepArgs& a, int t, int slot, int res) {
    const int lane = threadIdx.x & 63;
    const unsigned long long keep = __ballot(res == 1);
    const unsigned long long done = __ballot(res == 2);
    const int rank = __popcll(keep & ((1ull << lane) - 1ull));
    if (a.ordered) {
        int32_t* rows = run_rows<D>(a, slot - lane);
        if (res == 1) rows[rank] = a.act_in[slot];
        if (lane == 0) {
            rows[64] = __popcll(keep);
            if (done) add_converged(a.ctl, t, __popcll(done));
        }
        return;
    }
    int off = 0;
    if (lane == 0) {
        if (keep) off = atomicAdd(&a.ctl->count[(t + 1) % 3], __popcll(keep));
        if (done) add_converged(a.ctl, t, __popcll(done));
    }
    off = __shfl(off, 0);
    if (res == 1) a.act_out[off + rank] = a.act_in[slot];
}

// The ordered compaction's second half, by one workgroup of kFinThreads
// after the finalize has written every run's rows: the kept ids of the runs,
// run after run, into act_out, and the next iteration's active count.
// Up to 64 runs (4,096 active slots), wave w takes runs w, w + 16, w + 32,
// w + 48, whose rows it loads together with the active count (`cap_runs`,
// the runs the rows of `red` hold, bounds those loads; rows past the count
// are loaded but not used).  More runs: their counts are scanned
// kFinThreads at a time, and wave w copies runs w, w + 16, ... of each batch.
// A last-workgroup placement inside the finalize (device-scope fences
// around a count of finished workgroups) measured slower on the 512 x 200K
// iteration than this launch of its own.
constexpr int kRunsPerWave = 4;

template <int D>
__device__ void ordered_place_many(const StepArgs& a, int t, int nruns) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ int pre[kFinThreads], cnt[kFinThreads], wtot[kFinWaves];
    int total = 0;
    for (int r0 = 0; r0 < nruns; r0 += kFinThreads) {
        const int r = r0 + threadIdx.x;
        const int c = r < nruns ? run_rows<D>(a, r * 64)[64] : 0;
        int x = c;   // inclusive scan within the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wtot[wave] = x;
        __syncthreads();
        int wbase = 0, btot = 0;
        for (int w = 0; w < kFinWaves; ++w) {
            wbase += w < wave ? wtot[w] : 0;
            btot += wtot[w];
        }
        pre[threadIdx.x] = total + wbase + x - c;
        cnt[threadIdx.x] = c;
        __syncthreads();
        const int nr = nruns - r0 < kFinThreads ? nruns - r0 : kFinThreads;
        for (int q = wave; q < nr; q += kFinWaves) {
            if (lane < cnt[q]) a.act_out[pre[q] + lane] = run_rows<D>(a, (r0 + q) * 64)[lane];
        }
        total += btot;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.ctl->count[(t + 1) % 3] = total;
}

template <int D>
__global__ __launch_bounds__(kFinThreads) void ordered_compact_kernel(StepArgs a, int t, int cap_runs) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int c[kRunsPerWave], id[kRunsPerWave];
#pragma unroll
    for (int u = 0; u < kRunsPerWave; ++u) {
        const int r = wave + kFinWaves * u;
        c[u] = 0;
        id[u] = 0;
        if (r < cap_runs) {
            const int32_t* rows = run_rows<D>(a, r * 64);
            c[u] = rows[64];
            id[u] = rows[lane];
        }
    }
    const int m = active_count(a.ctl, t);
    if (m == 0) return;
    const int nruns = (m + 63) / 64;
    if (nruns > kFinWaves * kRunsPerWave) {
        ordered_place_many<D>(a, t, nruns);
        return;
    }
    __shared__ int wc[kFinWaves * kRunsPerWave];
    if (lane == 0) {
#pragma unroll
        for (int u = 0; u < kRunsPerWave; ++u) {
            const int r = wave + kFinWaves * u;
            wc[r] = r < nruns ? c[u] : 0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRunsPerWave; ++u) {
        const int r = wave + kFinWaves * u;
        if (r < nruns) {
            int off = 0;   // kept ids of the runs before r
            for (int q = 0; q < r; ++q) off += wc[q];
            if (lane < c[u]) a.act_out[off + lane] = id[u];
        }
    }
    if (threadIdx.x == 0) {
        int total = 0;
        for (int q = 0; q < nruns; ++q) total += wc[q];
        a.ctl->count[(t + 1) % 3] = total;
    }
}

template <int D, int R>
__global__ __launch_bounds__(kRedThreads) void reduce_kernel(StepArgs a, int t, int grid) {
    constexpr int TS = 64 * R;
    constexpr int kRedMaxSG = D >= 32 ? 8 : 16;   // keeps wsum within 36 KB of LDS
    const int m = active_count(a.ctl, t);
    if (m == 0) return;
    const int chunks = chunks_for(m, TS, a.n, grid, a.min_chunk);
    if (chunks <= kDirectChunks) return;
    const int per = (m + (int)gridDim.x - 1) / (int)gridDim.x;
    int SG = 1;
    while (SG < per && SG < kRedMaxSG) SG <<= 1;
    const int CL = kRedThreads / SG;
    const int sidx = threadIdx.x & (SG - 1), cl = threadIdx.x / SG;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ float wsum[kRedThreads / 64][kRedMaxSG][D + 1];
    // workgroups are dealt to the 8 XCDs round-robin; consecutive seed groups
    // go to workgroups of one XCD so that the partial rows they share (8 seeds
    // per 128-byte line) are fetched into one L2 only
    int lb = blockIdx.x;
    if (gridDim.x % 8 == 0) lb = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    for (int g0 = lb * SG; g0 < m; g0 += gridDim.x * SG) {
        const int slot = g0 + sidx;
        float v[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) v[k] = 0.0f;
        if (slot < m) {
            const int tile = slot / TS, pos = slot % TS;
            const float* src = a.part + ((long long)tile * chunks * TS + pos) * (D + 1);
            for (int c = cl; c < chunks; c += CL) {
                const float* p = src + (long long)c * TS * (D + 1);
#pragma unroll
                for (int k = 0; k <= D; ++k) v[k] += p[k];
            }
        }
        // lanes of a wave holding the same seed differ in the bits >= SG
        for (int off = 32; off >= SG; off >>= 1)
#pragma unroll
            for (int k = 0; k <= D; ++k) v[k] += __shfl_xor(v[k], off);
        if (lane < SG) {
#pragma unroll
            for (int k = 0; k <= D; ++k) wsum[wave][lane][k] = v[k];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < SG * (D + 1); e += kRedThreads) {
            const int s2 = e / (D + 1), k = e % (D + 1);
            if (g0 + s2 < m) {
                float acc = 0.0f;
                for (int w = 0; w < kRedThreads / 64; ++w) acc += wsum[w][s2][k];
                a.red[(long long)(g0 + s2) * (D + 1) + k] = acc;
            }
        }
        __syncthreads();
    }
}

template <int D, int DP, int R>
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(StepArgs a, int t, int grid) {
    constexpr int TS = 64 * R;
    const int m = active_count(a.ctl, t);
    if (m == 0) return;
    const int chunks = chunks_for(m, TS, a.n, grid, a.min_chunk);
    if (chunks == 1 && !a.ordered) return;   // finalized inside the step kernel
    const bool pre = chunks > kDirectChunks;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = gridDim.x * kFinWaves;
    for (int base = (blockIdx.x * kFinWaves + wave) * 64; base < m; base += nwaves * 64) {
        const int slot = base + lane;
        int res = 0;
        if (slot < m) {
            float v[D + 1];
            if (pre) {
#pragma unroll
                for (int k = 0; k <= D; ++k) v[k] = a.red[(long long)slot * (D + 1) + k];
            } else {
                const int tile = slot / TS, pos = slot % TS;
#pragma unroll
                for (int k = 0; k <= D; ++k) v[k] = 0.0f;
                const float* src = a.part + ((long long)tile * chunks * TS + pos) * (D + 1);
                // U chunks' loads in flight at once, added in chunk order
                constexpr int U = D <= 4 ? 16 : (D <= 8 ? 8 : (D <= 16 ? 4 : (D <= 32 ? 2 : 1)));
                if constexpr (U == 1) {   // wide seeds: no staging registers
                    for (int c = 0; c < chunks; ++c) {
                        const float* p = src + (long long)c * TS * (D + 1);
#pragma unroll
                        for (int k = 0; k <= D; ++k) v[k] += p[k];
                    }
                } else
                for (int c0 = 0; c0 < chunks; c0 += U) {
                    float tmp[U][D + 1];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const float* p = src + (long long)(c0 + u < chunks ? c0 + u : c0) * TS * (D + 1);
#pragma unroll
                        for (int k = 0; k <= D; ++k) tmp[u][k] = p[k];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (c0 + u < chunks) {
#pragma unroll
                            for (int k = 0; k <= D; ++k) v[k] += tmp[u][k];
                        }
                    }
                }
            }
            res = update_seed<D, DP>(a, slot, v);
        }
        compact_wave<D, DP>(a, t, slot, res);
    }
}

// Reduction and finalize in one launch, for narrow seeds (D <= 8) whose
// partials per 64-slot run are few enough for one workgroup (at most
// kFusedFloats floats per slot: chunks x (D+1)).  A workgroup takes a run of
// 64 consecutive active slots: wave w adds the partials of chunks w, w + 16,
// w + 32, ... of every slot of the run (lane = slot, so each chunk's 64
// partials are one contiguous read), U chunks' loads in flight, in chunk
// order; the 16 wave sums are added in wave order through LDS; wave 0 then
// updates the 64 seeds and compacts them with one ballot and one atomic, as
// finalize_kernel does.  No second launch, no reduced copy in memory.
constexpr int kFusedFloats = 2048;

template <int D, int DP, int R>
__global__ __launch_bounds__(kFinThreads) void finalize_fused_kernel(StepArgs a, int t, int grid) {
    static_assert(D <= 8, "the wave sums of wide seeds do not fit in LDS");
    constexpr int TS = 64 * R;
    constexpr int U = D <= 4 ? 8 : 4;
    const int m = active_count(a.ctl, t);
    if (m == 0) return;
    const int chunks = chunks_for(m, TS, a.n, grid, a.min_chunk);
    if (chunks == 1 && !a.ordered) return;   // finalized inside the step kernel
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ float wsum[kFinWaves - 1][D + 1][64];
    for (int base = blockIdx.x * 64; base < m; base += gridDim.x * 64) {
        const int slot = base + lane;
        float v[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) v[k] = 0.0f;
        if (slot < m) {
            const int tile = slot / TS, pos = slot % TS;
            const float* src = a.part + ((long long)tile * chunks * TS + pos) * (D + 1);
            for (int c0 = wave; c0 < chunks; c0 += U * kFinWaves) {
                float tmp[U][D + 1];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = c0 + u * kFinWaves;
                    const float* p = src + (long long)(c < chunks ? c : c0) * TS * (D + 1);
#pragma unroll
                    for (int k = 0; k <= D; ++k) tmp[u][k] = p[k];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (c0 + u * kFinWaves < chunks) {
#pragma unroll
                        for (int k = 0; k <= D; ++k) v[k] += tmp[u][k];
                    }
                }
            }
        }
        if (wave > 0) {
#pragma unroll
            for (int k = 0; k <= D; ++k) wsum[wave - 1][k][lane] = v[k];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int w = 1; w < kFinWaves; ++w)
#pragma unroll
                for (int k = 0; k <= D; ++k) v[k] += wsum[w - 1][k][lane];
            const int res = slot < m ? update_seed<D, DP>(a, slot, v) : 0;
            compact_wave<D, DP>(a, t, slot, res);
        }
        __syncthreads();
    }
}

// Launch of the reduction and the finalize for a batch of B seeds.  Narrow
// seeds whose partials fit the fused kernel for every active count (the most
// chunks a tile can have is that of a one-tile batch) take the one launch of
// finalize_fused_kernel.  Otherwise: the reduction (exits at once unless many
// chunks) and the finalize (exits at once when the step kernel finalized);
// may_reduce = false: the caller's shape never has more than kDirectChunks
// chunks per tile, and the reduction launch is left out.
template <int D, int DP, int R>
inline hipError_t launch_finalize(const StepArgs& a, int t, int grid, int B, hipStream_t s,
                                  bool may_reduce = true) {
    if constexpr (D <= 8) {
        const long long cmax = std::min<long long>(grid, ((long long)a.n + a.min_chunk - 1) / a.min_chunk);
        if (cmax * (D + 1) <= kFusedFloats) {
            int fblocks = (B + 63) / 64;
            if (fblocks > 4096) fblocks = 4096;
            if (fblocks < 1) fblocks = 1;
            hipLaunchKernelGGL((finalize_fused_kernel<D, DP, R>), dim3(fblocks), dim3(kFinThreads), 0, s, a,
                               t, grid);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess || !a.ordered) return e;
            hipLaunchKernelGGL((ordered_compact_kernel<D>), dim3(1), dim3(kFinThreads), 0, s, a, t,
                               (B + 63) / 64);
            return hipGetLastError();
        }
    }
    if (may_reduce) {
        const int rblocks = B < 256 ? (B < 1 ? 1 : B) : 256;
        hipLaunchKernelGGL((reduce_kernel<D, R>), dim3(rblocks), dim3(kRedThreads), 0, s, a, t, grid);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    int fblocks = (B + kFinThreads - 1) / kFinThreads;
    if (fblocks > 512) fblocks = 512;
    if (fblocks < 1) fblocks = 1;
    hipLaunchKernelGGL((finalize_kernel<D, DP, R>), dim3(fblocks), dim3(kFinThreads), 0, s, a, t,
                       grid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.ordered) return e;
    hipLaunchKernelGGL((ordered_compact_kernel<D>), dim3(1), dim3(kFinThreads), 0, s, a, t, (B + 63) / 64);
    return hipGetLastError();
}

}  // namespace
}  // namespace fms
