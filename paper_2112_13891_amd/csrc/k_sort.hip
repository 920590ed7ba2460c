// k_sort.hip -- spatial order of the points for the BF16 step (gfx950).
//
// The BF16 form centres every 256-point block of points on a local reference
// so that the bf16 products stay accurate; that needs blocks that are compact
// in space.  For D <= 4 points are ordered by the Morton code of their
// quantized coordinates; for larger D (where a Morton code has too few bits
// per axis) by their nearest pivot, pivots being a fixed sample of the points
// (one per 256, at most 1,024, taken in the order of a greedy
// nearest-neighbour chain), and within a pivot's run by distance; points far from
// every pivot follow all the runs, so that they do not widen the runs' last
// blocks.  Both use a stable LSD radix sort, deterministic (no
// floating-point atomics; ranks inside a block come from wave ballots in wave
// order).  The order only changes which points share a block: the update sums
// over all points whatever their order.

#include "fms_internal.h"

namespace fms {

namespace {

constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / 64;

// Per-dimension min/max of the packed points (first D of DP columns).
__global__ __launch_bounds__(256) void bounds_kernel(const float* __restrict__ Xp, int n, int DP,
                                                     int D, float* out /* 2*D, init +/-inf */) {
    __shared__ float smin[256], smax[256];
    for (int k = 0; k < D; ++k) {
        float lo = __builtin_inff(), hi = -__builtin_inff();
        for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
            const float v = Xp[(long long)i * DP + k];
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        smin[threadIdx.x] = lo;
        smax[threadIdx.x] = hi;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
                smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + off]);
                smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + off]);
            }
            __syncthreads();
        }
        // per-block results go to a scratch row; the host-side launcher reduces
        // them in a second pass (see bounds_final_kernel)
        if (threadIdx.x == 0) {
            out[2 * D + (2 * blockIdx.x) * D + k] = smin[0];
            out[2 * D + (2 * blockIdx.x + 1) * D + k] = smax[0];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void bounds_final_kernel(float* out, int D, int blocks) {
    __shared__ float lo_s[256], hi_s[256];
    for (int k = 0; k < D; ++k) {
        float lo = __builtin_inff(), hi = -__builtin_inff();
        for (int b = threadIdx.x; b < blocks; b += 256) {
            lo = fminf(lo, out[2 * D + (2 * b) * D + k]);
            hi = fmaxf(hi, out[2 * D + (2 * b + 1) * D + k]);
        }
        lo_s[threadIdx.x] = lo;
        hi_s[threadIdx.x] = hi;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) {
                lo_s[threadIdx.x] = fminf(lo_s[threadIdx.x], lo_s[threadIdx.x + off]);
                hi_s[threadIdx.x] = fmaxf(hi_s[threadIdx.x], hi_s[threadIdx.x + off]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[2 * k] = lo_s[0];
            out[2 * k + 1] = hi_s[0];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ unsigned spread_bits(unsigned v, int D) {
    // interleave: bit b of v goes to bit b*D
    unsigned r = 0;
    for (int b = 0; b < 30 / D; ++b) r |= ((v >> b) & 1u) << (b * D);
    return r;
}

// Morton key of one row (first D coordinates, times `scale`) on the grid of
// 2^(30/D) cells per axis spanned by the point bounds.
__device__ __forceinline__ unsigned morton_key(const float* row, int D, float scale,
                                               const float* __restrict__ bnd) {
    const int bits = 30 / D;
    const float cells = (float)(1u << bits);
    unsigned key = 0;
    for (int k = 0; k < D; ++k) {
        const float lo = bnd[2 * k], hi = bnd[2 * k + 1];
        const float span = hi - lo;
        float f = span > 0.0f ? (row[k] * scale - lo) / span * cells : 0.0f;
        if (!(f >= 0.0f)) f = 0.0f;   // also NaN
        if (f > cells - 1.0f) f = cells - 1.0f;
        key |= spread_bits((unsigned)(int)f, D) << k;
    }
    return key;
}

constexpr int kPointKeyDrop = 6;   // Morton bits dropped from the point keys

__global__ void morton_kernel(const float* __restrict__ Xp, int n, int DP, int D,
                              const float* __restrict__ bnd, unsigned* keys, int* vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // the top 24 bits of the Morton code (256 cells per axis for D = 3):
    // three radix passes instead of four
    keys[i] = morton_key(Xp + (long long)i * DP, D, 1.0f, bnd) >> kPointKeyDrop;
    vals[i] = i;
}

// Seed keys: Morton key of the seed position in the points' grid; seeds that
// are not active get bit 30 so that they sort after every active seed.
__global__ void seed_key_kernel(const float* __restrict__ S, int DP, int D, int m, float scale,
                                const uint8_t* __restrict__ status, const float* __restrict__ bnd,
                                unsigned* keys, int* vals) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    unsigned key = morton_key(S + (long long)j * DP, D, scale, bnd);
    if (status[j] != ST_ACTIVE) key |= 1u << 30;
    keys[j] = key;
    vals[j] = j;
}

// Small batches (m <= 4096) in one workgroup: keys as above (or given), then a bitonic
// sort of (key << 32 | slot) in LDS -- the slot in the low bits makes every
// key distinct, so the result is the stable order.
constexpr int kSeedSortMax = 4096;

__global__ __launch_bounds__(1024) void seed_order_small_kernel(
    const float* __restrict__ S, int DP, int D, int m, float scale,
    const uint8_t* __restrict__ status, const float* __restrict__ bnd,
    const unsigned* __restrict__ keys_in, int32_t* act0) {
    __shared__ unsigned long long key[kSeedSortMax];
    int P = 1;
    while (P < m) P <<= 1;
    for (int e = threadIdx.x; e < P; e += 1024) {
        unsigned long long k = ~0ull;
        if (e < m) {
            unsigned mk;
            if (keys_in) {
                mk = keys_in[e];
            } else {
                mk = morton_key(S + (long long)e * DP, D, scale, bnd);
                if (status[e] != ST_ACTIVE) mk |= 1u << 30;
            }
            k = ((unsigned long long)mk << 32) | (unsigned)e;
        }
        key[e] = k;
    }
    __syncthreads();
    if (P <= 1024) {
        // one key per thread: exchanges within a wave through lane shuffles,
        // the others through LDS (one barrier per such stage)
        const int e = threadIdx.x;
        unsigned long long k = e < P ? key[e] : ~0ull;
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                unsigned long long y;
                if (stride < 64) {
                    const unsigned lo = __shfl_xor((unsigned)k, stride);
                    const unsigned hi = __shfl_xor((unsigned)(k >> 32), stride);
                    y = ((unsigned long long)hi << 32) | lo;
                } else {
                    __syncthreads();
                    if (e < P) key[e] = k;
                    __syncthreads();
                    y = e < P ? key[e ^ stride] : ~0ull;
                }
                // the lower element of an ascending pair keeps the minimum
                const bool up = (e & size) == 0;
                const bool lower = (e & stride) == 0;
                const unsigned long long lo_v = k < y ? k : y, hi_v = k < y ? y : k;
                k = (lower == up) ? lo_v : hi_v;
            }
        }
        if (e < m) act0[e] = (int32_t)(k & 0xffffffffu);
        return;
    }
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = threadIdx.x; e < P; e += 1024) {
                const int o = e ^ stride;
                if (o > e) {
                    const bool up = (e & size) == 0;
                    const unsigned long long x = key[e], y = key[o];
                    if ((x > y) == up) {
                        key[e] = y;
                        key[o] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < m; e += 1024) act0[e] = (int32_t)(key[e] & 0xffffffffu);
}

// Stable LSD radix sort, 8 bits per pass.  Per-block digit counts go to
// hist (digit-major, 256 x nblocks); the digit totals are summed into dtot with
// integer atomics (order-independent).
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const unsigned* __restrict__ keys,
                                                                  int n, int shift, int nblocks,
                                                                  int* hist, int* dtot) {
    __shared__ int h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    __syncthreads();
    if (threadIdx.x < 256) {
        const int c = h[threadIdx.x];
        hist[threadIdx.x * nblocks + blockIdx.x] = c;
        if (c) atomicAdd(&dtot[threadIdx.x], c);
    }
}

__global__ void zero_ints_kernel(int* a, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) a[i] = 0;
}

// Inclusive scan of one value per thread over a 256-thread block; returns the
// block total in *total.
__device__ __forceinline__ int block_scan256(int v, int* wsum, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return v + before;
}

// Exclusive offsets: one workgroup per digit.  The digit's base is the sum of
// the totals of all smaller digits; its row of per-block counts is then
// scanned in 256-wide steps (coalesced).
__global__ __launch_bounds__(256) void radix_scan_kernel(int* hist, int nblocks,
                                                         const int* __restrict__ dtot) {
    __shared__ int wsum[4];
    const int dig = blockIdx.x;
    int base;   // sum of the totals of the digits below this one
    (void)block_scan256(threadIdx.x < dig ? dtot[threadIdx.x] : 0, wsum, &base);
    int* row = hist + (long long)dig * nblocks;
    for (int c0 = 0; c0 < nblocks; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const int v = i < nblocks ? row[i] : 0;
        int step;
        const int incl = block_scan256(v, wsum, &step);
        if (i < nblocks) row[i] = base + incl - v;
        base += step;
    }
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const unsigned* __restrict__ kin, const int* __restrict__ vin, int n, int shift, int nblocks,
    const int* __restrict__ offs, unsigned* kout, int* vout) {
    __shared__ int wcount[kSortWaves][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < kSortWaves * 256; e += kSortThreads) (&wcount[0][0])[e] = 0;
    __syncthreads();
    const int i = blockIdx.x * kSortThreads + threadIdx.x;
    const bool live = i < n;
    const unsigned key = live ? kin[i] : 0u;
    const unsigned dig = (key >> shift) & 255u;
    // lanes of this wave with the same digit
    unsigned long long peers = __ballot(live);
    for (int b = 0; b < 8; ++b) {
        const unsigned long long bal = __ballot(live && ((dig >> b) & 1u));
        peers &= ((dig >> b) & 1u) ? bal : ~bal;
    }
    const int rank = __popcll(peers & ((1ull << lane) - 1ull));
    // the lowest peer lane records the wave's count for this digit
    if (live && rank == 0) wcount[wave][dig] = __popcll(peers);
    __syncthreads();
    // exclusive prefix over waves, per digit (wave order = index order)
    if (threadIdx.x < 256) {
        int s = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            const int c = wcount[w][threadIdx.x];
            wcount[w][threadIdx.x] = s;
            s += c;
        }
    }
    __syncthreads();
    if (live) {
        const int pos = offs[dig * nblocks + blockIdx.x] + wcount[wave][dig] + rank;
        kout[pos] = key;
        vout[pos] = vin[i];
    }
}

// Xs[i] = Xp[perm[i]] - shift (shift over the first D columns, NULL = 0).
__global__ void gather_rows_kernel(const float* __restrict__ Xp, int DP, int D,
                                   const int* __restrict__ perm, int n,
                                   const float* __restrict__ shift, float* Xs) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * DP) return;
    const int i = (int)(e / DP), k = (int)(e % DP);
    const float v = Xp[(long long)perm[i] * DP + k];
    Xs[e] = (shift && k < D) ? v - shift[k] : v;
}

// Midpoint of the bounding box (the frame of the sorted points for D > 4).
__global__ void shift_kernel(const float* __restrict__ bnd, int D, float* shift) {
    const int k = threadIdx.x;
    if (k < D) shift[k] = 0.5f * (bnd[2 * k] + bnd[2 * k + 1]);
}

// Nearest pivot of each row r of `rows` (stride DPr, times `scale`), pivots
// being the points Xp[j * n / P], j < P, in two launches: pivot_near_kernel
// takes a tile of rows against a chunk of PC pivots and folds its result into
// best[r] = (squared distance bits << 32 | pivot index) with a 64-bit atomic
// minimum (the nearest pivot, ties to the lowest index, whatever the order of
// the chunks); pivot_key_kernel turns it into the sort key.  Chunks of
// kPivChunk pivots for the seeds (few rows still fill the machine), of
// kPivChunkPoints for the points (each row is loaded, and its minimum folded,
// once per chunk: at 262,144 x 32 with 1,024 pivots, 16 chunks re-read the
// rows 16 times).
constexpr int kPivChunk = 64;
constexpr int kPivChunkPoints = 256;

// Many clouds (rc.roff set): blockIdx.x is a 256-row tile of one cloud's
// rows, whose pivots are the cloud's own (points Xp[xoff[c] ..], poff).
template <int D, int PC = kPivChunk>
__global__ __launch_bounds__(256) void pivot_near_kernel(const float* __restrict__ rows, long long m, int DPr,
                                                         float scale, const float* __restrict__ Xp, int n,
                                                         int DP, int P, unsigned long long* best,
                                                         CloudRows rc, const long long* __restrict__ xoff,
                                                         const int32_t* __restrict__ poff) {
    static_assert(D % 4 == 0 && (PC * D) % 256 == 0, "pivot chunk layout");
    constexpr int kPer = PC * D / 256;   // pivot coordinates each thread stages
    __shared__ __attribute__((aligned(16))) float piv[PC][D];
    long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    const int j0 = blockIdx.y * PC;
    if (rc.roff) {
        const int c = upper_cloud(rc.tpre, rc.ncl, blockIdx.x);
        r = rc.roff[c] + (long long)(blockIdx.x - rc.tpre[c]) * 256 + threadIdx.x;
        m = rc.roff[c + 1];
        const long long x0 = xoff[c];
        n = (int)(xoff[c + 1] - x0);
        P = poff[c + 1] - poff[c];
        Xp += x0 * DP;
        if (j0 >= P) return;   // the whole workgroup
    }
    const int cnt = min(PC, P - j0);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = u * 256 + threadIdx.x;
        const int j = e / D, k = e % D;
        piv[j][k] = j < cnt ? Xp[((long long)(j0 + j) * n / P) * DP + k] : 0.0f;
    }
    // rows past m load a valid row (nothing is written for them)
    const long long rr = r < m ? r : m - 1;
    float x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = rows[rr * DPr + k] * scale;
    __syncthreads();
    float bq = __builtin_inff();
    int bi = 0;
    for (int j = 0; j < cnt; ++j) {
        const float4* pj = reinterpret_cast<const float4*>(piv[j]);   // broadcast reads
        float q = 0.0f;
#pragma unroll
        for (int k4 = 0; k4 < D / 4; ++k4) {
            const float4 pv = pj[k4];
            const float t0 = x[4 * k4] - pv.x, t1 = x[4 * k4 + 1] - pv.y;
            const float t2 = x[4 * k4 + 2] - pv.z, t3 = x[4 * k4 + 3] - pv.w;
            q = fmaf(t0, t0, q);
            q = fmaf(t1, t1, q);
            q = fmaf(t2, t2, q);
            q = fmaf(t3, t3, q);
        }
        if (q < bq) {
            bq = q;
            bi = j0 + j;
        }
    }
    if (r < m) atomicMin(&best[r], ((unsigned long long)__float_as_uint(bq) << 32) | (unsigned)bi);
}

__global__ void fill_u64_kernel(unsigned long long* a, int count, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) a[i] = v;
}

// Distance (packed units) from the nearest pivot beyond which a point or seed
// is sorted into the far region, after every pivot run.
constexpr float kFarPivot = 8.0f;

// Sort key of row r from its nearest pivot: the pivot's rank in the chain
// order << 14 | the top 14 bits of the squared distance's FP32 pattern
// (monotone in the distance), so that a pivot's rows run from near to far and
// runs of nearby pivots are adjacent; rows farther than kFarPivot from every
// pivot get bit 24, so that they follow all the runs instead of widening the
// runs' last blocks.  Rows whose status is not active (when status is given)
// get bit 30, so that they sort last.
__global__ void pivot_key_kernel(const unsigned long long* __restrict__ best, int m,
                                 const uint8_t* __restrict__ status, const int* __restrict__ prank,
                                 unsigned* keys, int* vals) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const unsigned long long b = best[r];
    const unsigned qbits = (unsigned)(b >> 32);
    const int bi = (int)(unsigned)b;
    unsigned key = ((unsigned)prank[bi] << 14) | (qbits >> 17);
    if (__uint_as_float(qbits) > kFarPivot * kFarPivot) key |= 1u << 24;
    if (status && status[r] != ST_ACTIVE) key |= 1u << 30;
    keys[r] = key;
    vals[r] = r;
}

// Many clouds: the sort key of row r of cloud c (the cloud found from the
// row offsets) keeps the clouds apart and each cloud's rows in the order of
// the one-cloud key: c << 19 | inactive << 18 | far << 17 | the pivot's chain
// rank within the cloud (< 256) << 9 | the top 9 bits of the squared distance.
__global__ void bpivot_key_kernel(const unsigned long long* __restrict__ best, long long m,
                                  const uint8_t* __restrict__ status, const long long* __restrict__ roff, int ncl,
                                  const int32_t* __restrict__ poff, const int* __restrict__ prank, unsigned* keys,
                                  int* vals) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int c = upper_cloud(roff, ncl, r);
    const unsigned long long b = best[r];
    const unsigned qbits = (unsigned)(b >> 32);
    const int bi = (int)(unsigned)b;
    unsigned key = ((unsigned)c << 19) | ((unsigned)prank[poff[c] + bi] << 9) | (qbits >> 22);
    if (__uint_as_float(qbits) > kFarPivot * kFarPivot) key |= 1u << 17;
    if (status && status[r] != ST_ACTIVE) key |= 1u << 18;
    keys[r] = key;
    vals[r] = (int)r;
}

// Order of the pivots along a greedy nearest-neighbour chain: from pivot 0,
// each next pivot is the nearest one not yet taken (ties to the lowest
// index), so that the pivots of one cluster follow each other.  Two
// launches: pivot_knn_kernel lists each pivot's kKnn nearest other pivots in
// (distance, index) order; pivot_chain_kernel walks the chain in one thread,
// whose next pivot is the first untaken one of the current pivot's list
// (exactly the nearest untaken pivot), and only when every listed pivot is
// taken does the whole workgroup search all pivots.  prank[j] = the chain
// position of pivot j.
constexpr int kKnn = 8;
constexpr int kBatchedPivotMax = 256;   // pivots of one cloud in a batched sort

// One workgroup per 64 pivots; wave q of the sixteen scans the candidates
// i = q (mod 16), and the sixteen lists of a pivot are merged through LDS.
// Many clouds (xoff set): blockIdx.y is the cloud, whose pivots and lists
// are its own (indices within the cloud).
template <int D>
__global__ __launch_bounds__(1024) void pivot_knn_kernel(const float* __restrict__ Xp, int n, int DP, int P,
                                                         int* knn, const long long* __restrict__ xoff,
                                                         const int32_t* __restrict__ poff) {
    constexpr int kW = 16;                     // waves
    constexpr int kCand = 256;                 // candidates staged per pass
    constexpr int kPer = kCand * D / 1024;
    __shared__ __attribute__((aligned(16))) float cand[kCand][D];
    __shared__ unsigned long long lists[kW][64][kKnn];
    if (xoff) {
        const int c = blockIdx.y;
        const long long x0 = xoff[c];
        n = (int)(xoff[c + 1] - x0);
        P = poff[c + 1] - poff[c];
        Xp += x0 * DP;
        knn += (long long)poff[c] * kKnn;
        if ((int)blockIdx.x * 64 >= P) return;   // the whole workgroup
    }
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    const long long row = j < P ? (long long)j * n / P : 0;
    float x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = Xp[row * DP + k];
    unsigned long long best[kKnn];
#pragma unroll
    for (int t = 0; t < kKnn; ++t) best[t] = ~0ull;
    for (int i0 = 0; i0 < P; i0 += kCand) {
        const int cnt = min(kCand, P - i0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = u * 1024 + threadIdx.x;
            const int c = e / D, k = e % D;
            cand[c][k] = c < cnt ? Xp[((long long)(i0 + c) * n / P) * DP + k] : 0.0f;
        }
        __syncthreads();
        for (int c = q; c < cnt; c += kW) {
            const int i = i0 + c;
            const float4* pc = reinterpret_cast<const float4*>(cand[c]);
            float d2 = 0.0f;
#pragma unroll
            for (int k4 = 0; k4 < D / 4; ++k4) {
                const float4 v = pc[k4];
                const float t0 = x[4 * k4] - v.x, t1 = x[4 * k4 + 1] - v.y;
                const float t2 = x[4 * k4 + 2] - v.z, t3 = x[4 * k4 + 3] - v.w;
                d2 = fmaf(t0, t0, d2);
                d2 = fmaf(t1, t1, d2);
                d2 = fmaf(t2, t2, d2);
                d2 = fmaf(t3, t3, d2);
            }
            unsigned long long key = i == j ? ~0ull : ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)i;
            // insertion into the sorted list (registers: a fixed compare-swap chain)
#pragma unroll
            for (int t = 0; t < kKnn; ++t) {
                const unsigned long long lo = key < best[t] ? key : best[t];
                const unsigned long long hi = key < best[t] ? best[t] : key;
                best[t] = lo;
                key = hi;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kKnn; ++t) lists[q][lane][t] = best[t];
    __syncthreads();
    if (q == 0 && j < P) {
        // merge the sixteen sorted lists: the kKnn smallest keys
        int h[kW];
#pragma unroll
        for (int r = 0; r < kW; ++r) h[r] = 0;
        for (int t = 0; t < kKnn; ++t) {
            int wq = 0;
            unsigned long long m = lists[0][lane][h[0]];
#pragma unroll
            for (int r = 1; r < kW; ++r) {
                const unsigned long long v = lists[r][lane][h[r]];
                if (v < m) {
                    m = v;
                    wq = r;
                }
            }
#pragma unroll
            for (int r = 0; r < kW; ++r) h[r] += r == wq;
            knn[j * kKnn + t] = m == ~0ull ? -1 : (int)(unsigned)m;
        }
    }
}

// The walk.  Wave 0 walks while the other waves wait at a barrier: lanes
// 0..7 each read one entry of the current pivot's list and its taken flag,
// and a ballot picks the first untaken entry (two LDS round trips a step).
// When every listed pivot is taken, the whole workgroup searches all pivots
// (a pivot per thread, its coordinates in registers; the current pivot's
// coordinates from LDS) and wave 0 goes on from the nearest untaken one.
// The taken flags and the ranks stay in LDS; the ranks go out at the end.
// Many clouds (xoff set): one workgroup per cloud (blockIdx.x), ranks within
// the cloud.
template <int D>
__global__ __launch_bounds__(1024) void pivot_chain_kernel(const float* __restrict__ Xp, int n, int DP, int P,
                                                          const int* __restrict__ knn, int* prank,
                                                          const long long* __restrict__ xoff,
                                                          const int32_t* __restrict__ poff) {
    __shared__ __attribute__((aligned(16))) float4 pc[D / 4][1024];
    __shared__ short lst[1024 * kKnn];
    __shared__ unsigned char taken[1024];
    __shared__ int rk[1024];
    __shared__ unsigned long long wbest[16];
    __shared__ int s_cur, s_step;
    if (xoff) {
        const int c = blockIdx.x;
        const long long x0 = xoff[c];
        n = (int)(xoff[c + 1] - x0);
        P = poff[c + 1] - poff[c];
        Xp += x0 * DP;
        knn += (long long)poff[c] * kKnn;
        prank += poff[c];
        if (P == 0) return;   // the whole workgroup
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool mine = tid < P;
    float x[D];
    const long long row = mine ? (long long)tid * n / P : 0;
#pragma unroll
    for (int k4 = 0; k4 < D / 4; ++k4) {
        const float4 v = *reinterpret_cast<const float4*>(Xp + row * DP + 4 * k4);
        pc[k4][tid] = v;
        x[4 * k4] = v.x;
        x[4 * k4 + 1] = v.y;
        x[4 * k4 + 2] = v.z;
        x[4 * k4 + 3] = v.w;
    }
#pragma unroll
    for (int t = 0; t < kKnn; ++t) lst[t * 1024 + tid] = mine ? (short)knn[tid * kKnn + t] : (short)-1;
    taken[tid] = tid == 0 ? 1 : 0;
    if (tid == 0) {
        rk[0] = 0;
        s_cur = 0;
        s_step = 1;
    }
    __syncthreads();
    int cur = 0, step = 1;   // wave 0's walk state
    for (;;) {
        if (wave == 0) {
            while (step < P) {
                const int c = lane < kKnn ? lst[lane * 1024 + cur] : -1;
                const bool fr = c >= 0 && !taken[c < 0 ? 0 : c];
                const unsigned long long bal = __ballot(fr);
                if (!bal) break;
                const int nx = __builtin_amdgcn_readlane(c, __builtin_ctzll(bal));
                if (lane == 0) {
                    taken[nx] = 1;
                    rk[nx] = step;
                }
                cur = nx;
                ++step;
            }
            if (lane == 0) {
                s_cur = cur;
                s_step = step;
            }
        }
        __syncthreads();
        const int c0 = s_cur, st = s_step;
        if (st >= P) break;
        // every listed pivot is taken: the nearest untaken one over all
        float q = 0.0f;
#pragma unroll
        for (int k4 = 0; k4 < D / 4; ++k4) {
            const float4 v = pc[k4][c0];
            const float t0 = x[4 * k4] - v.x, t1 = x[4 * k4 + 1] - v.y;
            const float t2 = x[4 * k4 + 2] - v.z, t3 = x[4 * k4 + 3] - v.w;
            q = fmaf(t0, t0, q);
            q = fmaf(t1, t1, q);
            q = fmaf(t2, t2, q);
            q = fmaf(t3, t3, q);
        }
        unsigned long long key = (mine && !taken[tid]) ? ((unsigned long long)__float_as_uint(q) << 32) | (unsigned)tid : ~0ull;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off);
            key = o < key ? o : key;
        }
        if (lane == 0) wbest[wave] = key;
        __syncthreads();
        if (wave == 0) {
            unsigned long long b = wbest[0];
#pragma unroll
            for (int w = 1; w < 16; ++w) b = wbest[w] < b ? wbest[w] : b;
            const int nx = (int)(unsigned)b;
            if (lane == 0) {
                taken[nx] = 1;
                rk[nx] = st;
            }
            cur = nx;
            step = st + 1;
        }
    }
    if (mine) prank[tid] = rk[tid];
}

// Per 256-point block of the sorted points: centre = midpoint of the bounding
// box, radius = max distance of a block point from the centre (FP32, rounded
// up slightly so that it bounds the FP32 distances the step computes).
// geom row (geom_stride(D) floats): centre[0..D); radius at [4] for D <= 4,
// at [D] for larger D, followed there by the centre's norm at [D + 1].
__global__ __launch_bounds__(256) void block_geom_kernel(const float* __restrict__ Xs, int n, int DP,
                                                         int D, int gs, float* geom) {
    __shared__ float red[256];
    __shared__ float ctr[64];
    const int b = blockIdx.x;
    const int i = b * 256 + threadIdx.x;
    const bool live = i < n;
    for (int k = 0; k < D; ++k) {
        const float v = live ? Xs[(long long)i * DP + k] : 0.0f;
        red[threadIdx.x] = live ? v : __builtin_inff();
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] = fminf(red[threadIdx.x], red[threadIdx.x + off]);
            __syncthreads();
        }
        const float lo = red[0];
        __syncthreads();
        red[threadIdx.x] = live ? v : -__builtin_inff();
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
            __syncthreads();
        }
        if (threadIdx.x == 0) ctr[k] = 0.5f * (lo + red[0]);
        __syncthreads();
    }
    float r2 = 0.0f;
    if (live)
        for (int k = 0; k < D; ++k) {
            const float t = Xs[(long long)i * DP + k] - ctr[k];
            r2 = fmaf(t, t, r2);
        }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    const float radius = sqrtf(red[0]) * 1.0001f + 1e-30f;
    float* g = geom + (long long)b * gs;
    const int rpos = D <= 4 ? 4 : D;
    for (int e = threadIdx.x; e < gs; e += 256) {
        float v = 0.0f;
        if (e < D) v = ctr[e];
        else if (e == rpos) v = radius;
        else if (e == rpos + 1 && D > 4) {
            float c2 = 0.0f;
            for (int k = 0; k < D; ++k) c2 = fmaf(ctr[k], ctr[k], c2);
            v = sqrtf(c2) * 1.0001f;
        }
        g[e] = v;
    }
}

}  // namespace

namespace {

// Sort workspace: the point bounds first (fixed offset, so a later seed sort
// can use the bounds of the points), digit totals, then keys/values x2 and the
// per-block histogram sized for `count` elements.
struct SortWs {
    float* bnd;
    int* dtot;
    unsigned* k0;
    unsigned* k1;
    int* v0;
    int* v1;
    unsigned long long* best;   // nearest pivot per row (count)
    int* hist;
};

// bounds: 2D final + 2D per bounds block (256 blocks), D <= 32; then the
// frame shift (32 floats)
constexpr size_t kShiftOff = 2 * 32 + 2 * 32 * 256;
constexpr size_t kRankOff = kShiftOff + 64;        // chain rank of each pivot (1024 ints)
constexpr size_t kBndFloats = kRankOff + 1024;

// the nearest-pivot keys (8 bytes per row), first used for the pivots'
// neighbour lists (kKnn ints per pivot, at most 1,024 pivots)
size_t best_bytes(int count) {
    const size_t a = (size_t)count * 8, b = (size_t)1024 * kKnn * 4;
    return a > b ? a : b;
}

SortWs carve(void* ws, int count) {
    SortWs w;
    char* p = (char*)ws;
    w.bnd = (float*)p; p += kBndFloats * 4;
    w.dtot = (int*)p; p += 4 * 256 * 4;
    w.k0 = (unsigned*)p; p += (size_t)count * 4;
    w.k1 = (unsigned*)p; p += (size_t)count * 4;
    w.v0 = (int*)p; p += (size_t)count * 4;
    w.v1 = (int*)p; p += (size_t)count * 4;
    w.best = (unsigned long long*)p; p += best_bytes(count);
    w.hist = (int*)p;
    return w;
}

// Stable sort of (k0, v0) by the 32-bit keys, four 8-bit passes; the result
// is back in (k0, v0).
// LSD radix sort of (key, value) pairs on the low 8 * passes bits of the keys;
// returns the array that holds the sorted values (v0 after an even number of
// passes, v1 after an odd one).
int* radix_sort_pairs(const SortWs& w, int n, hipStream_t s, int passes = 4) {
    const int nblocks = (n + kSortThreads - 1) / kSortThreads;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(4), dim3(256), 0, s, w.dtot, 4 * 256);
    unsigned* ka = w.k0; unsigned* kb = w.k1;
    int* va = w.v0; int* vb = w.v1;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * 8;
        int* dt = w.dtot + pass * 256;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, ka, n, shift,
                           nblocks, w.hist, dt);
        hipLaunchKernelGGL(radix_scan_kernel, dim3(256), dim3(256), 0, s, w.hist, nblocks, dt);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, ka, va, n,
                           shift, nblocks, w.hist, kb, vb);
        unsigned* tk = ka; ka = kb; kb = tk;
        int* tv = va; va = vb; vb = tv;
    }
    return va;
}

}  // namespace

size_t sort_workspace_bytes(int count) {
    const size_t nblocks = (count + kSortThreads - 1) / kSortThreads;
    return kBndFloats * 4 + 4 * 256 * 4 + (size_t)count * 4 * 4 + best_bytes(count) + nblocks * 256 * 4 + 256;
}

// Packed points Xp (n x DP) -> sorted copy Xs, permutation perm (Xs[i] =
// Xp[perm[i]]) and per-256-block geometry (centre, radius).  Leaves the point
// bounds in the workspace for launch_seed_order.
#define FMS_PIVOT_DSWITCH(D_, CALL)                       \
    switch (D_) {                                         \
        case 8: { constexpr int DD = 8; CALL; } break;    \
        case 16: { constexpr int DD = 16; CALL; } break;  \
        case 32: { constexpr int DD = 32; CALL; } break;  \
        default: return hipErrorInvalidValue;             \
    }

int pivot_count(int n) {
    int P = n / 256;
    return P < 1 ? 1 : (P > 1024 ? 1024 : P);
}

hipError_t launch_spatial_sort(const float* Xp, int n, int DP, int D, float* Xs, int* perm,
                               float* geom, void* ws, hipStream_t s) {
    const SortWs w = carve(ws, n);
    const int bblocks = 256;
    hipLaunchKernelGGL(bounds_kernel, dim3(bblocks), dim3(256), 0, s, Xp, n, DP, D, w.bnd);
    hipLaunchKernelGGL(bounds_final_kernel, dim3(1), dim3(256), 0, s, w.bnd, D, bblocks);
    const float* shift = nullptr;
    if (D <= 4) {
        hipLaunchKernelGGL(morton_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Xp, n, DP, D, w.bnd,
                           w.k0, w.v0);
    } else {
        float* sh = w.bnd + kShiftOff;
        hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(64), 0, s, w.bnd, D, sh);
        shift = sh;
        const int P = pivot_count(n);
        int* prank = reinterpret_cast<int*>(w.bnd + kRankOff);
        int* knn = reinterpret_cast<int*>(w.best);   // free until the nearest-pivot search
        FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_knn_kernel<DD>), dim3((P + 63) / 64), dim3(1024), 0, s,
                                                Xp, n, DP, P, knn, nullptr, nullptr));
        FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_chain_kernel<DD>), dim3(1), dim3(1024), 0, s, Xp, n, DP,
                                                P, knn, prank, nullptr, nullptr));
        hipLaunchKernelGGL(fill_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w.best, n, ~0ull);
        FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_near_kernel<DD, kPivChunkPoints>),
                                                dim3((n + 255) / 256, (P + kPivChunkPoints - 1) / kPivChunkPoints),
                                                dim3(256), 0, s, Xp, (long long)n, DP, 1.0f, Xp, n, DP, P, w.best,
                                                CloudRows{}, nullptr, nullptr));
        hipLaunchKernelGGL(pivot_key_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w.best, n, nullptr, prank,
                           w.k0, w.v0);
    }
    // point keys: 24-bit Morton codes (D <= 4) or a far bit, pivot index and
    // distance (1 + 10 + 14 bits)
    const int* sorted = radix_sort_pairs(w, n, s, D <= 4 ? 3 : 4);
    hipError_t e = hipMemcpyAsync(perm, sorted, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)(((long long)n * DP + 255) / 256)), dim3(256),
                       0, s, Xp, DP, D, perm, n, shift, Xs);
    hipLaunchKernelGGL(block_geom_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Xs, n, DP, D,
                       geom_stride(D), geom);
    return hipGetLastError();
}

// ---- many clouds -------------------------------------------------------------

int batched_pivot_count(long long n_cloud) {
    if (n_cloud <= 0) return 0;
    const long long P = n_cloud / 256;
    return (int)(P < 1 ? 1 : (P > kBatchedPivotMax ? kBatchedPivotMax : P));
}

namespace {

// Batched sort workspace: the sort's (as for `count` rows), then the pivots'
// neighbour lists and chain ranks.
size_t bws_sort_bytes(int count) {
    const size_t nblocks = (count + kSortThreads - 1) / kSortThreads;
    return kBndFloats * 4 + 4 * 256 * 4 + (size_t)count * 4 * 4 + (size_t)count * 8 + nblocks * 256 * 4 + 256;
}

SortWs carve_batched(void* ws, int count, int ptot, int** knn, int** prank) {
    SortWs w;
    char* p = (char*)ws;
    w.bnd = (float*)p; p += kBndFloats * 4;
    w.dtot = (int*)p; p += 4 * 256 * 4;
    w.k0 = (unsigned*)p; p += (size_t)count * 4;
    w.k1 = (unsigned*)p; p += (size_t)count * 4;
    w.v0 = (int*)p; p += (size_t)count * 4;
    w.v1 = (int*)p; p += (size_t)count * 4;
    w.best = (unsigned long long*)p; p += (size_t)count * 8;
    w.hist = (int*)p;
    p = (char*)ws + bws_sort_bytes(count);
    *knn = (int*)p; p += (size_t)ptot * kKnn * 4;
    *prank = (int*)p;
    return w;
}

}  // namespace

size_t batched_sort_workspace_bytes(int count, int ptot) {
    return bws_sort_bytes(count) + (size_t)ptot * (kKnn + 1) * 4 + 256;
}

hipError_t launch_batched_sort(const float* Xp, int n, int D, const CloudRows& pts, const int32_t* poff, int ptot,
                               float* Xs, void* ws, int count, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > count) return hipErrorInvalidValue;
    int *knn, *prank;
    const SortWs w = carve_batched(ws, count, ptot, &knn, &prank);
    const int ncl = pts.ncl;
    const dim3 pgroups((kBatchedPivotMax + 63) / 64, ncl);
    FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_knn_kernel<DD>), pgroups, dim3(1024), 0, s, Xp, 0, D, 0, knn,
                                            pts.roff, poff));
    FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_chain_kernel<DD>), dim3(ncl), dim3(1024), 0, s, Xp, 0, D, 0,
                                            knn, prank, pts.roff, poff));
    hipLaunchKernelGGL(fill_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w.best, n, ~0ull);
    const dim3 ngrid(pts.tiles, (kBatchedPivotMax + kPivChunkPoints - 1) / kPivChunkPoints);
    FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_near_kernel<DD, kPivChunkPoints>), ngrid, dim3(256), 0, s, Xp,
                                            (long long)n, D, 1.0f, Xp, 0, D, 0, w.best, pts, pts.roff, poff));
    hipLaunchKernelGGL(bpivot_key_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w.best, (long long)n, nullptr,
                       pts.roff, ncl, poff, prank, w.k0, w.v0);
    const int* sorted = radix_sort_pairs(w, n, s, 4);
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)(((long long)n * D + 255) / 256)), dim3(256), 0, s, Xp,
                       D, D, sorted, n, nullptr, Xs);
    return hipGetLastError();
}

hipError_t launch_batched_seed_order(const float* S, int DP, int D, int M, float scale, const uint8_t* status,
                                     const CloudRows& seeds, const float* Xp, const CloudRows& pts,
                                     const int32_t* poff, void* ws, int count, int ptot, int32_t* act0,
                                     hipStream_t s) {
    if (M <= 0) return hipSuccess;
    if (M > count) return hipErrorInvalidValue;
    int *knn, *prank;
    // the ranks the point sort left (sized for `count` rows there too)
    SortWs w = carve_batched(ws, count, ptot, &knn, &prank);
    hipLaunchKernelGGL(fill_u64_kernel, dim3((M + 255) / 256), dim3(256), 0, s, w.best, M, ~0ull);
    const dim3 ngrid(seeds.tiles, (kBatchedPivotMax + kPivChunk - 1) / kPivChunk);
    if (seeds.tiles > 0)
        FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_near_kernel<DD>), ngrid, dim3(256), 0, s, S, (long long)M,
                                                DP, scale, Xp, 0, D, 0, w.best, seeds, pts.roff, poff));
    hipLaunchKernelGGL(bpivot_key_kernel, dim3((M + 255) / 256), dim3(256), 0, s, w.best, (long long)M, status,
                       seeds.roff, seeds.ncl, poff, prank, w.k0, w.v0);
    const int* sorted = radix_sort_pairs(w, M, s, 4);
    hipError_t e = hipMemcpyAsync(act0, sorted, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

const float* sort_frame_shift(const void* ws) {
    return (const float*)ws + kShiftOff;
}

// Active list of a batch in the order of the seed positions (S in original
// units, `scale` to packed units) -- Morton order for D <= 4, nearest pivot
// of the points Xp for larger D -- active seeds first; the active count in
// the control block is unchanged.  ws: a sort workspace of at least max(n, m)
// elements that launch_spatial_sort filled.
hipError_t launch_seed_order(const float* S, int DP, int D, int m, float scale,
                             const uint8_t* status, void* ws, int32_t* act0, const float* Xp, int n,
                             hipStream_t s) {
    if (m < 2) return hipSuccess;
    const SortWs w = carve(ws, m);
    if (D > 4) {
        const int P = pivot_count(n);
        const int* prank = reinterpret_cast<const int*>(w.bnd + kRankOff);   // from launch_spatial_sort
        hipLaunchKernelGGL(fill_u64_kernel, dim3((m + 255) / 256), dim3(256), 0, s, w.best, m, ~0ull);
        FMS_PIVOT_DSWITCH(D, hipLaunchKernelGGL((pivot_near_kernel<DD>),
                                                dim3((m + 255) / 256, (P + kPivChunk - 1) / kPivChunk), dim3(256), 0,
                                                s, S, (long long)m, DP, scale, Xp, n, DP, P, w.best, CloudRows{},
                                                nullptr, nullptr));
        hipLaunchKernelGGL(pivot_key_kernel, dim3((m + 255) / 256), dim3(256), 0, s, w.best, m, status, prank,
                           w.k0, w.v0);
    }
    if (m <= kSeedSortMax) {
        hipLaunchKernelGGL(seed_order_small_kernel, dim3(1), dim3(1024), 0, s, S, DP, D, m, scale,
                           status, w.bnd, D > 4 ? w.k0 : nullptr, act0);
        return hipGetLastError();
    }
    if (D <= 4)
        hipLaunchKernelGGL(seed_key_kernel, dim3((m + 255) / 256), dim3(256), 0, s, S, DP, D, m, scale,
                           status, w.bnd, w.k0, w.v0);
    const int* sorted = radix_sort_pairs(w, m, s);
    hipError_t e = hipMemcpyAsync(act0, sorted, (size_t)m * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace fms
