// k_merge.hip -- round epilogue kernels: seed gather from the pool, greedy
// mode merging ("prune modes", Algorithms 1-2), pool coverage and stable
// pool compaction, for gfx950.
//
// Merge rule (greedy, in draw order): a converged seed joins the first mode
// (lowest index) within r = merge_radius*h, else it founds a new mode at its
// own final position.  Modes of earlier rounds precede every new one.
//
// The sequential rule is evaluated in parallel passes.  A seed i is decided
// as soon as the first seed j < i (in index order) that lies within r and is
// a founder or still undecided is a founder (i joins j), or when there is no
// such j (i founds a mode).  The lowest undecided seed is always decidable,
// every decision is final, and a stale read of "undecided" only postpones a
// decision, so the passes reproduce the sequential greedy result exactly.

#include "fms_internal.h"

namespace fms {

namespace {

constexpr int kT = 256;

__global__ void iota_kernel(int32_t* a, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = i;
}

__global__ void fill_u8_kernel(uint8_t* a, int n, uint8_t v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

template <int D>
__device__ __forceinline__ float dist2(const float* a, const float* b) {
    float q = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float t = a[k] - b[k];
        q = fmaf(t, t, q);
    }
    return q;
}

constexpr int kWavesT = kT / 64;

// One wave per seed from here on: the lanes test 64 candidates at a time and
// a ballot picks the first (lowest index) hit.

// One decision pass.  Joined-to-batch-seed j is stored as K_old + j.  Every
// state starts as MG_UNDECIDED (set when the round starts); the first pass
// also settles seeds that did not converge (MG_SKIP) and seeds within r of an
// old mode (the index of the first such mode).  A state another wave has not
// settled yet reads as undecided, which only postpones a decision.
template <int D, bool kFirst>
__global__ __launch_bounds__(kT) void decide_kernel(const float* __restrict__ S, int DP,
                                                    const uint8_t* __restrict__ status, int B,
                                                    const float* __restrict__ modes, int K_old, int k_scan,
                                                    float r2, int32_t* state, int32_t* und_counter) {
    const int i = blockIdx.x * kWavesT + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= B) return;
    if (kFirst && status[i] != ST_CONVERGED) {
        if (lane == 0) __atomic_store_n(&state[i], (int32_t)MG_SKIP, __ATOMIC_RELAXED);
        return;
    }
    // (a seed the block join matched to an old mode is decided already)
    if (__atomic_load_n(&state[i], __ATOMIC_RELAXED) != MG_UNDECIDED) return;
    float si[D];
#pragma unroll
    for (int k = 0; k < D; ++k) si[k] = S[(long long)i * DP + k];
    if (kFirst) {
        for (int base = 0; base < k_scan; base += 64) {
            const int j = base + lane;
            bool hit = false;
            if (j < k_scan) hit = dist2<D>(si, modes + (long long)j * DP) <= r2;
            const unsigned long long bal = __ballot(hit);
            if (bal) {
                if (lane == 0)
                    __atomic_store_n(&state[i], (int32_t)(base + __ffsll((unsigned long long)bal) - 1),
                                     __ATOMIC_RELAXED);
                return;
            }
        }
    }
    int result = MG_FOUNDER;   // unless an earlier founder or undecided seed is within r
    for (int base = 0; base < i; base += 64) {
        const int j = base + lane;
        int sj = MG_SKIP;
        bool hit = false;
        if (j < i) {
            sj = __atomic_load_n(&state[j], __ATOMIC_RELAXED);
            if (sj == MG_FOUNDER || sj == MG_UNDECIDED) hit = dist2<D>(si, S + (long long)j * DP) <= r2;
        }
        const unsigned long long bal = __ballot(hit);
        if (bal) {
            const int first = __ffsll((unsigned long long)bal) - 1;
            const int sf = __shfl(sj, first);
            result = (sf == MG_FOUNDER) ? (K_old + base + first) : MG_UNDECIDED;
            break;
        }
    }
    if (lane == 0) {
        if (result != MG_UNDECIDED) __atomic_store_n(&state[i], result, __ATOMIC_RELAXED);
        else atomicAdd(und_counter, 1);
    }
}

// Tiled form of one decision pass, for large batches (the degenerate case of
// a window so narrow that every seed founds a mode makes every seed scan
// every mode and every earlier seed).  A workgroup takes kT consecutive
// seeds, one per lane, and streams the old modes (first pass) and then the
// earlier seeds through LDS, kDecideRows rows per tile, so that each row is
// read once per workgroup instead of once per seed.  A lane scans a tile in
// index order and stops at its first hit; the workgroup leaves a loop once no
// lane searches.  The decisions are exactly those of decide_kernel: the same
// first-hit rule, and a state staged before another workgroup settles it can
// only read as undecided, which postpones a decision.
constexpr int kDecideRows = 64;
// rows staged per tile: 64, fewer for rows wider than 64 floats (16 KB of LDS)
template <int D>
constexpr int decide_rows() { return D <= 64 ? kDecideRows : (kDecideRows * 64) / D; }
constexpr int kDecideTiledMinBatch = 16384;

template <int D, bool kFirst>
__global__ __launch_bounds__(kT) void decide_tiled_kernel(const float* __restrict__ S, int DP,
                                                          const uint8_t* __restrict__ status, int B,
                                                          const float* __restrict__ modes, int K_old,
                                                          int k_scan, float r2, int32_t* state,
                                                          int32_t* und_counter) {
    constexpr int kRows = decide_rows<D>();
    __shared__ float rows[kRows][D];
    __shared__ int32_t rst[kRows];
    const int i0 = blockIdx.x * kT;
    const int i = i0 + threadIdx.x;
    bool todo = false;   // this lane decides seed i in this pass
    if (i < B) {
        if (kFirst && status[i] != ST_CONVERGED) __atomic_store_n(&state[i], (int32_t)MG_SKIP, __ATOMIC_RELAXED);
        else todo = __atomic_load_n(&state[i], __ATOMIC_RELAXED) == MG_UNDECIDED;
    }
    const bool owner = todo;
    float si[D];
#pragma unroll
    for (int k = 0; k < D; ++k) si[k] = todo ? S[(long long)i * DP + k] : 0.0f;
    int result = MG_FOUNDER;   // unless an old mode or an earlier founder / undecided seed is within r
    if (kFirst) {
        for (int base = 0; base < k_scan; base += kRows) {
            if (!__syncthreads_or(todo)) break;
            const int cnt = min(kRows, k_scan - base);
            for (int e = threadIdx.x; e < cnt * D; e += kT)
                rows[e / D][e % D] = modes[(long long)(base + e / D) * DP + e % D];
            __syncthreads();
            if (todo) {
                for (int q = 0; q < cnt; ++q) {
                    if (dist2<D>(si, rows[q]) <= r2) {
                        result = base + q;
                        todo = false;
                        break;
                    }
                }
            }
        }
    }
    const int ilast = min(i0 + kT, B) - 1;   // the workgroup's last seed: candidates j < ilast
    for (int base = 0; base < ilast; base += kRows) {
        if (!__syncthreads_or(todo)) break;
        const int cnt = min(kRows, ilast - base);
        for (int e = threadIdx.x; e < cnt * D; e += kT)
            rows[e / D][e % D] = S[(long long)(base + e / D) * DP + e % D];
        if (threadIdx.x < cnt) rst[threadIdx.x] = __atomic_load_n(&state[base + threadIdx.x], __ATOMIC_RELAXED);
        __syncthreads();
        if (todo) {
            const int qend = min(cnt, i - base);   // j < i
            for (int q = 0; q < qend; ++q) {
                const int sj = rst[q];
                if ((sj == MG_FOUNDER || sj == MG_UNDECIDED) && dist2<D>(si, rows[q]) <= r2) {
                    result = (sj == MG_FOUNDER) ? (K_old + base + q) : MG_UNDECIDED;
                    todo = false;
                    break;
                }
            }
        }
    }
    if (owner && result != MG_UNDECIDED) __atomic_store_n(&state[i], result, __ATOMIC_RELAXED);
    const unsigned long long und = __ballot(owner && result == MG_UNDECIDED);
    if ((threadIdx.x & 63) == 0 && und) atomicAdd(und_counter, __popcll(und));
}

// After the passes: if every seed is decided, number the founders in seed
// order (mode K_old + q for the q-th founder) and append their positions to
// the mode store; ctl->k_new = K_old + founders.  Otherwise leave the modes
// alone and flag the round for the host (k_new = K_old, merge_host = 1).
// One workgroup; B may exceed its size.
constexpr int kFoundThreads = 1024;
constexpr int kFoundersOneGroup = 1;   // batches of up to 1,024 seeds: the one-workgroup form

__global__ __launch_bounds__(kFoundThreads) void founders_kernel(const float* __restrict__ S, int DP,
                                                                 int B, int K_old,
                                                                 const int32_t* __restrict__ state,
                                                                 float* modes, Ctl* ctl, int und_slot) {
    __shared__ int wsum[kFoundThreads / 64];
    __shared__ int carry_s;
    if (ctl->und[und_slot] > 0) {
        if (threadIdx.x == 0) {
            ctl->k_new = K_old;
            ctl->merge_host = 1;
        }
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < B; base += kFoundThreads) {
        const int i = base + threadIdx.x;
        const bool f = i < B && state[i] == MG_FOUNDER;
        const unsigned long long bal = __ballot(f);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int before = carry_s, total = 0;
        for (int w = 0; w < kFoundThreads / 64; ++w) {
            if (w < wave) before += wsum[w];
            total += wsum[w];
        }
        if (f) {
            const long long q = (long long)K_old + before + __popcll(bal & ((1ull << lane) - 1ull));
            for (int k = 0; k < DP; ++k) modes[q * DP + k] = S[(long long)i * DP + k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl->k_new = K_old + carry_s;
        ctl->merge_host = 0;
    }
}

// Large batches: the same numbering over many workgroups of kFoundThreads
// seeds -- each counts its founders, one workgroup turns the counts into
// offsets (and the new mode count), and each copies its founders' rows to
// their modes, the workgroup's rows contiguous (coalesced stores).
__global__ __launch_bounds__(kFoundThreads) void founders_count_kernel(int B, const int32_t* __restrict__ state,
                                                                       const Ctl* ctl, int und_slot, int32_t* cnt) {
    __shared__ int wsum[kFoundThreads / 64];
    if (ctl->und[und_slot] > 0) return;
    const int i = blockIdx.x * kFoundThreads + threadIdx.x;
    const unsigned long long bal = __ballot(i < B && state[i] == MG_FOUNDER);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kFoundThreads / 64; ++w) t += wsum[w];
        cnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kFoundThreads) void founders_scan_kernel(int nb, int K_old, int32_t* cnt, Ctl* ctl,
                                                                      int und_slot) {
    __shared__ int wsum[kFoundThreads / 64];
    __shared__ int carry_s;
    if (ctl->und[und_slot] > 0) {
        if (threadIdx.x == 0) {
            ctl->k_new = K_old;
            ctl->merge_host = 1;
        }
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += kFoundThreads) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? cnt[i] : 0;
        int incl = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_up(incl, off);
            if (lane >= off) incl += u;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int before = carry_s, total = 0;
        for (int w = 0; w < kFoundThreads / 64; ++w) {
            if (w < wave) before += wsum[w];
            total += wsum[w];
        }
        if (i < nb) cnt[i] = before + incl - v;   // exclusive offset
        __syncthreads();
        if (threadIdx.x == 0) carry_s += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl->k_new = K_old + carry_s;
        ctl->merge_host = 0;
    }
}

__global__ __launch_bounds__(kFoundThreads) void founders_copy_kernel(const float* __restrict__ S, int DP, int B,
                                                                      int K_old, const int32_t* __restrict__ state,
                                                                      const int32_t* __restrict__ off, float* modes,
                                                                      const Ctl* ctl, int und_slot) {
    __shared__ int wsum[kFoundThreads / 64];
    __shared__ int rows[kFoundThreads];   // the workgroup's founders, in seed order
    if (ctl->und[und_slot] > 0) return;
    const int i0 = blockIdx.x * kFoundThreads;
    const int i = i0 + threadIdx.x;
    const bool f = i < B && state[i] == MG_FOUNDER;
    const unsigned long long bal = __ballot(f);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kFoundThreads / 64; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    if (f) rows[before + __popcll(bal & ((1ull << lane) - 1ull))] = i;
    __syncthreads();
    const long long q0 = (long long)K_old + off[blockIdx.x];
    for (int e = threadIdx.x; e < total * DP; e += kFoundThreads) {
        const int r = e / DP, k = e - r * DP;
        modes[(q0 + r) * DP + k] = S[(long long)rows[r] * DP + k];
    }
}

constexpr int kModeTile = 256;

// Pool coverage: entries of the pool list within r of a new mode [k0, k1)
// are marked removed (k1 is read from the control block when ctl is given).
// Workgroups are the compaction blocks: each also writes how many of its
// entries stay in the pool.
template <int D>
__global__ __launch_bounds__(kCompactBlock) void cover_kernel(
    const float* __restrict__ X, int d, const int32_t* __restrict__ pool, int len,
    const float* __restrict__ modes, int DP, int k0, int k1, const Ctl* ctl, float r2,
    uint8_t* removed, int32_t* block_cnt) {
    constexpr int kTile = D <= 64 ? kModeTile : (kModeTile * 64) / D;   // at most 64 KB of LDS
    // rows up to 64 floats stay in registers; wider ones are read from memory
    // at each distance (1,024 threads leave 128 registers per lane)
    constexpr int RD = D <= 64 ? D : 1;
    __shared__ float tileM[kTile * D];
    __shared__ int wsum[kCompactBlock / 64];
    if (ctl) k1 = ctl->k_new;
    const int e = blockIdx.x * kCompactBlock + threadIdx.x;
    bool todo = e < len && !removed[e];
    const long long id = todo ? pool[e] : 0;
    float x[RD];
#pragma unroll
    for (int k = 0; k < RD; ++k) x[k] = (todo && k < d) ? X[id * d + k] : 0.0f;
    bool hit = false;
    for (int base = k0; base < k1; base += kTile) {
        if (__syncthreads_and(!todo || hit)) break;
        const int cnt = min(kTile, k1 - base);
        for (int q = threadIdx.x; q < cnt * D; q += kCompactBlock)
            tileM[q] = modes[(long long)(base + q / D) * DP + q % D];
        __syncthreads();
        if (todo && !hit) {
            for (int j = 0; j < cnt; ++j) {
                float q2;
                if constexpr (D <= 64) {
                    q2 = dist2<D>(x, tileM + j * D);
                } else {
                    q2 = 0.0f;   // padded coordinates of the modes are zero
                    for (int k = 0; k < D; ++k) {
                        const float t = (k < d ? X[id * d + k] : 0.0f) - tileM[j * D + k];
                        q2 = fmaf(t, t, q2);
                    }
                }
                if (q2 <= r2) {
                    hit = true;
                    break;
                }
            }
        }
    }
    if (todo && hit) removed[e] = 1;
    const unsigned long long bal = __ballot(todo && !hit);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int w = 0; w < kCompactBlock / 64; ++w) c += wsum[w];
        block_cnt[blockIdx.x] = c;
    }
}



// Exclusive scan of the block counts by one workgroup; writes the total.
__global__ __launch_bounds__(1024) void compact_scan_kernel(int32_t* block_cnt, int nb,
                                                            int32_t* total) {
    __shared__ int32_t buf[1024];
    int carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int e = base + threadIdx.x;
        const int v = e < nb ? block_cnt[e] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (e < nb) block_cnt[e] = carry + buf[threadIdx.x] - v;
        const int blk_total = buf[1023];
        __syncthreads();
        carry += blk_total;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kCompactBlock) void compact_scatter_kernel(
    const int32_t* __restrict__ pool_in, uint8_t* removed, int len,
    const int32_t* __restrict__ block_off, int32_t* pool_out) {
    __shared__ int wbase[kCompactBlock / 64];
    const int e = blockIdx.x * kCompactBlock + threadIdx.x;
    const bool keep = e < len && !removed[e];
    if (e < len && !keep) removed[e] = 0;   // leaves the flags clear for the next round
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long b = __ballot(keep);
    if (lane == 0) wbase[w] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int q = 0; q < kCompactBlock / 64; ++q) {
            int c = wbase[q];
            wbase[q] = s;
            s += c;
        }
    }
    __syncthreads();
    if (keep)
        pool_out[block_off[blockIdx.x] + wbase[w] + __popcll(b & ((1ull << lane) - 1ull))] =
            pool_in[e];
}

}  // namespace

hipError_t launch_iota(int32_t* a, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* a, int n, uint8_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u8_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, n, v);
    return hipGetLastError();
}

#define FMS_DSWITCH(D_, CALL)                                 \
    switch (D_) {                                             \
        case 1: { constexpr int DD = 1; CALL; } break;        \
        case 2: { constexpr int DD = 2; CALL; } break;        \
        case 3: { constexpr int DD = 3; CALL; } break;        \
        case 4: { constexpr int DD = 4; CALL; } break;        \
        case 8: { constexpr int DD = 8; CALL; } break;        \
        case 16: { constexpr int DD = 16; CALL; } break;      \
        case 32: { constexpr int DD = 32; CALL; } break;      \
        case 64: { constexpr int DD = 64; CALL; } break;      \
        case 128: { constexpr int DD = 128; CALL; } break;    \
        case 256: { constexpr int DD = 256; CALL; } break;    \
        default: return hipErrorInvalidValue;                 \
    }

hipError_t launch_merge_decide_pass(const float* S, int DP, int d, const uint8_t* status, int B,
                                    const float* modes, int K_old, int k_scan, float r2, int32_t* state,
                                    int32_t* und_counter, bool first, hipStream_t s) {
    const int D = step_shape(d).D;
    if (B <= 0) return hipSuccess;
    if (B >= kDecideTiledMinBatch) {
        const dim3 tgrid((B + kT - 1) / kT);
        if (first) {
            FMS_DSWITCH(D, hipLaunchKernelGGL((decide_tiled_kernel<DD, true>), tgrid, dim3(kT), 0, s, S, DP,
                                              status, B, modes, K_old, k_scan, r2, state, und_counter));
        } else {
            FMS_DSWITCH(D, hipLaunchKernelGGL((decide_tiled_kernel<DD, false>), tgrid, dim3(kT), 0, s, S, DP,
                                              status, B, modes, K_old, k_scan, r2, state, und_counter));
        }
        return hipGetLastError();
    }
    const dim3 grid((B + kWavesT - 1) / kWavesT);
    if (first) {
        FMS_DSWITCH(D, hipLaunchKernelGGL((decide_kernel<DD, true>), grid, dim3(kT), 0, s, S, DP,
                                          status, B, modes, K_old, k_scan, r2, state, und_counter));
    } else {
        FMS_DSWITCH(D, hipLaunchKernelGGL((decide_kernel<DD, false>), grid, dim3(kT), 0, s, S, DP,
                                          status, B, modes, K_old, k_scan, r2, state, und_counter));
    }
    return hipGetLastError();
}

hipError_t launch_merge_founders(const float* S, int DP, int B, int K_old, const int32_t* state,
                                 float* modes, Ctl* ctl, int und_slot, int32_t* block_tmp, hipStream_t s) {
    const int nb = (B + kFoundThreads - 1) / kFoundThreads;
    if (nb <= kFoundersOneGroup || !block_tmp) {
        hipLaunchKernelGGL(founders_kernel, dim3(1), dim3(kFoundThreads), 0, s, S, DP, B, K_old, state,
                           modes, ctl, und_slot);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(founders_count_kernel, dim3(nb), dim3(kFoundThreads), 0, s, B, state, ctl, und_slot,
                       block_tmp);
    hipLaunchKernelGGL(founders_scan_kernel, dim3(1), dim3(kFoundThreads), 0, s, nb, K_old, block_tmp, ctl,
                       und_slot);
    hipLaunchKernelGGL(founders_copy_kernel, dim3(nb), dim3(kFoundThreads), 0, s, S, DP, B, K_old, state,
                       block_tmp, modes, ctl, und_slot);
    return hipGetLastError();
}

hipError_t launch_cover(const float* X, int d, const int32_t* pool, int len, const float* modes,
                        int k0, int k1, const Ctl* ctl, float r2, uint8_t* removed,
                        int32_t* block_cnt, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    const StepShape sh = step_shape(d);
    FMS_DSWITCH(sh.D, hipLaunchKernelGGL((cover_kernel<DD>), dim3((len + kCompactBlock - 1) / kCompactBlock),
                                         dim3(kCompactBlock), 0, s, X, d, pool, len, modes, sh.DP,
                                         k0, k1, ctl, r2, removed, block_cnt));
    return hipGetLastError();
}

int pool_compact_blocks(int len) { return (len + kCompactBlock - 1) / kCompactBlock; }

hipError_t launch_pool_compact(const int32_t* pool_in, uint8_t* removed, int len,
                               int32_t* pool_out, int32_t* block_tmp, Ctl* ctl, hipStream_t s) {
    const int nb = pool_compact_blocks(len);
    if (nb == 0) {
        hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(1024), 0, s, block_tmp, 0,
                           &ctl->pool_len);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(1024), 0, s, block_tmp, nb,
                       &ctl->pool_len);
    hipLaunchKernelGGL(compact_scatter_kernel, dim3(nb), dim3(kCompactBlock), 0, s, pool_in,
                       removed, len, block_tmp, pool_out);
    return hipGetLastError();
}

}  // namespace fms
