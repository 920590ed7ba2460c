// k_join.hip -- block join of two row sets in spatial order (gfx950), for the
// round epilogue and the labelling when both sides are large: a window so
// narrow that nearly every seed founds its own mode leaves K close to n, and
// every seed, pool point and point would otherwise scan every mode.
//
// Each side is indexed once: its rows in the spatial order of the step
// (Morton code for d <= 4, pivot chain above), copied unchanged, with their
// original indices, each row's distance rho to its block's centre, and a
// bounding ball (bounding-box midpoint, largest distance) per block of 256
// rows.  A workgroup takes one block of 256 queries, one per lane, and visits
// only the row blocks whose ball can come within the lane's reach (the merge or coverage radius; when labelling, the
// lane's smallest distance so far, or its second smallest when the margin is
// asked for); there a row whose rho differs from the query's distance to the
// centre by more than the reach is passed over (the triangle inequality:
// blocks of scattered rows have balls that hold every query), and for the
// others it computes the FP32
// distances exactly as the brute-force kernels do (direct differences, the
// same order of operations, the same inputs), so the decisions are the same:
//   nearest (labels): the smallest (distance, mode index), ties to the lowest
//     index, and the second smallest distance for the margin;
//   first (merge against the old modes, Algorithms 1-2): the lowest mode
//     index within r of a converged seed;
//   any (pool coverage): whether a point lies within r of a new mode (a
//     batch seed that founded one);
//   decide (one merge decision pass among the seeds of a batch): the lowest
//     earlier seed j < i within r whose state is founder or undecided; if it
//     is a founder seed i joins it, if it is undecided i waits for the next
//     pass, and with no such j seed i founds a mode.  This is the rule of
//     the brute-force passes: a state read before another workgroup settles
//     it can only read as undecided, which postpones a decision.
// Every result is a minimum or an OR over the candidates, so the order in
// which row blocks are visited changes nothing.

#include "fms_internal.h"

namespace fms {

namespace {

constexpr int kJB = 256;   // rows per block, on both sides

__global__ void join_pack_kernel(const float* __restrict__ src, int count, int ld, int d, int DP, float scale,
                                 float* out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)count * DP) return;
    const long long r = e / DP;
    const int k = (int)(e % DP);
    out[e] = k < d ? src[r * ld + k] * scale : 0.0f;
}

// Rows in sorted order (unchanged values, zero beyond d) and the ball of
// each block: one workgroup per block.
template <int D>
__global__ __launch_bounds__(kJB) void join_gather_kernel(const float* __restrict__ src, int count, int ld, int d,
                                                          int DP, const int32_t* __restrict__ perm, float* rows,
                                                          float* ball, float* rho) {
    __shared__ float lo[kJB / 64][D], hi[kJB / 64][D], ctr[D];
    __shared__ float rmax[kJB / 64];
    const int blk = blockIdx.x;
    const int i = blk * kJB + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool live = i < count;
    const long long row = live ? perm[i] : 0;
    float x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = (live && k < d) ? src[row * ld + k] : 0.0f;
    if (live)
        for (int k = 0; k < DP; ++k) rows[(long long)i * DP + k] = k < D ? x[k] : 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float a = live ? x[k] : __builtin_inff(), b = live ? x[k] : -__builtin_inff();
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a = fminf(a, __shfl_xor(a, off));
            b = fmaxf(b, __shfl_xor(b, off));
        }
        if (lane == 0) {
            lo[wave][k] = a;
            hi[wave][k] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < D) {
        float a = lo[0][threadIdx.x], b = hi[0][threadIdx.x];
        for (int w = 1; w < kJB / 64; ++w) {
            a = fminf(a, lo[w][threadIdx.x]);
            b = fmaxf(b, hi[w][threadIdx.x]);
        }
        ctr[threadIdx.x] = 0.5f * (a + b);
    }
    __syncthreads();
    float r2 = 0.0f;
    if (live)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float t = x[k] - ctr[k];
            r2 = fmaf(t, t, r2);
        }
    if (live) rho[i] = sqrtf(r2);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) r2 = fmaxf(r2, __shfl_xor(r2, off));
    if (lane == 0) rmax[wave] = r2;
    __syncthreads();
    float* g = ball + (long long)blk * (D + 4);
    if (threadIdx.x < D) g[threadIdx.x] = ctr[threadIdx.x];
    if (threadIdx.x == 0) {
        float m = rmax[0];
        for (int w = 1; w < kJB / 64; ++w) m = fmaxf(m, rmax[w]);
        // rounded up slightly, so that it bounds the FP32 distances
        g[D] = sqrtf(m) * 1.0001f + 1e-30f;
    }
}

struct JoinArgs {
    JoinIndex q, r;
    int DP;
    float r2;
    // nearest: written at the query's original index; cand (optional): a row
    // index per query (or -1) whose distance starts the search, read from
    // rows_orig (stride DP)
    int32_t* labels;
    float* margin;
    const int32_t* cand;
    const float* rows_orig;
    // first: the queries are batch seeds; only converged seeds whose state is
    // still undecided are searched, and a hit writes the mode index
    const uint8_t* status;
    int32_t* state;
    // any: the rows are batch seeds, used where rstate == MG_FOUNDER; nothing
    // is done while the decision passes left a seed undecided (the host then
    // merges and covers)
    const int32_t* rstate;
    const Ctl* ctl;
    int und_slot;
    uint8_t* covered;
    // decide: queries and rows are the batch seeds; founders join as K_old + j
    int K_old;
    bool first_pass;
    int32_t* und_counter;
};

// FP32 squared distance, the order of operations of the brute-force kernels
template <int D>
__device__ __forceinline__ float jdist2(const float (&a)[D], const float* b) {
    float q = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float t = a[k] - b[k];
        q = fmaf(t, t, q);
    }
    return q;
}

// A lower bound (with FP32 slack) on the squared distance from x to any row
// of a ball, compared with a reach: true if the ball may hold a row within it.
template <int D>
__device__ __forceinline__ float centre_dist(const float (&x)[D], const float* c) {
    float q = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float t = x[k] - c[k];
        q = fmaf(t, t, q);
    }
    return sqrtf(q);
}

__device__ __forceinline__ bool ball_reaches(float dxc, float R, float reach) {
    const float lb = dxc * (1.0f - 1e-5f) - R;
    return !(lb > 0.0f && lb * lb > reach * 1.001f + 1e-30f);
}

template <int D, int OP>
__global__ __launch_bounds__(kJB) void join_kernel(JoinArgs a) {
    __shared__ float tile[kJB][D];
    __shared__ int32_t tid_of[kJB];
    __shared__ float rho_of[kJB];
    __shared__ int32_t tst_of[OP == JOIN_DECIDE ? kJB : 1];
    __shared__ float cq[D];
    __shared__ unsigned long long wkey[kJB / 64];
    __shared__ float wmax[kJB / 64];
    if (OP == JOIN_ANY && a.ctl->und[a.und_slot] > 0) return;
    const int qb = blockIdx.x;
    const int qi = qb * kJB + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool live = qi < a.q.count;
    const int qid = live ? a.q.idx[qi] : 0;
    float x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = live ? a.q.rows[(long long)qi * a.DP + k] : 0.0f;
    if (OP == JOIN_FIRST)
        live = live && a.status[qid] == ST_CONVERGED && __atomic_load_n(&a.state[qid], __ATOMIC_RELAXED) == MG_UNDECIDED;
    if (OP == JOIN_DECIDE && live) {
        if (a.first_pass && a.status[qid] != ST_CONVERGED) {
            __atomic_store_n(&a.state[qid], (int32_t)MG_SKIP, __ATOMIC_RELAXED);
            live = false;
        } else {
            live = __atomic_load_n(&a.state[qid], __ATOMIC_RELAXED) == MG_UNDECIDED;
        }
    }
    const bool owner = live;
    if (threadIdx.x < D) cq[threadIdx.x] = a.q.ball[(long long)qb * (D + 4) + threadIdx.x];
    const float Rq = a.q.ball[(long long)qb * (D + 4) + D];
    const int nbr = (a.r.count + kJB - 1) / kJB;
    float best = __builtin_inff(), second = __builtin_inff();
    int arg = 0x7fffffff, first = 0x7fffffff;
    int32_t fst = MG_UNDECIDED;   // decide: the state of `first` as read
    bool hit = false;
    __syncthreads();
    float cqv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) cqv[k] = cq[k];

    // the lanes' candidates among the rows of block b
    // dxc: the lane's distance to the block's centre
    auto scan = [&](int b, bool need, float dxc) {
        const int base = b * kJB;
        const int cnt = min(kJB, a.r.count - base);
        __syncthreads();   // the previous block is no longer read
        for (int e = threadIdx.x; e < cnt * D; e += kJB)
            tile[e / D][e % D] = a.r.rows[(long long)(base + e / D) * a.DP + e % D];
        if (threadIdx.x < cnt) {
            rho_of[threadIdx.x] = a.r.rho[base + threadIdx.x];
            int id = a.r.idx[base + threadIdx.x];
            if (OP == JOIN_ANY && a.rstate[id] != MG_FOUNDER) id = -1;
            if (OP == JOIN_DECIDE) {
                // candidates: founders and undecided seeds (-1 - state keeps
                // which); a state read now can only be stale as undecided
                const int32_t st = __atomic_load_n(&a.state[id], __ATOMIC_RELAXED);
                tst_of[threadIdx.x] = st;
                if (st != MG_FOUNDER && st != MG_UNDECIDED) id = -1;
            }
            tid_of[threadIdx.x] = id;
        }
        __syncthreads();
        if (!need) return;
        const float dlo = dxc * (1.0f - 1e-5f), dhi = dxc * (1.0f + 1e-5f);
        for (int j = 0; j < cnt; ++j) {
            const int id = tid_of[j];
            if ((OP == JOIN_ANY || OP == JOIN_DECIDE) && id < 0) continue;
            {
                // |x - r| >= |dxc - rho|, with FP32 slack on both sides
                const float rh = rho_of[j];
                const float g = fmaxf(dlo - rh * (1.0f + 1e-5f), rh * (1.0f - 1e-5f) - dhi);
                const float reach = OP == JOIN_NEAREST ? (a.margin ? second : best) : a.r2;
                if (g > 0.0f && g * g > reach * 1.001f + 1e-30f) continue;
            }
            const float dd = jdist2<D>(x, tile[j]);
            if (OP == JOIN_NEAREST) {
                if (id == arg) continue;   // the starting candidate, already counted
                if (dd < best || (dd == best && id < arg)) {
                    second = best;
                    best = dd;
                    arg = id;
                } else if (dd < second) {
                    second = dd;
                }
            } else if (OP == JOIN_FIRST) {
                if (dd <= a.r2 && id < first) first = id;
            } else if (OP == JOIN_DECIDE) {
                if (id >= 0 && id < qid && id < first && dd <= a.r2) {
                    first = id;
                    fst = tst_of[j];
                }
            } else {
                if (dd <= a.r2) {
                    hit = true;
                    break;
                }
            }
        }
    };

    int b0 = -1;
    float wreach = a.r2;
    if (OP == JOIN_NEAREST && a.cand && live) {
        const int c0 = a.cand[qid];
        if (c0 >= 0) {
            best = jdist2<D>(x, a.rows_orig + (long long)c0 * a.DP);
            arg = c0;
        }
    }
    if (OP == JOIN_NEAREST) {
        // the row block whose centre is nearest the query block's centre
        // first: its rows bound every lane's second distance
        unsigned long long key = ~0ull;
        for (int b = threadIdx.x; b < nbr; b += kJB) {
            const float* c = a.r.ball + (long long)b * (D + 4);
            const float q = jdist2<D>(cqv, c);
            const unsigned long long k2 = ((unsigned long long)__float_as_uint(q) << 32) | (unsigned)b;
            key = k2 < key ? k2 : key;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off);
            key = o < key ? o : key;
        }
        if (lane == 0) wkey[wave] = key;
        __syncthreads();
        unsigned long long k0 = wkey[0];
        for (int w = 1; w < kJB / 64; ++w) k0 = wkey[w] < k0 ? wkey[w] : k0;
        b0 = (int)(unsigned)k0;
        scan(b0, live, live ? centre_dist<D>(x, a.r.ball + (long long)b0 * (D + 4)) : 0.0f);
        float m = live ? (a.margin ? second : best) : 0.0f;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        if (lane == 0) wmax[wave] = m;
        __syncthreads();
        wreach = wmax[0];
        for (int w = 1; w < kJB / 64; ++w) wreach = fmaxf(wreach, wmax[w]);
    }
    for (int b = 0; b < nbr; ++b) {
        if (b == b0) continue;
        const float* c = a.r.ball + (long long)b * (D + 4);
        const float Rb = c[D];
        // ball to ball: no query of the block can reach the row block
        {
            const float q = jdist2<D>(cqv, c);
            const float lb = sqrtf(q) * (1.0f - 1e-5f) - Rq - Rb;
            if (lb > 0.0f && lb * lb > wreach * 1.001f + 1e-30f) continue;
        }
        bool need = live && !(OP == JOIN_ANY && hit);
        float dxc = 0.0f;
        if (need) {
            dxc = centre_dist<D>(x, c);
            need = ball_reaches(dxc, Rb, OP == JOIN_NEAREST ? (a.margin ? second : best) : a.r2);
        }
        if (!__syncthreads_or(need)) continue;
        scan(b, need, dxc);
    }
    if (OP == JOIN_NEAREST) {
        if (live) {
            a.labels[qid] = arg;
            if (a.margin) a.margin[qid] = (a.r.count > 1) ? sqrtf(second) - sqrtf(best) : __builtin_inff();
        }
    } else if (OP == JOIN_FIRST) {
        if (live && first != 0x7fffffff) __atomic_store_n(&a.state[qid], (int32_t)first, __ATOMIC_RELAXED);
    } else if (OP == JOIN_DECIDE) {
        int32_t result = MG_FOUNDER;
        if (first != 0x7fffffff) result = fst == MG_FOUNDER ? a.K_old + first : MG_UNDECIDED;
        if (owner && result != MG_UNDECIDED) __atomic_store_n(&a.state[qid], result, __ATOMIC_RELAXED);
        const unsigned long long und = __ballot(owner && result == MG_UNDECIDED);
        if (lane == 0 && und) atomicAdd(a.und_counter, __popcll(und));
    } else {
        if (live && hit) a.covered[qid] = 1;
    }
}

// Pool entries whose point is covered leave the pool; each workgroup (a
// compaction block) also writes how many of its entries stay.
__global__ __launch_bounds__(kCompactBlock) void pool_mark_kernel(const int32_t* __restrict__ pool, int len,
                                                                  const uint8_t* __restrict__ covered,
                                                                  uint8_t* removed, int32_t* block_cnt) {
    __shared__ int wsum[kCompactBlock / 64];
    const int e = blockIdx.x * kCompactBlock + threadIdx.x;
    bool stay = false;
    if (e < len && !removed[e]) {
        if (covered[pool[e]]) removed[e] = 1;
        else stay = true;
    }
    const unsigned long long bal = __ballot(stay);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        for (int w = 0; w < kCompactBlock / 64; ++w) c += wsum[w];
        block_cnt[blockIdx.x] = c;
    }
}

}  // namespace

bool join_shape_ok(int D) { return D <= 4 || D == 8 || D == 16 || D == 32; }

JoinLayout join_layout(int count, int DP, int D) {
    JoinLayout L;
    const size_t nb = (size_t)(count + kJB - 1) / kJB;
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) / a * a; };
    L.packed = 0;
    L.sorted_tmp = L.packed + up((size_t)count * DP * 4);
    L.perm = L.sorted_tmp + up((size_t)count * DP * 4);
    L.geom_tmp = L.perm + up((size_t)count * 4);
    L.sort_ws = L.geom_tmp + up(nb * geom_stride(D) * 4);
    L.rows = L.sort_ws + up(sort_workspace_bytes(count));
    L.ball = L.rows + up((size_t)count * DP * 4);
    L.rho = L.ball + up(nb * (D + 4) * 4);
    L.total = L.rho + up((size_t)count * 4);
    return L;
}

#define FMS_JDSWITCH(D_, CALL)                            \
    switch (D_) {                                         \
        case 1: { constexpr int DD = 1; CALL; } break;    \
        case 2: { constexpr int DD = 2; CALL; } break;    \
        case 3: { constexpr int DD = 3; CALL; } break;    \
        case 4: { constexpr int DD = 4; CALL; } break;    \
        case 8: { constexpr int DD = 8; CALL; } break;    \
        case 16: { constexpr int DD = 16; CALL; } break;  \
        case 32: { constexpr int DD = 32; CALL; } break;  \
        default: return hipErrorInvalidValue;             \
    }

hipError_t launch_join_index(const float* src, int count, int ld, int d, int DP, int D, float scale, void* ws,
                             JoinIndex* out, hipStream_t s) {
    if (count <= 0 || !join_shape_ok(D)) return hipErrorInvalidValue;
    const JoinLayout L = join_layout(count, DP, D);
    char* base = (char*)ws;
    float* packed = (float*)(base + L.packed);
    float* sorted_tmp = (float*)(base + L.sorted_tmp);
    int32_t* perm = (int32_t*)(base + L.perm);
    float* geom_tmp = (float*)(base + L.geom_tmp);
    float* rows = (float*)(base + L.rows);
    float* ball = (float*)(base + L.ball);
    const long long cells = (long long)count * DP;
    hipLaunchKernelGGL(join_pack_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, src, count, ld, d,
                       DP, scale, packed);
    hipError_t e = launch_spatial_sort(packed, count, DP, D, sorted_tmp, perm, geom_tmp, base + L.sort_ws, s);
    if (e != hipSuccess) return e;
    const int nb = (count + kJB - 1) / kJB;
    float* rho = (float*)(base + L.rho);
    FMS_JDSWITCH(D, hipLaunchKernelGGL((join_gather_kernel<DD>), dim3(nb), dim3(kJB), 0, s, src, count, ld, d, DP,
                                       perm, rows, ball, rho));
    out->rows = rows;
    out->rho = rho;
    out->idx = perm;
    out->ball = ball;
    out->count = count;
    return hipGetLastError();
}

hipError_t launch_join(int op, const JoinIndex& q, const JoinIndex& r, int DP, int D, float r2, int32_t* labels,
                       float* margin, const uint8_t* status, int32_t* state, const int32_t* rstate, const Ctl* ctl,
                       int und_slot, uint8_t* covered, hipStream_t s, int K_old, bool first_pass,
                       int32_t* und_counter, const int32_t* cand, const float* rows_orig) {
    if (q.count <= 0 || r.count <= 0) return hipSuccess;
    JoinArgs a;
    a.K_old = K_old;
    a.first_pass = first_pass;
    a.und_counter = und_counter;
    a.q = q;
    a.r = r;
    a.DP = DP;
    a.r2 = r2;
    a.labels = labels;
    a.margin = margin;
    a.cand = cand;
    a.rows_orig = rows_orig;
    a.status = status;
    a.state = state;
    a.rstate = rstate;
    a.ctl = ctl;
    a.und_slot = und_slot;
    a.covered = covered;
    const int nb = (q.count + kJB - 1) / kJB;
    if (op == JOIN_NEAREST) {
        FMS_JDSWITCH(D, hipLaunchKernelGGL((join_kernel<DD, JOIN_NEAREST>), dim3(nb), dim3(kJB), 0, s, a));
    } else if (op == JOIN_FIRST) {
        FMS_JDSWITCH(D, hipLaunchKernelGGL((join_kernel<DD, JOIN_FIRST>), dim3(nb), dim3(kJB), 0, s, a));
    } else if (op == JOIN_DECIDE) {
        FMS_JDSWITCH(D, hipLaunchKernelGGL((join_kernel<DD, JOIN_DECIDE>), dim3(nb), dim3(kJB), 0, s, a));
    } else {
        FMS_JDSWITCH(D, hipLaunchKernelGGL((join_kernel<DD, JOIN_ANY>), dim3(nb), dim3(kJB), 0, s, a));
    }
    return hipGetLastError();
}

hipError_t launch_pool_mark(const int32_t* pool, int len, const uint8_t* covered, uint8_t* removed,
                            int32_t* block_cnt, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(pool_mark_kernel, dim3((len + kCompactBlock - 1) / kCompactBlock), dim3(kCompactBlock), 0, s,
                       pool, len, covered, removed, block_cnt);
    return hipGetLastError();
}

#undef FMS_JDSWITCH

}  // namespace fms
