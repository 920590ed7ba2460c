// fms_internal.h -- declarations shared by the host control code and the
// kernel launchers of libfms.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fms.h"

namespace fms {

// Seed status values (device and host).
enum : uint8_t { ST_ACTIVE = 0, ST_CONVERGED = 1, ST_FAILED = 2 };

// Merge decision state of a batch seed.
enum : int32_t { MG_SKIP = -3, MG_UNDECIDED = -2, MG_FOUNDER = -1 };

constexpr int kMaxIterCap = 4096;   // hard cap on max_iter / n_iter
constexpr int kMaxMergePasses = 64;
// BF16 forms: the refined-pair count is spread over counters 128 bytes apart
// (a workgroup adds its count to counter workgroup % kRefinedSlots), so that
// the workgroups of a launch do not queue on one address at the end of the
// kernel.
constexpr int kRefinedSlots = 64;
constexpr int kRefinedStride = 16;   // long longs: 128 bytes

// Device-resident control block of one seed batch.  Written only by kernels
// (single designated threads or integer atomics) and read back by the host
// through a pinned mirror.
struct Ctl {
    int32_t count[3];          // active-list lengths, by iteration t % 3
    int32_t conv_base[3];      // seeds converged before iteration t, by t % 3
    int32_t need;              // early-stop threshold ceil(gamma*B); INT_MAX disables
    int32_t iters_run;         // iterations that processed >= 1 seed
    int32_t pool_len;          // seed pool length after compaction
    int32_t k_new;             // merge: modes after this round's founders
    int32_t merge_host;        // merge: 1 if the device passes left seeds undecided
    long long pairs;           // sum of active seeds x n over iterations
    long long refined[kRefinedSlots * kRefinedStride];   // BF16 path: pairs recomputed in
                                                         // FP32, at [slot * kRefinedStride]
    int32_t und[kMaxMergePasses];        // merge: undecided seeds after each pass
    int32_t conv_it[kMaxIterCap + 2];    // seeds that converged at iteration t
};

inline long long ctl_refined(const Ctl& c) {
    long long r = 0;
    for (int i = 0; i < kRefinedSlots; ++i) r += c.refined[i * kRefinedStride];
    return r;
}

// Geometry of the fused step for one dimension class.
struct StepShape {
    int D;      // coordinates computed per pair (>= d, padding is zero)
    int DP;     // row stride of the packed point / seed arrays (floats)
    int R;      // seeds per lane
    int TS;     // seeds per tile = 64 * R
    int MC;     // points per point chunk, at least
};

// Default shape for dimension d; step_shape_for() also picks R from the
// batch size (fewer seeds per lane for small batches).
StepShape step_shape(int d);
StepShape step_shape_for(int d, int B);


// Packed device state of one batch (all pointers device memory).
struct Batch {
    int n;                 // points
    int d;                 // true dimension
    int n_seeds;           // seeds in the batch (capacity of the seed arrays)
    StepShape sh;
    int kernel;            // ms_kernel
    float h;
    float scale;           // coordinate scale of the packed points
    float thr2;            // (tol*h)^2 in original units
    float inv_scale;       // 1/scale
    const float* Xp;       // n x DP packed points (scaled, zero padded)
    float* S;              // cap x DP seed positions (original units, padded)
    int32_t* act[2];       // active seed lists
    uint8_t* status;       // cap
    int32_t* iters;        // cap
    float* shift2;         // cap
    float* part;           // chunk partials, one (D+1)-vector per seed and chunk
    int grid;              // workgroups of the fused step
    int chunk_points = 1024;   // batched step: points per point chunk
    int grid_cap = 2048;       // batched step: most workgroups of the step launch
    int prec;              // ms_precision
    const float* Xs;       // BF16 and culled FP32 forms: points in spatial order (n x DP)
    const float* geom;     // BF16 and culled FP32 forms: per 256-point block centre and radius
    const void* pf;        // BF16 form: point features of the first product
    const void* xv;        // BF16 form: point operand of the second product
    float e_thr;           // BF16 form: refine threshold (packed units)
    float kappa;           // BF16 form: error bound coefficient
    const float* shift = nullptr;   // BF16 form, D > 4: frame of the sorted points
    int feat_blocks = 0;   // BF16 form over many clouds: 256-point blocks of the features (0: from n)
    const int32_t* boff = nullptr;   // BF16 form over many clouds: blocks before each cloud
    unsigned long long* prog = nullptr;   // host-mapped progress word (t << 32 | m), or NULL
    int metric = MS_METRIC_EUCLIDEAN;     // cosine: seeds are renormalized after each update
    Ctl* ctl;
};

long long step_part_floats(const StepShape& sh, int B, int grid);
long long step_red_offset(const StepShape& sh, int B, int grid);

// ---- launchers (k_step.hip) ----------------------------------------------
hipError_t launch_pack_points(const float* X, int n, int d, int DP, float scale,
                              float* Xp, hipStream_t s);
// Cosine metric: Xn = rows of X divided by their length; *bad (if not NULL)
// is set to 1 when a row has no finite nonzero length.
hipError_t launch_normalize_rows(const float* X, int n, int d, float* Xn, int32_t* bad, hipStream_t s);
// Fit round start: drawn seeds (pool[pos[j]]; j itself when pos is NULL)
// leave the pool, become the batch's seeds, and the control block is reset.
hipError_t launch_round_init(const float* X, int d, int DP, const int32_t* pool,
                             const int32_t* pos, int B, int32_t* ids, uint8_t* removed,
                             int32_t* merge_state, Batch& b, int need, int max_iter, hipStream_t s);
hipError_t launch_seed_init_from_array(const float* seeds, const uint8_t* conv_in,
                                       int d, int m, Batch& b, hipStream_t s);
hipError_t launch_ctl_reset(Ctl* ctl, int B, int need, int max_iter, hipStream_t s);
hipError_t launch_iteration(Batch& b, int t, hipStream_t s);
hipError_t launch_seed_export(const Batch& b, int m, float* seeds, uint8_t* conv,
                              int32_t* iters, float* shift2, hipStream_t s);
int step_grid(const StepShape& sh, int B, int n);

// ---- launchers (k_step_wide.hip): FP32 step for padded D = 128, 256 --------
hipError_t launch_iteration_wide(Batch& b, int t, hipStream_t s);

// ---- launchers (k_step_cull.hip): FP32 step over Morton-ordered points, d <= 4 --
bool cull_supported(int d, int n);
// Distance beyond which the culled step may skip pairs (original units).
double cull_reach(int kernel, double h);
StepShape step_shape_cull(int d, int B, int n);
hipError_t launch_iteration_cull(Batch& b, int t, hipStream_t s);

// ---- many clouds ---------------------------------------------------------------
// The cloud c with pre[c] <= v < pre[c + 1] (pre ascending over ncl + 1
// entries; empty clouds, whose range is empty, are never returned).
template <class T>
__device__ __forceinline__ int upper_cloud(const T* pre, int ncl, long long v) {
    int lo = 0, hi = ncl;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((long long)pre[mid] <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Device plan of one batched iteration (k_batched.hip fills it; the step
// kernels read it).
struct BatchedArgs {
    int ncl;
    const long long* x_off;   // ncl + 1 point offsets
    const int32_t* seg;       // ncl + 1 seed offsets
    int32_t* cnt;             // 2 x ncl active counts, by iteration t % 2
    int32_t* tiles;           // ncl
    int32_t* chunks;          // ncl
    int32_t* item_pre;        // ncl + 1
    int32_t* slot_pre;        // ncl + 1
    int32_t* item_cloud;      // cloud of each work item
    int32_t* slot_cloud;      // cloud of each active slot
    int32_t* queue;           // next work item to take (zeroed by the plan)
    int chunk_points;         // points per point chunk (BF16 form: a multiple of 256)
    int grid_cap;             // most workgroups of the step
    const int32_t* boff;      // BF16 form: 256-point blocks before cloud c (ncl + 1), else NULL
};

// ---- launchers (k_step_bf16.hip) -----------------------------------------
StepShape step_shape_bf16(int d, int B);
bool bf16_supported(int d);
hipError_t launch_iteration_bf16(Batch& b, int t, hipStream_t s);
size_t bf16_feature_bytes(int n);
hipError_t launch_bf16_features(const float* Xs, int n, int d, const float* geom, void* feat,
                                hipStream_t s);

// ---- launchers (k_step_bf16w.hip): BF16 form for D in {8, 16, 32} ------------
bool bf16w_dims(int D);
hipError_t launch_iteration_bf16w(Batch& b, int t, hipStream_t s);
size_t bf16w_feature_bytes(int n, int D);
hipError_t launch_bf16w_features(const float* Xs, int n, int D, const float* geom, void* feat,
                                 hipStream_t s);

// ---- launchers (k_step_bf16f.hip): BF16 form, Gaussian, D in {8, 16, 32} --------
hipError_t launch_iteration_bf16f(Batch& b, int t, hipStream_t s);
size_t bf16f_feature_bytes(int n, int D);
hipError_t launch_bf16f_features(const float* Xs, int n, int D, const float* geom, void* feat, hipStream_t s);
// Many clouds: the features of nblk blocks, block b of cloud c holding the
// sorted rows x_off[c] + 256 (b - boff[c]) .. (at most 256, within the cloud).
size_t bf16f_feature_bytes_blocks(long long nblk, int D);
hipError_t launch_bf16f_features_batched(const float* Xs, int D, const long long* x_off, const int32_t* boff,
                                         int ncl, int nblk, void* feat, hipStream_t s);
// The step of one batched iteration in this form (one partial per seed and
// work item, as the FP32 batched step stores them; seed tiles of 128).
hipError_t launch_bstep_bf16f(const Batch& b, const BatchedArgs& B, int t, int grid, hipStream_t s);
constexpr int kBf16fTile = 128;
// Feature bytes and builder of the BF16 form for D > 4 (the Gaussian kernel's
// compensated form or the flat window's screen form).
inline size_t bf16_wide_feature_bytes(int n, int D, int kernel) {
    return kernel == MS_KERNEL_GAUSSIAN ? bf16f_feature_bytes(n, D) : bf16w_feature_bytes(n, D);
}
inline hipError_t launch_bf16_wide_features(const float* Xs, int n, int D, const float* geom, void* feat,
                                            int kernel, hipStream_t s) {
    return kernel == MS_KERNEL_GAUSSIAN ? launch_bf16f_features(Xs, n, D, geom, feat, s)
                                        : launch_bf16w_features(Xs, n, D, geom, feat, s);
}

// ---- launchers (k_batched.hip): the step over many clouds ----------------------
int batched_max_clouds();
long long batched_max_items(const long long* x_off, const int32_t* seg, int ncl, int TS, int chunk_points);
hipError_t launch_batched_init(const float* seeds, const uint8_t* conv_in, int d, int M,
                               const int32_t* seg_dev, int ncl, int32_t* cnt, Batch& b, hipStream_t s);
// plan: 4 ncl + 3 ints of device scratch (per-cloud tiles, chunks, item and
// slot prefixes, the work-item queue head)
hipError_t launch_batched_iteration(const Batch& b, const long long* x_off_dev, const int32_t* seg_dev,
                                    int ncl, int32_t* cnt, int32_t* plan, int32_t* item_cloud,
                                    int32_t* slot_cloud, int t, hipStream_t s);

// ---- launchers (k_sort.hip) ----------------------------------------------
constexpr int kGeomStride = 8;      // per-256-point block (D <= 4): centre[4], radius
// Floats per block geometry row: centre[D], radius (and for D > 4 the centre's norm).
inline int geom_stride(int D) { return D <= 4 ? kGeomStride : D + 8; }
// Frame shift (bounding-box midpoint) the D > 4 sort subtracts from the sorted points.
const float* sort_frame_shift(const void* ws);
size_t sort_workspace_bytes(int count);
hipError_t launch_spatial_sort(const float* Xp, int n, int DP, int D, float* Xs, int* perm,
                               float* geom, void* ws, hipStream_t s);
hipError_t launch_seed_order(const float* S, int DP, int D, int m, float scale,
                             const uint8_t* status, void* ws, int32_t* act0, const float* Xp, int n,
                             hipStream_t s);
// Many clouds (D in {8, 16, 32}): every cloud's points ordered as the D > 4
// sort orders one cloud's, within the cloud's own rows and against its own
// pivots (batched_pivot_count of them, poff their prefix).  The workspace
// keeps the pivots' chain ranks for launch_batched_seed_order.
int batched_pivot_count(long long n_cloud);
size_t batched_sort_workspace_bytes(int count, int ptot);
struct CloudRows {
    int ncl;
    const long long* roff;   // device, ncl + 1 row offsets of the clouds
    const int32_t* tpre;     // device, ncl + 1: 256-row tiles before each cloud
    int tiles;               // tpre[ncl]
};
// ws: batched_sort_workspace_bytes(count, ptot) bytes, count >= the points
// and the seeds to be ordered (the same count for both calls).
hipError_t launch_batched_sort(const float* Xp, int n, int D, const CloudRows& pts, const int32_t* poff, int ptot,
                               float* Xs, void* ws, int count, hipStream_t s);
// Active lists of a batch of seeds (S in original units, `scale` to packed
// units) in the order of their positions within each cloud, the active seeds
// of a cloud first: act0[seg[c] ..] holds cloud c's seeds.  count: as for
// launch_batched_sort (>= M).
hipError_t launch_batched_seed_order(const float* S, int DP, int D, int M, float scale, const uint8_t* status,
                                     const CloudRows& seeds, const float* Xp, const CloudRows& pts,
                                     const int32_t* poff, void* ws, int count, int ptot, int32_t* act0,
                                     hipStream_t s);

// ---- launchers (k_merge.hip) ---------------------------------------------
hipError_t launch_iota(int32_t* a, int n, hipStream_t s);
// ---- whole method for many clouds (k_fit_batched.hip) ---------------------
hipError_t launch_bf_iota(const long long* x_off, int ncl, int32_t* pool, long long n, hipStream_t s);
hipError_t launch_bf_gather(const float* X, int d, const long long* x_off, const long long* s_off, int ncl,
                            const int32_t* pos, const int32_t* pool, uint8_t* removed, float* seeds, int M,
                            hipStream_t s);
// mstore: the mode store, cloud c's modes at rows x_off[c] + k (n x d)
hipError_t launch_bf_cover(const float* X, int d, const long long* x_off, int ncl, const int32_t* pool,
                           const int32_t* pool_len, const float* mstore, const int32_t* k_old,
                           const int32_t* k_new, float r2, uint8_t* removed, long long n, hipStream_t s);
// The round's merge: state (M ints) to undecided, then decision passes until
// *und (device) reads 0, then the founders appended to each cloud's modes.
hipError_t launch_bf_merge_init(int32_t* state, int M, hipStream_t s);
hipError_t launch_bf_decide_pass(const float* S, int d, const uint8_t* conv, const long long* s_off, int ncl,
                                 const float* mstore, const long long* x_off, const int32_t* k_cnt, float r2,
                                 int32_t* state, int32_t* und, int M, bool first, hipStream_t s);
hipError_t launch_bf_founders(const float* S, int d, const long long* s_off, int ncl, const int32_t* state,
                              const long long* x_off, float* mstore, int32_t* k_cnt, int32_t* k_old, hipStream_t s);
hipError_t launch_bf_modes_out(const float* mstore, int d, const long long* x_off, int ncl, const int32_t* k_off,
                               float* modes, hipStream_t s);
hipError_t launch_bf_fill_i32(int32_t* a, long long count, int32_t v, hipStream_t s);
hipError_t launch_bf_compact(const long long* x_off, int ncl, const int32_t* pool_in, uint8_t* removed,
                             int32_t* pool_len, int32_t* pool_out, hipStream_t s);
hipError_t launch_bf_assign(const float* X, int d, const long long* x_off, int ncl, const float* modes,
                            const int32_t* m_off, int32_t* labels, long long n, hipStream_t s);

hipError_t launch_fill_u8(uint8_t* a, int n, uint8_t v, hipStream_t s);
constexpr int kCompactBlock = 1024;   // pool entries per compaction block
// One merge decision pass over a batch of B seeds (the first pass also
// settles seeds that did not converge and seeds that join one of the first
// k_scan old modes: K_old, or 0 when the block join matched them already).
// A seed joining batch seed j is recorded as K_old + j.
hipError_t launch_merge_decide_pass(const float* S, int DP, int d, const uint8_t* status, int B,
                                    const float* modes, int K_old, int k_scan, float r2, int32_t* state,
                                    int32_t* und_counter, bool first, hipStream_t s);
// block_tmp: ceil(B / 1024) ints of device scratch (NULL: one workgroup).
hipError_t launch_merge_founders(const float* S, int DP, int B, int K_old, const int32_t* state,
                                 float* modes, Ctl* ctl, int und_slot, int32_t* block_tmp, hipStream_t s);
// Pool coverage by the modes [k0, k1) (k1 read from ctl->k_new on the device
// when ctl is not NULL); also writes the per-block counts that
// launch_pool_compact consumes.
hipError_t launch_cover(const float* X, int d, const int32_t* pool, int len,
                        const float* modes, int k0, int k1, const Ctl* ctl, float r2,
                        uint8_t* removed, int32_t* block_cnt, hipStream_t s);
// Stable compaction of the pool entries not flagged removed, from the block
// counts launch_cover wrote; clears the flags of [0, len) for the next round.
// Writes the new length to ctl->pool_len.
hipError_t launch_pool_compact(const int32_t* pool_in, uint8_t* removed, int len,
                               int32_t* pool_out, int32_t* block_tmp, Ctl* ctl,
                               hipStream_t s);
int pool_compact_blocks(int len);

// ---- block join of two large row sets (k_join.hip) ------------------------
// Used when both sides have at least kJoinMin rows and the padded D is one of
// 1..4, 8, 16, 32.
constexpr int kJoinMin = 4096;
enum : int { JOIN_NEAREST = 0, JOIN_FIRST = 1, JOIN_ANY = 2, JOIN_DECIDE = 3 };
// Rows in spatial order (unchanged values, stride DP, zero beyond d), their
// original indices, a ball (centre[D], radius; stride D + 4) per block of 256
// rows, and each row's distance to its block's centre.
struct JoinIndex {
    const float* rows;
    const int32_t* idx;
    const float* ball;
    const float* rho;
    int count;
};
struct JoinLayout {
    size_t packed, sorted_tmp, perm, geom_tmp, sort_ws, rows, ball, rho, total;
};
bool join_shape_ok(int D);
JoinLayout join_layout(int count, int DP, int D);
// Index of count rows of src (stride ld, d coordinates); `scale` only sets
// the units of the spatial sort.  ws: join_layout(count, DP, D).total bytes,
// which the index points into.
hipError_t launch_join_index(const float* src, int count, int ld, int d, int DP, int D, float scale, void* ws,
                             JoinIndex* out, hipStream_t s);
// nearest: labels[q] = the nearest row's index (ties to the lowest), margin
//   (optional) = sqrt(second) - sqrt(best); cand (optional, with rows_orig:
//   the unsorted rows) gives per query a row to start from, or -1;
// first: for converged queries whose state is MG_UNDECIDED, state[q] = the
//   lowest row index within r2, if any;
// any: covered[q] = 1 if a row whose rstate is MG_FOUNDER lies within r2
//   (nothing while ctl->und[und_slot] > 0);
// decide: one merge decision pass of a batch against itself (q and r index
//   the batch seeds): seeds it leaves undecided are counted in und_counter;
//   the first pass also settles the seeds that did not converge.
hipError_t launch_join(int op, const JoinIndex& q, const JoinIndex& r, int DP, int D, float r2, int32_t* labels,
                       float* margin, const uint8_t* status, int32_t* state, const int32_t* rstate, const Ctl* ctl,
                       int und_slot, uint8_t* covered, hipStream_t s, int K_old = 0, bool first_pass = false,
                       int32_t* und_counter = nullptr, const int32_t* cand = nullptr,
                       const float* rows_orig = nullptr);
// Pool entries whose point is covered leave the pool; writes the block counts
// launch_pool_compact consumes.
hipError_t launch_pool_mark(const int32_t* pool, int len, const uint8_t* covered, uint8_t* removed,
                            int32_t* block_cnt, hipStream_t s);

// ---- launchers (k_assign.hip) --------------------------------------------
hipError_t launch_assign(const float* X, int n, int d, const float* modes, int k,
                         int32_t* labels, float* margin, hipStream_t s);
hipError_t launch_check_finite(const float* X, long long count, int32_t* flag,
                               hipStream_t s);

// ---- launchers (k_adjoint.hip) -------------------------------------------
// ws: device workspace of adjoint_workspace_bytes() bytes.
hipError_t launch_forward_update(const void* X, int nb, int n, const void* S, int m, int d,
                                 double h, void* S_out, int bytes, void* ws, hipStream_t s);
hipError_t launch_step_adjoint(const void* X, int nb, int n, const void* S, int m, int d,
                               double h, const void* G, void* dS, void* dX, int bytes,
                               void* ws, hipStream_t s);
size_t adjoint_workspace_bytes(int nb, int n, int m, int d, int bytes);

}  // namespace fms
