/*
 * fms.h -- C ABI of libfms, an MI355X (gfx950) implementation of GPU Faster
 * Mean Shift with the Euclidean metric (You et al., arXiv 2112.13891).
 *
 * Problem statement (Algorithms 1 and 2): given a bandwidth h and a vector set
 * S = {x_1..x_n} in R^d, return the modes of the kernel density estimate of
 * eq. (7) and a cluster for every point, by iterating seeds s <- m(s), where
 * m(s) is the kernel-weighted mean of ALL n points (Section II-B, the batched
 * update that replaces the window search of eq. (13)-(15)).
 *
 * Conventions shared by every entry point
 *   - Arrays are row-major and contiguous.  Every array argument named as a
 *     "device" pointer is GPU memory owned by the caller (for instance a torch
 *     tensor); the library never frees caller memory and never keeps a pointer
 *     after the call returns (ms_fit) or after the enqueued work finishes
 *     (ms_step, ms_assign).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     ms_step and ms_assign are stream-ordered and asynchronous; ms_fit
 *     returns only once K is known on the host.
 *   - 1 <= n <= 2^31 - 1.  1 <= d <= 256 for ms_fit, ms_step,
 *     ms_step_noalloc and ms_assign (the BF16 form: d <= 32); 1 <= d <= 64
 *     for the batched calls and the differentiable form.
 *   - Return value: MS_OK (0) or a negative ms_status.  No exception crosses
 *     the ABI.  ms_last_error() gives a thread-local message for the last
 *     failure on the calling thread.
 *   - Calls on distinct streams may run concurrently from different threads.
 *   - Same inputs, parameters and rng_seed give bitwise-identical outputs on
 *     the same device and build (no floating-point atomics on result paths).
 */
#ifndef FMS_H
#define FMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MS_OK = 0,
    MS_E_INVALID = -1,   /* bad argument (message says which) */
    MS_E_NONFINITE = -2, /* X holds NaN or Inf (only when check_finite != 0) */
    MS_E_CAPACITY = -3,  /* more modes than max_modes; *k_out = required K */
    MS_E_NO_MODES = -4,  /* no seed converged */
    MS_E_NOMEM = -5,     /* device workspace allocation failed */
    MS_E_HIP = -6        /* a HIP runtime call failed */
} ms_status;

typedef enum {
    /* windowed kernel of eq. (12): weight 1 iff |s - x|^2 <= h^2 (inclusive) */
    MS_KERNEL_FLAT = 0,
    /* Gaussian profile: weight exp(-|s - x|^2 / (2 h^2)) */
    MS_KERNEL_GAUSSIAN = 1
} ms_kernel;

typedef enum {
    /* Euclidean distance (the paper's method) */
    MS_METRIC_EUCLIDEAN = 0,
    /* cosine metric (the authors' earlier Faster Mean Shift on cosine
       embeddings): every row x of X is replaced by its direction x/|x|, seeds
       are unit vectors, every distance is the chord between unit vectors,
       |s - u|^2 = 2 - 2 cos(s, u) (so the flat window keeps cos >= 1 - h^2/2
       and the Gaussian weight is exp((cos - 1)/h^2)), the update is the
       weighted mean direction sum w u / |sum w u|, and tol, the merge and
       cover radii and the labels use chords (labels: largest cosine).
       Modes are unit vectors. */
    MS_METRIC_COSINE = 1
} ms_metric;

typedef enum {
    MS_PREC_FP32 = 0,        /* FP32 direct differences, FP32 accumulation */
    MS_PREC_BF16_REFINE = 1  /* BF16 MFMA products, FP32 recompute within
                                refine_radius*h, FP32 accumulation */
} ms_precision;

/* Method parameters.  Field order is part of the ABI. */
typedef struct {
    uint64_t rng_seed;        /* SplitMix64 state for the seed draws */
    float h;                  /* bandwidth, > 0 (Algorithms 1-2 "Require h") */
    int32_t kernel;           /* ms_kernel */
    int32_t precision;        /* ms_precision */
    float tol;                /* converged iff |s_t - s_{t-1}| < tol*h; > 0 */
    int32_t max_iter;         /* at most this many updates per seed; >= 1 */
    float merge_radius;       /* modes within merge_radius*h merge (x h) */
    float cover_radius;       /* pool points within cover_radius*h of a mode
                                 leave the seed pool (x h); >= 0 */
    float gamma;              /* early stop once ceil(gamma*B) of a batch of B
                                 seeds converged (Section II-C); (0, 1] */
    int32_t n_initial;        /* initial seed count N (Section II-D: 128) */
    int32_t L;                /* stop once N >= L*M (Section II-D: 8) */
    float refine_radius;      /* BF16 path: every pair that may lie within
                                 refine_radius*h (rigorous bound on the bf16
                                 estimate) gets the exact FP32 distance,
                                 weight and accumulation; >= 1 is used for
                                 the flat window */
    int32_t all_points_as_seeds; /* 1: Algorithm 1 (every point is a seed,
                                    one batch); 0: Algorithm 2 (pool) */
    int32_t check_finite;     /* 1: scan X for NaN/Inf first */
    int32_t metric;           /* ms_metric (ms_fit, ms_step); ms_step_batched,
                                 ms_assign: Euclidean only */
    int32_t graph;            /* ms_step_batched: 1 = capture the n_iter
                                 iterations in one HIP graph and launch it
                                 once (the call then returns when it is done);
                                 the executable graph is kept per host thread
                                 and updated in place by later calls of the
                                 same topology (instantiated once per shape);
                                 0 = launch kernel by kernel.  Other calls
                                 ignore it */
    int32_t tile_R;           /* ms_step_batched: seeds per lane of a seed
                                 tile (1, 2 or 4, as the padded dimension
                                 allows: D <= 4 any, D = 8 or 16 1 or 2,
                                 D >= 32 1); 0 = the shape ms_tune_batched chose for
                                 inputs of this kind, else a default.  The
                                 results do not depend on it */
    int32_t plain;            /* ms_fit, ms_step with MS_PREC_FP32: 1 = the
                                 plain step, every pair computed in input
                                 order (no spatial order, no block culling;
                                 the skipped blocks contribute exact zeros,
                                 so only the summation order differs); for
                                 comparison.  Ignored by the BF16 form */
    int32_t tile_chunk;       /* ms_step_batched, ms_fit_batched: points per
                                 point chunk of a cloud, 64..65536; 0 = the
                                 size ms_tune_batched chose for inputs of this
                                 kind, else 1024.  It sets how each seed's sums
                                 are grouped (the rounding of the results,
                                 not their parity) */
    int32_t tile_grid;        /* ms_step_batched, ms_fit_batched: most
                                 workgroups of the step launch, 1..65536; 0 =
                                 the tuned value, else 2048.  The results do
                                 not depend on it */
    int32_t reserved[1];      /* must be 0 */
} ms_params;

/* Fills *p with the defaults: h = 1, Gaussian, FP32, tol = 1e-3,
 * max_iter = 100, merge_radius = cover_radius = 1, gamma = 1,
 * n_initial = 128, L = 8, refine_radius = 3, pool mode, rng_seed = 0,
 * Euclidean metric. */
void ms_default_params(ms_params *p);

#define MS_DIAG_MAX_ROUNDS 64

/* Optional diagnostics of ms_fit (host memory).  The pointer fields are
 * optional host arrays the caller provides (NULL to skip); "drawn" arrays
 * need room for n entries (all drawn seeds, concatenated by round). */
typedef struct {
    int32_t rounds;                          /* rounds run */
    int32_t round_N[MS_DIAG_MAX_ROUNDS];     /* requested seed count N */
    int32_t round_B[MS_DIAG_MAX_ROUNDS];     /* seeds drawn */
    int32_t round_M[MS_DIAG_MAX_ROUNDS];     /* modes after the round */
    int32_t round_T[MS_DIAG_MAX_ROUNDS];     /* iterations the batch ran */
    int32_t round_converged[MS_DIAG_MAX_ROUNDS];
    int64_t pairs;            /* sum over iterations of active seeds x n */
    int64_t refined_pairs;    /* BF16 path: pairs recomputed in FP32 */
    double iterate_ms;        /* GPU time of the seed iterations (events) */
    double merge_ms;          /* GPU+host time of merge and pool update */
    double assign_ms;         /* GPU time of the labelling */
    double total_ms;          /* host wall time inside ms_fit */
    int64_t workspace_bytes;  /* peak device workspace */
    int32_t *drawn;           /* [n] drawn point ids */
    int32_t *drawn_iters;     /* [n] updates each drawn seed received */
    int8_t *drawn_status;     /* [n] 1 converged, 0 discarded, 2 failed */
    float *drawn_final;       /* [n*d] final seed positions */
    int32_t *counts;          /* [max_modes] seeds merged into each mode */
} ms_diag;

/*
 * ms_fit -- the whole method: Algorithm 2 (seed selection, batched
 * iteration with early stopping, prune modes, cluster by distance to modes)
 * with the seed-count control of Section II-D; Algorithm 1 when
 * p->all_points_as_seeds is set.
 *
 *   X       device, n x d float32 points.
 *   modes   device, max_modes x d float32; receives the K modes in creation
 *           order (a mode is the final position of the first seed that
 *           founded it).
 *   k_out   host; receives K (also on MS_E_CAPACITY: the K required).
 *   labels  device, n int32 (may be NULL); nearest mode, ties to the lowest
 *           index.
 *   diag    host, optional (NULL to skip).
 * With p->metric = MS_METRIC_COSINE the method runs on the directions of the
 * rows of X (a row of length 0 makes the call fail with MS_E_INVALID) and the
 * modes are unit vectors.
 * Host-synchronous: returns when K is on the host and labels are written.
 * Errors: MS_E_INVALID, MS_E_NONFINITE, MS_E_CAPACITY, MS_E_NO_MODES,
 * MS_E_NOMEM, MS_E_HIP.  On error the contents of modes/labels are
 * unspecified.
 */
int ms_fit(const ms_params *p, const float *X, int64_t n, int32_t d,
           float *modes, int32_t max_modes, int32_t *k_out, int32_t *labels,
           ms_diag *diag, void *stream);

/*
 * ms_step -- up to n_iter updates s <- m(s) of caller-given seeds (the inner
 * "while not converge" loop of Algorithms 1-2), without early stopping of
 * the batch.  Seeds whose converged flag is nonzero on entry are left as
 * they are.  Stream-ordered and asynchronous.
 *
 *   seeds      device, m x d float32, in/out.
 *   converged  device, m uint8, in/out: 0 active, 1 converged
 *              (|shift| < tol*h), 2 failed (sum of weights 0 or non-finite).
 *   iters      device, m int32, out: updates applied during this call.
 *   shift2     device, m float32, out: squared length of the last update
 *              (unchanged for seeds that received none).
 * Uses p->h, kernel, precision, tol, refine_radius, metric; other fields
 * ignored.  Cosine metric: the seeds are made unit vectors on entry and stay
 * unit vectors; a row of X of length 0 has no direction and makes every seed
 * that sees it fail.
 */
int ms_step(const ms_params *p, const float *X, int64_t n, int32_t d,
            float *seeds, int32_t m, int32_t n_iter, uint8_t *converged,
            int32_t *iters, float *shift2, void *stream);

/*
 * ms_step_noalloc -- ms_step for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as ms_step, but every
 * workspace buffer (packed and spatially ordered points, control block,
 * active lists, chunk partials) is carved out of one fixed device scratch
 * array of 32 MiB that the library holds on each GPU it runs on until the
 * process ends; the call itself makes no hipMalloc, hipFree or other
 * allocating call.  The caller still passes X and the seed arrays.
 *   Size limit: the call is sized before anything is launched; one that
 *   needs more than 32 MiB of workspace (for instance n = 200,000 points of
 *   d = 3 need about 8 MB in FP32 and 24 MB in the BF16 form; n x d of a
 *   few million floats and more do not fit) fails with MS_E_INVALID and a
 *   message that gives the bytes it needs.
 *   Concurrency: every call on one GPU uses that GPU's one scratch array and
 *   leaves its contents behind; calls that overlap on one GPU (other
 *   streams, other threads) race and must be serialized by the caller.
 * Stream-ordered and asynchronous, as ms_step.
 */
int ms_step_noalloc(const ms_params *p, const float *X, int64_t n, int32_t d, float *seeds,
                    int32_t m, int32_t n_iter, uint8_t *converged, int32_t *iters,
                    float *shift2, void *stream);

/*
 * ms_step_batched -- ms_step for many independent point clouds at once: cloud
 * c owns the points X[x_off[c], x_off[c+1]) and the seeds
 * seeds[s_off[c], s_off[c+1]), and each seed is updated with its own cloud's
 * points only, as ms_step on that cloud would (Section II-B update, per-seed
 * convergence of Algorithms 1-2; FP32 form).  Each iteration is one launch
 * of each kernel for all clouds, over work items (cloud, seed tile, point
 * chunk) planned on the device from per-cloud active counts.
 *
 *   X          device, (x_off[ncl]) x d float32, the clouds' points back to back.
 *   x_off      host, ncl + 1 nondecreasing point offsets, x_off[0] = 0.
 *   seeds      device, (s_off[ncl]) x d float32, in/out.
 *   s_off      host, ncl + 1 nondecreasing seed offsets, s_off[0] = 0; a
 *              cloud with seeds must have points.
 *   ncl        1..8192 clouds.
 *   converged, iters, shift2: as ms_step, one entry per seed.
 * Uses p->h, kernel, tol, precision, graph, tile_R, tile_chunk, tile_grid.
 * MS_PREC_FP32: every pair in FP32 (the fused step of ms_step).
 * MS_PREC_BF16_REFINE: the BF16 form of ms_step for D > 4, per cloud, for
 * the Gaussian kernel at 5 <= d <= 32 (else MS_E_INVALID): each cloud's
 * points are put in spatial order within the cloud's own rows (nearest of
 * the cloud's own pivots, one per 256 points, at most 256), centred per
 * 256-point block, and every seed's sums take the seed-point products and
 * W.X on MFMA with three-part bf16 operands, the pairs whose weight the
 * expanded form cannot resolve computed in FP32 by direct differences; the
 * active seeds of a cloud are ordered by position; tiles of 128 seeds
 * (tile_R does not apply), chunks of whole 256-point blocks (tile_chunk is
 * rounded up to a multiple of 256).  Each call sorts the points again.
 * Stream-ordered; the call returns once the offsets are on the device (it
 * waits for the work already queued on the stream), the iterations
 * themselves run asynchronously -- with p->graph = 1 they are captured on a
 * private stream as one HIP graph (3 kernels per iteration, no memory
 * nodes), launched on `stream`, and the call returns when the graph is done.
 */
int ms_step_batched(const ms_params *p, const float *X, const int64_t *x_off,
                    float *seeds, const int64_t *s_off, int32_t ncl, int32_t d,
                    int32_t n_iter, uint8_t *converged, int32_t *iters,
                    float *shift2, void *stream);

/*
 * ms_assign -- "cluster x by the distance to modes" (Algorithm 2, last
 * loop): labels[i] = argmin_j |x_i - mode_j|^2 by FP32 direct differences,
 * ties to the lowest j.  margin (optional, may be NULL): distance to the
 * second-nearest mode minus distance to the nearest (+inf when k == 1).
 * All pointers are device memory.  Stream-ordered and asynchronous.
 */
int ms_assign(const float *X, int64_t n, int32_t d, const float *modes,
              int32_t k, int32_t *labels, float *margin, void *stream);

/*
 * ms_forward_update -- one Gaussian update of every seed with no stopping,
 * S_out = m(S_in) (Section II-B), for `nbatch` independent point sets at
 * once: X is nbatch x n x d, S_in and S_out are nbatch x m x d, and each
 * set's seeds see only that set's points.  The element type is float32
 * (dtype_bytes = 4) or float64 (8).  The differentiable form of the method
 * (Section II-B unrolled T times with S_0 = X) is built from this call and
 * ms_step_adjoint.  Device pointers; stream-ordered and asynchronous.
 */
int ms_forward_update(const void *X, int32_t nbatch, int64_t n, const void *S_in,
                      int64_t m, int32_t d, double h, void *S_out,
                      int32_t dtype_bytes, void *stream);

/*
 * ms_step_adjoint -- reverse-mode derivative of ms_forward_update.  With
 * w_ij = exp(-|s_j - x_i|^2/(2h^2)), W_j = sum_i w_ij, s'_j = sum_i w_ij x_i
 * / W_j and the upstream gradient G = dL/dS' (nbatch x m x d):
 *     beta_ij = w_ij * (g_j . (x_i - s'_j)) / (h^2 W_j)
 *     dL/ds_j = sum_i beta_ij (x_i - s_j)
 *     dL/dx_i = sum_j [ (w_ij / W_j) g_j + beta_ij (s_j - x_i) ]
 * are ADDED to dS (nbatch x m x d) and dX (nbatch x n x d).  The weights
 * are recomputed, never stored.  Same layout and dtype rules as
 * ms_forward_update.  dS may be the same array as dX when m == n: in the
 * first step of the unrolled form S_0 = X, so dL/dS_0 belongs to dX, and
 * passing dX as both adds the seed term and the point term there (the
 * passes that read X, S and G never read dS or dX, which are only added
 * into, one after the other).  G must not overlap dS or dX.  Device pointers;
 * stream-ordered and asynchronous.
 */
int ms_step_adjoint(const void *X, int32_t nbatch, int64_t n, const void *S,
                    int64_t m, int32_t d, double h, const void *G, void *dS,
                    void *dX, int32_t dtype_bytes, void *stream);

/*
 * ms_seed_draw -- the library's seed selection on host memory: draws
 * `count` ids from pool[0..len) by a partial Fisher-Yates shuffle driven by
 * SplitMix64 with the multiply-high bound (the same draw ms_fit makes each
 * round).  *state is the generator state (in/out); out receives the ids in
 * slot order.  pool is not modified.  Host only; no GPU needed.
 */
int ms_seed_draw(uint64_t *state, const int32_t *pool, int32_t len,
                 int32_t count, int32_t *out);

/*
 * ms_fit_batched -- the whole method (Algorithm 2 with the seed pool of
 * Section II-D; Algorithm 1 with all_points_as_seeds) for every cloud of a
 * batch, as ms_fit on each cloud alone would run it, the clouds' rounds
 * advancing together: every round's iterations of all clouds run through
 * the batched fused step (ms_step_batched's kernels), the seeds of cloud c
 * are drawn with the SplitMix64 state rng_seed + c, each cloud merges its
 * converged seeds into its own modes, coverage and compaction act on its own
 * pool, and its seed-count rule is its own.  Labels are the nearest mode
 * within the point's cloud.
 *   p          as ms_fit; metric Euclidean and gamma 1 (every round runs
 *              until each seed converged, failed or made max_iter
 *              updates).  p->precision MS_PREC_FP32, or MS_PREC_BF16_REFINE
 *              for the Gaussian kernel at 5 <= d <= 32 (else MS_E_INVALID):
 *              the iterations take ms_step_batched's BF16 form, the clouds'
 *              points sorted and their block features built once per call;
 *              merges, coverage and labels stay FP32.
 *   X          device, n x d row-major float32, the clouds' points
 *              concatenated; cloud c is rows x_off[c] .. x_off[c+1].
 *   x_off      host, ncl + 1 nondecreasing offsets, x_off[0] = 0, at
 *              least one point in total.
 *   ncl, d     1..8192 clouds, 1 <= d <= 64.
 *   modes      device, max_modes x d float32 out: cloud c's modes are rows
 *              k_off[c] .. k_off[c+1], in creation order.
 *   max_modes  rows of modes, >= 1.
 *   k_off      host, ncl + 1 out: mode offsets (filled on MS_E_CAPACITY too,
 *              so the caller can size modes).
 *   labels     device, n int32 out (may be NULL): index of the point's mode
 *              within its cloud, ties to the lowest index.
 *   rounds     host, may be NULL: rounds run (the most any cloud ran).
 * Errors: MS_E_INVALID (arguments), MS_E_CAPACITY (more modes than
 * max_modes), MS_E_NO_MODES (a cloud with points has no converged seed),
 * MS_E_NOMEM, MS_E_HIP.  Host-synchronous: the host draws the seeds and
 * applies the seed-count rule between rounds, and reads back whether a
 * round's seeds and its merge passes are done; the merges run on the
 * device.  Allocates device workspace on `stream`.
 */
int ms_fit_batched(const ms_params *p, const float *X, const int64_t *x_off, int32_t ncl, int32_t d,
                   float *modes, int64_t max_modes, int64_t *k_off, int32_t *labels, int32_t *rounds,
                   void *stream);

/*
 * ms_tune_batched -- launch-shape tuning for ms_step_batched and
 * ms_fit_batched.
 *
 * Times `trials` iterations (every seed active) of each launch shape on this
 * input -- the seeds per lane R that the padded dimension allows (see
 * ms_params.tile_R; the BF16 form: R = 2 only), times the points per chunk
 * 512, 1024, 2048, 4096 (see tile_chunk), times the step grids of 1024, 2048
 * and 4096 workgroups (see tile_grid) -- keeps the fastest, and records it
 * for the rest of the process under the input's kind: padded dimension,
 * floor(log2) of the mean points per cloud, floor(log2) of the mean seeds
 * per cloud and the precision.  Later calls
 * with tile_R, tile_chunk or tile_grid = 0 on inputs of that kind use it.
 * The iterations run on private copies of the seeds: nothing the caller
 * passed is written.  R and the grid never change the results; the chunk
 * size groups each seed's sums differently, so a tuned chunk size changes
 * their rounding (within the same parity with the oracle).
 *   p, X, x_off, seeds, s_off, ncl, d: as ms_step_batched (p->tile_R,
 *              tile_chunk, tile_grid and graph are ignored); at least one
 *              cloud must have seeds.
 *   trials     1..64 iterations per candidate.
 *   best_R     host, may be NULL: the chosen R.
 *   ms_per_iter host, may be NULL: 3 entries, the fastest milliseconds per
 *              iteration measured with R = 1, 2, 4 (over the chunk sizes and
 *              grids; -1 where R is not a candidate).
 *   best_chunk, best_grid  host, may be NULL: the chosen chunk size and grid.
 * Synchronous (returns once the candidates are timed).  Allocates device
 * workspace on `stream`.
 */
int ms_tune_batched(const ms_params *p, const float *X, const int64_t *x_off,
                    const float *seeds, const int64_t *s_off, int32_t ncl, int32_t d,
                    int32_t trials, int32_t *best_R, float *ms_per_iter, int32_t *best_chunk,
                    int32_t *best_grid, void *stream);

/*
 * ms_seed_count_next -- seed-count adaptation across the frames of a
 * sequence (video, tracking; Section II-D).  A frame starts with the seed
 * count N the previous frame ended with (ms_params.n_initial; ms_fit still
 * doubles it while N < L*M), and a count that grew above H times the mode
 * count is cut by one mode count per frame:
 *     *n_next = N - M  if N > H*M,  else N   (and at least 1),
 * with N = n_last, the seed count of the previous frame's last round
 * (ms_diag.round_N[rounds - 1]), and M = modes, its mode count.  The paper
 * uses H = 32.  MS_E_INVALID unless n_last >= 1, modes >= 0 and H >= 1.
 * Host only; no GPU needed.
 */
int ms_seed_count_next(int32_t n_last, int32_t modes, int32_t H, int32_t *n_next);

/*
 * ms_release_workspace -- frees the device workspace and pinned host staging
 * that ms_fit and ms_fit_batched keep for the calling thread between calls
 * (grown on demand for reuse by the next call on the same thread and
 * device), and whatever host threads that have exited left behind.  A thread
 * that exits hands its caches to the library, which frees them in the next
 * ms_fit or ms_fit_batched call on any thread, or here; so memory held for
 * exited threads never outlives the next call.  Those calls are
 * host-synchronous, so nothing is in flight on the released memory when they
 * have returned.  It also drops the calling thread's kept executable graph
 * of ms_step_batched (ms_params.graph = 1).  The next call allocates again.
 * Always returns MS_OK.
 */
int ms_release_workspace(void);

/*
 * ms_graph_stats -- how ms_step_batched's graph launches (ms_params.graph = 1)
 * on the calling thread came to be: graphs instantiated, and launches that
 * reused the kept executable graph, updated in place because the call
 * captured the same topology (same cloud count, iteration count and tile
 * shape).  Counts since the thread's first graph launch; either pointer
 * (host) may be NULL.  Always MS_OK.  Host only.
 */
int ms_graph_stats(int64_t *instantiations, int64_t *updates);

/* Thread-local message for the last failure on this thread ("" if none). */
const char *ms_last_error(void);

/* Library version string. */
const char *ms_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FMS_H */
