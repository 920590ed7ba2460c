/*
 * fms_oracle.c -- plain FP64 CPU oracle for GPU Faster Mean Shift with the
 * Euclidean metric (You et al., arXiv 2112.13891).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, header, table or constant generator with the HIP library under
 * paper_2112_13891_amd/csrc, and the product path never calls it.
 *
 * Everything is computed in FP64.  The FP32 inputs are widened exactly, sums run
 * in index order, and no blocking or reordering is added beyond what the
 * definitions state.  OpenMP only distributes independent seeds (or points)
 * over threads; each seed's arithmetic is the same at any thread count.
 *
 * Readings of places where the paper is silent or garbled (listed with their
 * reasons in the design notes of the repository):
 *   - flat kernel = the windowed kernel of eq. (12): weight 1 iff the squared
 *     distance is <= h^2 (inclusive); the "Epanechnikov" of eq. (8) is printed
 *     as the same indicator.
 *   - Gaussian kernel (not in the paper) = exp(-q / (2 h^2)), q the squared
 *     distance.
 *   - update (Section II-B, Algorithm 2): the kernel-weighted mean of ALL n
 *     points, m(s) = sum_i w_i x_i / sum_i w_i; for the flat kernel this is the
 *     sample mean of the window S_h, eq. (13)-(15), with m = |S_h|.
 *   - "not converge" (Algorithms 1 and 2): a seed is converged at the first
 *     update whose shift satisfies |s_t - s_{t-1}|^2 < (tol*h)^2; an empty
 *     window (sum of weights 0) makes the seed fail.
 *   - early stopping (Section II-C): once at least ceil(gamma*B) of a batch of
 *     B seeds have converged the batch stops and its unconverged seeds are
 *     discarded; seeds still unconverged after max_iter updates are discarded.
 *   - seed selection (Algorithm 2, Section II-D): uniform draws without
 *     replacement from a pool that starts as all points; SplitMix64 (Steele,
 *     Lea and Flood, 2014) drives a partial Fisher-Yates shuffle (Durstenfeld,
 *     1964) with the multiply-high bounded integer of Lemire (2019).
 *   - "prune modes": greedy in draw order; a converged seed joins the first
 *     mode (lowest index) within merge_r*h, else it founds a new mode at its own
 *     final position.
 *   - seed pool: drawn seeds, and every pool point within cover_r*h of a mode,
 *     leave the pool.
 *   - seed-count control (Section II-D): N starts at n_initial; after each
 *     round M = number of modes; stop when N >= L*M or the pool is empty,
 *     otherwise N doubles and a new batch is drawn.
 *   - labelling (Algorithm 2, last loop): nearest mode, ties to the lowest
 *     index.
 *   - cosine metric (the authors' earlier Faster Mean Shift on cosine
 *     embeddings; the method itself is unchanged): every point is replaced by
 *     its direction u = x / |x|, a seed is a unit vector s, and every distance
 *     of the Euclidean form becomes the chord between unit vectors,
 *     |s - u|^2 = 2 - 2 cos(s, u) = 2 - 2 s.u.  So the flat window keeps the
 *     points with cos >= 1 - h^2/2, the Gaussian weight is exp((cos - 1)/h^2),
 *     the update is the weighted mean direction s' = sum w u / |sum w u|, and
 *     the convergence, merge, coverage and labelling radii are chords
 *     (labels: largest cosine, ties to the lowest index).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FLAT 0
#define ORC_GAUSSIAN 1

#define ORC_EUCLIDEAN 0
#define ORC_COSINE 1

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_CAPACITY (-3)
#define ORC_E_NO_MODES (-4)
#define ORC_E_NOMEM (-5)

/* seed status values */
#define ORC_ACTIVE 0
#define ORC_CONVERGED 1
#define ORC_FAILED 2

/* ------------------------------------------------------------------------ */
/* Distance and kernel                                                       */
/* ------------------------------------------------------------------------ */

/* Squared Euclidean distance (eq. 4, squared) by direct differences. */
static double sq_dist(const float *x, const double *s, int d)
{
    double q = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)x[k] - s[k];
        q += t * t;
    }
    return q;
}

static double sq_dist_dd(const double *a, const double *b, int d)
{
    double q = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        q += t * t;
    }
    return q;
}

static double dot_dd(const double *a, const double *b, int d)
{
    double c = 0.0;
    for (int k = 0; k < d; ++k)
        c += a[k] * b[k];
    return c;
}

/* The squared distance the method works with, between a point row x and a
 * position s (both FP64): Euclidean, or for the cosine metric the squared
 * chord 2 - 2 s.x between unit vectors. */
static double pair_q(const double *x, const double *s, int d, int metric)
{
    if (metric == ORC_COSINE)
        return 2.0 - 2.0 * dot_dd(x, s, d);
    return sq_dist_dd(x, s, d);
}

/* Kernel weight for squared distance q: flat window of eq. (12), inclusive
 * at q == h^2, or the Gaussian profile exp(-q/(2h^2)). */
double orc_weight(double q, double h, int kernel)
{
    if (kernel == ORC_FLAT)
        return (q <= h * h) ? 1.0 : 0.0;
    return exp(-q / (2.0 * h * h));
}

/* One update of one seed over all n points (Section II-B): writes
 * m(s) = sum_i w_i x_i / sum_i w_i into out and returns sum_i w_i.  When the
 * sum of weights is 0, out is left unchanged. */
double orc_mean(const float *X, int64_t n, int d, const double *s, double h,
                int kernel, double *out)
{
    double acc[256];
    double wsum = 0.0;
    for (int k = 0; k < d; ++k)
        acc[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const float *x = X + i * (int64_t)d;
        double w = orc_weight(sq_dist(x, s, d), h, kernel);
        wsum += w;
        for (int k = 0; k < d; ++k)
            acc[k] += w * (double)x[k];
    }
    if (wsum > 0.0)
        for (int k = 0; k < d; ++k)
            out[k] = acc[k] / wsum;
    return wsum;
}

/* The same update on FP64 point rows P (n x d) for either metric: the
 * weighted mean, or for the cosine metric the weighted mean direction
 * sum w u / |sum w u|.  Returns sum_i w_i, or 0 when the update is undefined
 * (no weight, or a zero mean vector of directions); out is then unchanged. */
static double mean_rows(const double *P, int64_t n, int d, const double *s, double h,
                        int kernel, int metric, double *out)
{
    double acc[256];
    double wsum = 0.0;
    for (int k = 0; k < d; ++k)
        acc[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *x = P + i * (int64_t)d;
        double w = orc_weight(pair_q(x, s, d, metric), h, kernel);
        wsum += w;
        for (int k = 0; k < d; ++k)
            acc[k] += w * x[k];
    }
    if (!(wsum > 0.0))
        return 0.0;
    if (metric == ORC_COSINE) {
        double norm = sqrt(dot_dd(acc, acc, d));
        if (!(norm > 0.0))
            return 0.0;
        for (int k = 0; k < d; ++k)
            out[k] = acc[k] / norm;
    } else {
        for (int k = 0; k < d; ++k)
            out[k] = acc[k] / wsum;
    }
    return wsum;
}

/* FP64 point rows for a metric: the exact widening of X, or the unit
 * directions x / |x| for the cosine metric (NULL if a row has no direction
 * or allocation fails). */
static double *point_rows(const float *X, int64_t n, int d, int metric)
{
    double *P = (double *)malloc(sizeof(double) * (size_t)n * (size_t)d);
    if (!P)
        return NULL;
    for (int64_t i = 0; i < n; ++i) {
        double *p = P + i * (int64_t)d;
        for (int k = 0; k < d; ++k)
            p[k] = (double)X[i * (int64_t)d + k];
        if (metric == ORC_COSINE) {
            double norm = sqrt(dot_dd(p, p, d));
            if (!(norm > 0.0) || !isfinite(norm)) {
                free(P);
                return NULL;
            }
            for (int k = 0; k < d; ++k)
                p[k] /= norm;
        }
    }
    return P;
}

/* ------------------------------------------------------------------------ */
/* Fixed-budget iteration of caller-given seeds                              */
/* ------------------------------------------------------------------------ */

/* Advance one seed by one update.  Returns the new status. */
static int advance(const double *P, int64_t n, int d, double h, int kernel, int metric,
                   double tol, double *s, double *shift2_out)
{
    double next[256];
    double wsum = mean_rows(P, n, d, s, h, kernel, metric, next);
    if (!(wsum > 0.0))
        return ORC_FAILED;
    double delta2 = sq_dist_dd(next, s, d);
    memcpy(s, next, sizeof(double) * (size_t)d);
    *shift2_out = delta2;
    double thr = tol * h;
    return (delta2 < thr * thr) ? ORC_CONVERGED : ORC_ACTIVE;
}

/* Up to n_iter updates of every seed whose status is ORC_ACTIVE (Algorithm 1,
 * inner while loop).  seeds: m x d in/out; status in/out; iters out = updates
 * applied during this call; shift2 out = last squared shift (untouched seeds
 * keep their value). */
int orc_step_metric(const float *X, int64_t n, int d, double h, int kernel, double tol,
                    double *seeds, int32_t m, int32_t n_iter, uint8_t *status,
                    int32_t *iters, double *shift2, int nthreads, int metric)
{
    if (d < 1 || d > 256 || n < 1 || m < 0 || n_iter < 0 || !(h > 0.0) ||
        (metric != ORC_EUCLIDEAN && metric != ORC_COSINE))
        return ORC_E_INVALID;
    double *P = point_rows(X, n, d, metric);
    if (!P)
        return ORC_E_INVALID;
    if (metric == ORC_COSINE) {
        /* caller seeds become unit vectors */
        for (int32_t j = 0; j < m; ++j) {
            double *s = seeds + (int64_t)j * d;
            double norm = sqrt(dot_dd(s, s, d));
            if (!(norm > 0.0)) {
                free(P);
                return ORC_E_INVALID;
            }
            for (int k = 0; k < d; ++k)
                s[k] /= norm;
        }
    }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int32_t j = 0; j < m; ++j) {
        iters[j] = 0;
        for (int32_t t = 0; t < n_iter && status[j] == ORC_ACTIVE; ++t) {
            status[j] = (uint8_t)advance(P, n, d, h, kernel, metric, tol,
                                         seeds + (int64_t)j * d, shift2 + j);
            if (status[j] != ORC_FAILED)
                iters[j] += 1;
        }
    }
    free(P);
    return ORC_OK;
}

int orc_step(const float *X, int64_t n, int d, double h, int kernel, double tol,
             double *seeds, int32_t m, int32_t n_iter, uint8_t *status,
             int32_t *iters, double *shift2, int nthreads)
{
    return orc_step_metric(X, n, d, h, kernel, tol, seeds, m, n_iter, status, iters,
                           shift2, nthreads, ORC_EUCLIDEAN);
}

/* ------------------------------------------------------------------------ */
/* Seed selection: SplitMix64 + partial Fisher-Yates                         */
/* ------------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea, Flood 2014): add the golden-ratio increment, then
 * the two xor-shift-multiply mixing rounds. */
uint64_t orc_splitmix64(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ULL;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Lemire's multiply-high map of a 64-bit word onto [0, range). */
static uint64_t bounded(uint64_t r, uint64_t range)
{
    return (uint64_t)(((unsigned __int128)r * (unsigned __int128)range) >> 64);
}

/* Partial Fisher-Yates on a[0..len): after the call a[0..count) is the draw,
 * in slot order.  Slot t swaps with t + bounded(next, len - t). */
void orc_draw(uint64_t *state, int32_t *a, int32_t len, int32_t count)
{
    for (int32_t t = 0; t < count; ++t) {
        uint64_t r = orc_splitmix64(state);
        int32_t j = t + (int32_t)bounded(r, (uint64_t)(len - t));
        int32_t tmp = a[t];
        a[t] = a[j];
        a[j] = tmp;
    }
}

/* ------------------------------------------------------------------------ */
/* Labelling (Algorithm 2, final loop)                                        */
/* ------------------------------------------------------------------------ */

static int assign_rows(const double *P, int64_t n, int d, const double *modes, int32_t K,
                       int metric, int32_t *labels, double *margin, int nthreads)
{
    if (K < 1 || d < 1)
        return ORC_E_INVALID;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
        const double *x = P + i * (int64_t)d;
        double best = INFINITY, second = INFINITY;
        int32_t arg = 0;
        for (int32_t j = 0; j < K; ++j) {
            double q = pair_q(x, modes + (int64_t)j * d, d, metric);
            if (q < best) {
                second = best;
                best = q;
                arg = j;
            } else if (q < second) {
                second = q;
            }
        }
        labels[i] = arg;
        if (margin)
            margin[i] = (K > 1) ? sqrt(fmax(second, 0.0)) - sqrt(fmax(best, 0.0)) : INFINITY;
    }
    return ORC_OK;
}

int orc_assign_metric(const float *X, int64_t n, int d, const double *modes, int32_t K,
                      int32_t *labels, double *margin, int nthreads, int metric)
{
    double *P = point_rows(X, n, d, metric);
    if (!P)
        return ORC_E_INVALID;
    int rc = assign_rows(P, n, d, modes, K, metric, labels, margin, nthreads);
    free(P);
    return rc;
}

int orc_assign(const float *X, int64_t n, int d, const double *modes, int32_t K,
               int32_t *labels, double *margin, int nthreads)
{
    return orc_assign_metric(X, n, d, modes, K, labels, margin, nthreads, ORC_EUCLIDEAN);
}

/* ------------------------------------------------------------------------ */
/* The whole method (Algorithm 2 with Section II-C/D; Algorithm 1 when        */
/* all_points != 0)                                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t max_rounds;
    int32_t *n_rounds;     /* rounds run */
    int32_t *round_N;      /* requested seeds */
    int32_t *round_B;      /* drawn seeds */
    int32_t *round_M;      /* modes after the round */
    int32_t *round_T;      /* iterations the batch ran */
    int32_t *drawn;        /* all drawn ids, concatenated by round (cap n) */
    int32_t *drawn_iters;  /* updates each drawn seed received */
    int8_t *drawn_status;  /* 1 converged, 0 discarded, 2 failed */
    double *drawn_final;   /* final position of each drawn seed (cap n x d) */
    int64_t *pairs;        /* sum over iterations of active seeds x n */
} orc_trace;

/* Iterate one batch of B seeds (Algorithm 2 lines "for each seed / while not
 * converge" with the early-stopping rule of Section II-C).  pos: B x d in/out,
 * status out, iters out.  Returns the number of iterations run. */
static int32_t run_batch(const double *P, int64_t n, int d, double h, int kernel, int metric,
                         double tol, int32_t max_iter, double gamma, int32_t B,
                         double *pos, int8_t *status, int32_t *iters,
                         int64_t *pairs, int nthreads)
{
    int32_t need = (int32_t)ceil(gamma * (double)B);
    int32_t converged = 0;
    int32_t t = 0;
    for (int32_t j = 0; j < B; ++j) {
        status[j] = ORC_ACTIVE;
        iters[j] = 0;
    }
    while (t < max_iter) {
        int32_t active = 0;
        for (int32_t j = 0; j < B; ++j)
            active += (status[j] == ORC_ACTIVE);
        if (active == 0)
            break;
        t += 1;
        *pairs += (int64_t)active * n;
        int32_t newly = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : newly) num_threads(nthreads)
        for (int32_t j = 0; j < B; ++j) {
            if (status[j] != ORC_ACTIVE)
                continue;
            double s2 = 0.0;
            int st = advance(P, n, d, h, kernel, metric, tol, pos + (int64_t)j * d, &s2);
            if (st != ORC_FAILED)
                iters[j] += 1;
            status[j] = (int8_t)st;
            newly += (st == ORC_CONVERGED);
        }
        converged += newly;
        if (converged >= need)
            break;
    }
    /* seeds still active are discarded: not converged in time */
    return t;
}

/* Greedy merge of one batch into the mode list, in draw order ("prune
 * modes").  Returns the new mode count, or -1 when max_modes is exceeded
 * (the count keeps growing in *k_needed). */
static int32_t merge_batch(int d, int metric, double radius, int32_t B, const double *pos,
                           const int8_t *status, int32_t K, int32_t max_modes,
                           double *modes, int32_t *counts, int32_t *k_needed)
{
    double r2 = radius * radius;
    for (int32_t i = 0; i < B; ++i) {
        if (status[i] != ORC_CONVERGED)
            continue;
        const double *p = pos + (int64_t)i * d;
        int32_t join = -1;
        int32_t kk = (K < max_modes) ? K : max_modes;
        for (int32_t j = 0; j < kk; ++j) {
            if (pair_q(p, modes + (int64_t)j * d, d, metric) <= r2) {
                join = j;
                break;
            }
        }
        if (join >= 0) {
            counts[join] += 1;
        } else {
            if (K < max_modes) {
                memcpy(modes + (int64_t)K * d, p, sizeof(double) * (size_t)d);
                counts[K] = 1;
            }
            K += 1;
        }
    }
    *k_needed = K;
    return K;
}

int orc_fit_metric(const float *X, int64_t n, int d, double h, int kernel, double tol,
                   int32_t max_iter, double merge_r, double cover_r, double gamma,
                   int32_t n_initial, int32_t L, int32_t all_points, uint64_t rng_seed,
                   int nthreads, int32_t max_modes, double *modes, int32_t *counts,
                   int32_t *k_out, int32_t *labels, double *margin, int32_t max_rounds,
                   int32_t *n_rounds, int32_t *round_N, int32_t *round_B,
                   int32_t *round_M, int32_t *round_T, int32_t *drawn,
                   int32_t *drawn_iters, int8_t *drawn_status, double *drawn_final,
                   int64_t *pairs, int metric)
{
    if (d < 1 || d > 256 || n < 1 || n > 0x7fffffffLL || !(h > 0.0) ||
        max_iter < 1 || !(gamma > 0.0 && gamma <= 1.0) || n_initial < 1 ||
        L < 1 || max_modes < 1 || (metric != ORC_EUCLIDEAN && metric != ORC_COSINE))
        return ORC_E_INVALID;
    double *P = point_rows(X, n, d, metric);
    if (!P)
        return (metric == ORC_COSINE) ? ORC_E_INVALID : ORC_E_NOMEM;

    int32_t *pool = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *batch = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *gone = (uint8_t *)malloc((size_t)n);
    double *pos = (double *)malloc(sizeof(double) * (size_t)n * (size_t)d);
    int8_t *status = (int8_t *)malloc((size_t)n);
    int32_t *iters = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!pool || !batch || !gone || !pos || !status || !iters) {
        free(pool); free(batch); free(gone); free(pos); free(status); free(iters); free(P);
        return ORC_E_NOMEM;
    }

    int32_t pool_len = (int32_t)n;
    for (int32_t i = 0; i < pool_len; ++i)
        pool[i] = i;
    uint64_t rng = rng_seed;
    int32_t N = n_initial;
    int32_t K = 0, k_needed = 0;
    int32_t rounds = 0;
    int64_t drawn_total = 0;
    *pairs = 0;

    for (;;) {
        int32_t B;
        if (all_points) {
            /* Algorithm 1: every point is a seed, one batch in index order */
            B = (int32_t)n;
            for (int32_t i = 0; i < B; ++i)
                batch[i] = i;
        } else {
            B = (N < pool_len) ? N : pool_len;
            orc_draw(&rng, pool, pool_len, B);
            memcpy(batch, pool, sizeof(int32_t) * (size_t)B);
        }
        for (int32_t j = 0; j < B; ++j)
            for (int k = 0; k < d; ++k)
                pos[(int64_t)j * d + k] = P[(int64_t)batch[j] * d + k];

        int32_t T = run_batch(P, n, d, h, kernel, metric, tol, max_iter, gamma, B, pos,
                              status, iters, pairs, nthreads);
        int32_t K_before = K;
        K = merge_batch(d, metric, merge_r * h, B, pos, status, K, max_modes, modes,
                        counts, &k_needed);

        if (rounds < max_rounds) {
            round_N[rounds] = all_points ? B : N;
            round_B[rounds] = B;
            round_M[rounds] = K;
            round_T[rounds] = T;
        }
        for (int32_t j = 0; j < B; ++j) {
            int64_t o = drawn_total + j;
            drawn[o] = batch[j];
            drawn_iters[o] = iters[j];
            drawn_status[o] = status[j];
            memcpy(drawn_final + o * d, pos + (int64_t)j * d,
                   sizeof(double) * (size_t)d);
        }
        drawn_total += B;
        rounds += 1;
        if (all_points)
            break;

        /* seed pool update (seed selection, Section II-D): the drawn seeds
         * leave the pool, and so does every remaining pool point within
         * cover_r*h of a mode.  Modes of earlier rounds already removed the
         * points they cover, so only this round's new modes are checked. */
        {
            double rc2 = (cover_r * h) * (cover_r * h);
            int32_t kk = (K < max_modes) ? K : max_modes;
            int32_t k0 = (K_before < max_modes) ? K_before : max_modes;
            /* after the draw, pool[B..pool_len) holds the undrawn points */
            memset(gone, 1, (size_t)n);
#pragma omp parallel for schedule(static) num_threads(nthreads)
            for (int32_t p = B; p < pool_len; ++p) {
                int32_t i = pool[p];
                int covered = 0;
                for (int32_t j = k0; j < kk && !covered; ++j)
                    covered = pair_q(P + (int64_t)i * d, modes + (int64_t)j * d, d, metric) <= rc2;
                gone[i] = (uint8_t)covered;
            }
            /* the pool is kept in ascending index order */
            int32_t w = 0;
            for (int32_t i = 0; i < (int32_t)n; ++i)
                if (!gone[i])
                    pool[w++] = i;
            pool_len = w;
        }
        if (pool_len == 0 || (int64_t)N >= (int64_t)L * K)
            break;
        N *= 2;
    }

    *n_rounds = rounds;
    *k_out = k_needed;
    int rc = ORC_OK;
    if (K > max_modes)
        rc = ORC_E_CAPACITY;
    else if (K == 0)
        rc = ORC_E_NO_MODES;
    else if (labels)
        assign_rows(P, n, d, modes, K, metric, labels, margin, nthreads);

    free(pool); free(batch); free(gone); free(pos); free(status); free(iters); free(P);
    return rc;
}

int orc_fit(const float *X, int64_t n, int d, double h, int kernel, double tol,
            int32_t max_iter, double merge_r, double cover_r, double gamma,
            int32_t n_initial, int32_t L, int32_t all_points, uint64_t rng_seed,
            int nthreads, int32_t max_modes, double *modes, int32_t *counts,
            int32_t *k_out, int32_t *labels, double *margin, int32_t max_rounds,
            int32_t *n_rounds, int32_t *round_N, int32_t *round_B,
            int32_t *round_M, int32_t *round_T, int32_t *drawn,
            int32_t *drawn_iters, int8_t *drawn_status, double *drawn_final,
            int64_t *pairs)
{
    return orc_fit_metric(X, n, d, h, kernel, tol, max_iter, merge_r, cover_r, gamma,
                          n_initial, L, all_points, rng_seed, nthreads, max_modes, modes,
                          counts, k_out, labels, margin, max_rounds, n_rounds, round_N,
                          round_B, round_M, round_T, drawn, drawn_iters, drawn_status,
                          drawn_final, pairs, ORC_EUCLIDEAN);
}

/* Squared-distance helper exported for tests of the oracle itself. */
double orc_sq_dist(const float *x, const double *s, int d) { return sq_dist(x, s, d); }

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
