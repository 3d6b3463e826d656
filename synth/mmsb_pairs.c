/*
 * Seeded sampler for the undirected edge set of a mixed-membership stochastic
 * block model with block matrix P = q*1*1^T + (p-q)*I: every unordered pair
 * {i, j}, i < j, is an edge independently with probability
 * q + (p - q) * <pi_i, pi_j>, which equals pi_i^T P pi_j (the Bernoulli model
 * of Section 2.2).
 *
 * Input generation only: nothing here is part of the method.
 *
 * Exact thinning: candidates are drawn at rate p by geometric skipping along
 * each row's upper triangle, then accepted with probability
 * (q + (p - q) * <pi_i, pi_j>) / p.  The memberships arrive as a sparse list
 * per node (entries below a caller-chosen floor dropped), so a dot product
 * costs a merge of two short sorted lists.
 *
 * Randomness: one counter-based splitmix64 stream per row, keyed by
 * (seed, row), so the edge set does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s; } row_rng;

static inline row_rng rng_for_row(uint64_t seed, int64_t row) {
    row_rng r;
    r.s = mix64(seed * 0x9E3779B97F4A7C15ULL + 0xD1B54A32D192ED03ULL * (uint64_t)(row + 1));
    return r;
}

/* uniform in (0, 1] */
static inline double next_u01(row_rng* r) {
    r->s += 0x9E3779B97F4A7C15ULL;
    uint64_t x = mix64(r->s);
    return ((double)((x >> 11) + 1)) * (1.0 / 9007199254740992.0);
}

static inline double sparse_dot(const int32_t* ia, const double* va, int na,
                                const int32_t* ib, const double* vb, int nb) {
    double s = 0.0;
    int a = 0, b = 0;
    while (a < na && b < nb) {
        if (ia[a] == ib[b]) { s += va[a] * vb[b]; ++a; ++b; }
        else if (ia[a] < ib[b]) ++a;
        else ++b;
    }
    return s;
}

/* Walk row i's candidates; when out_cols is NULL only count. */
static int64_t walk_row(int64_t i, int64_t n, double p, double q, uint64_t seed,
                        const int64_t* pptr, const int32_t* pidx, const double* pval,
                        int32_t* out_cols) {
    row_rng r = rng_for_row(seed, i);
    const double log1mp = log1p(-p);
    int64_t j = i;
    int64_t cnt = 0;
    const int32_t* ia = pidx + pptr[i];
    const double* va = pval + pptr[i];
    const int na = (int)(pptr[i + 1] - pptr[i]);
    for (;;) {
        double u = next_u01(&r);
        double skip = (p >= 1.0) ? 0.0 : floor(log(u) / log1mp);
        if (skip > (double)n) break;
        j += 1 + (int64_t)skip;
        if (j >= n) break;
        double s = sparse_dot(ia, va, na, pidx + pptr[j], pval + pptr[j],
                              (int)(pptr[j + 1] - pptr[j]));
        double acc = (q + (p - q) * s) / p;
        double v = next_u01(&r);
        if (v <= acc) {
            if (out_cols) out_cols[cnt] = (int32_t)j;
            ++cnt;
        }
    }
    return cnt;
}

/* Pass 1: per-row edge counts (upper triangle). */
void mmsb_count(int64_t n, double p, double q, uint64_t seed,
                const int64_t* pptr, const int32_t* pidx, const double* pval,
                int64_t* counts) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
        counts[i] = walk_row(i, n, p, q, seed, pptr, pidx, pval, NULL);
}

/* Pass 2: fill the upper-triangle column lists at offsets[i]. */
void mmsb_fill(int64_t n, double p, double q, uint64_t seed,
               const int64_t* pptr, const int32_t* pidx, const double* pval,
               const int64_t* offsets, int32_t* cols) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i)
        walk_row(i, n, p, q, seed, pptr, pidx, pval, cols + offsets[i]);
}

/*
 * Generalised sampler: row node i of a row set against the nodes j of a
 * column set (both with sparse membership lists).  triangular != 0: one node
 * set, pairs j > i only (an undirected graph); otherwise every j (a bipartite
 * graph between two node sets).
 *
 * poisson == 0: Bernoulli(q + (p - q) <pi_i, pi_j>) edges as above.
 * poisson != 0: the Poisson model of Section 2.2, counts
 * G_ij ~ Poisson(lambda_ij), lambda_ij = q + (p - q) <pi_i, pi_j> <= p: every
 * pair holds Poisson(p) candidates, each kept with probability lambda_ij / p
 * (thinning), so the kept count is Poisson(lambda_ij).  Pairs with at least
 * one candidate (probability 1 - e^-p) are reached by geometric skipping;
 * their candidate count is drawn from the Poisson(p) law conditioned on >= 1
 * by inversion.  A pair with a kept count >= 1 is an edge of that weight.
 *
 * Randomness: one splitmix64 stream per row keyed by (seed, row).
 */
static int64_t walk_row_gen(int64_t i, int64_t n_cols, int triangular, int poisson, double p, double q, uint64_t seed,
                            const int64_t* rptr, const int32_t* ridx, const double* rval,
                            const int64_t* cptr, const int32_t* cidx, const double* cval,
                            int32_t* out_cols, float* out_w) {
    row_rng r = rng_for_row(seed, i);
    const double hit = poisson ? -expm1(-p) : p;          /* P(pair has >= 1 candidate) */
    const double log1mh = log1p(-hit);
    int64_t j = triangular ? i : -1;
    int64_t cnt = 0;
    const int32_t* ia = ridx + rptr[i];
    const double* va = rval + rptr[i];
    const int na = (int)(rptr[i + 1] - rptr[i]);
    for (;;) {
        double u = next_u01(&r);
        double skip = (hit >= 1.0) ? 0.0 : floor(log(u) / log1mh);
        if (skip > (double)n_cols) break;
        j += 1 + (int64_t)skip;
        if (j >= n_cols) break;
        double s = sparse_dot(ia, va, na, cidx + cptr[j], cval + cptr[j], (int)(cptr[j + 1] - cptr[j]));
        double acc = (q + (p - q) * s) / p;
        int kept = 0;
        if (poisson) {
            /* candidates: Poisson(p) given >= 1, by inversion */
            double v = next_u01(&r);
            double term = p * exp(-p) / hit, cdf = term;
            int m = 1;
            while (v > cdf && m < 1000) {
                ++m;
                term *= p / m;
                cdf += term;
            }
            for (int c = 0; c < m; ++c)
                if (next_u01(&r) <= acc) ++kept;
        } else {
            kept = next_u01(&r) <= acc ? 1 : 0;
        }
        if (kept > 0) {
            if (out_cols) {
                out_cols[cnt] = (int32_t)j;
                if (out_w) out_w[cnt] = (float)kept;
            }
            ++cnt;
        }
    }
    return cnt;
}

void pairs_count(int64_t n_rows, int64_t n_cols, int triangular, int poisson, double p, double q, uint64_t seed,
                 const int64_t* rptr, const int32_t* ridx, const double* rval,
                 const int64_t* cptr, const int32_t* cidx, const double* cval, int64_t* counts) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_rows; ++i)
        counts[i] = walk_row_gen(i, n_cols, triangular, poisson, p, q, seed, rptr, ridx, rval, cptr, cidx, cval,
                                 NULL, NULL);
}

void pairs_fill(int64_t n_rows, int64_t n_cols, int triangular, int poisson, double p, double q, uint64_t seed,
                const int64_t* rptr, const int32_t* ridx, const double* rval,
                const int64_t* cptr, const int32_t* cidx, const double* cval,
                const int64_t* offsets, int32_t* cols, float* weights) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_rows; ++i)
        walk_row_gen(i, n_cols, triangular, poisson, p, q, seed, rptr, ridx, rval, cptr, cidx, cval,
                     cols + offsets[i], weights ? weights + offsets[i] : NULL);
}
