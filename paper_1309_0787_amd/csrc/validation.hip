// Validation of recovered memberships against ground truth (Section 5.1,
// p-value testing; Section 5.2, evaluation metrics).  FP64 arithmetic on FP32
// membership matrices Pi_hat (k_hat x n) and Pi (k x n).
//
//  * row_stats: mean and centred sum of squares of every row (one workgroup
//    per row, fixed-order tree reduction).
//  * pair_stats: for every (i, j), the centred cross sum and the l1 distance
//    sum over a chunk of the n nodes (16 x 16 output tiles, rows staged in
//    LDS), then a fixed-order reduction over the chunks.
//  * finalize: rho, the t statistic T = rho sqrt(n-2)/sqrt(1-rho^2) and the
//    right p-value P(t_(n-2) > T) through the regularized incomplete beta
//    function, P(t_nu > T) = I_(nu/(nu+T^2))(nu/2, 1/2) / 2 for T >= 0,
//    evaluated by its continued fraction with Lentz's method (and the
//    symmetry I_x(a, b) = 1 - I_(1-x)(b, a) past the fraction's convergence
//    boundary).
//  * Benjamini-Hochberg: rank of every p-value (ties by position), then in
//    one workgroup the running minimum of m p_(r) / r from the largest rank
//    down, capped at 1; edges p_adj <= threshold; recovery ratio and error.
//  * bridgeness (Eq. bridgeness) and its degree-corrected form.
#include <cmath>

#include "otm_internal.h"

namespace otm {
namespace {

constexpr int kStatThreads = 256;
constexpr int kTile = 16;
constexpr int kChunk = 128;          // nodes staged per LDS round
constexpr int kNodesPerBlock = 2048; // nodes per split of the pair sums
constexpr int kMaxTests = 16384;     // k_hat * k (128 x 128)

__device__ double block_sum(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kStatThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// rows 0..k_hat-1 from Pi_hat, k_hat..k_hat+k-1 from Pi
__global__ __launch_bounds__(kStatThreads) void row_stats_kernel(const float* __restrict__ Ph, int kh,
                                                                 const float* __restrict__ P, int n,
                                                                 double* __restrict__ mean, double* __restrict__ ss) {
    __shared__ double red[kStatThreads];
    const int r = blockIdx.x;
    const float* row = r < kh ? Ph + (size_t)r * n : P + (size_t)(r - kh) * n;
    double s = 0.0;
    for (int x = threadIdx.x; x < n; x += kStatThreads) s += row[x];
    const double mu = block_sum(s, red) / n;
    double q = 0.0;
    for (int x = threadIdx.x; x < n; x += kStatThreads) {
        const double d = row[x] - mu;
        q += d * d;
    }
    const double sq = block_sum(q, red);
    if (threadIdx.x == 0) {
        mean[r] = mu;
        ss[r] = sq;
    }
}

// partials over node split z: cross[z][i][j] = sum_x (a_ix - abar_i)(b_jx - bbar_j),
// l1[z][i][j] = sum_x |a_ix - b_jx|
__global__ __launch_bounds__(kTile * kTile) void pair_stats_kernel(const float* __restrict__ Ph, int kh,
                                                                   const float* __restrict__ P, int k, int n,
                                                                   const double* __restrict__ mean,
                                                                   double* __restrict__ cross, double* __restrict__ l1) {
    __shared__ double sa[kTile][kChunk + 1];
    __shared__ double sb[kTile][kChunk + 1];
    const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile, z = blockIdx.z;
    const int x0 = z * kNodesPerBlock, x1 = min(n, x0 + kNodesPerBlock);
    const int ti = threadIdx.x / kTile, tj = threadIdx.x % kTile;
    double c = 0.0, l = 0.0;
    for (int xb = x0; xb < x1; xb += kChunk) {
        for (int e = threadIdx.x; e < kTile * kChunk; e += kTile * kTile) {
            const int rr = e / kChunk, cc = e % kChunk;
            const int x = xb + cc;
            const int ia = i0 + rr, jb = j0 + rr;
            sa[rr][cc] = (ia < kh && x < x1) ? (double)Ph[(size_t)ia * n + x] : 0.0;
            sb[rr][cc] = (jb < k && x < x1) ? (double)P[(size_t)jb * n + x] : 0.0;
        }
        __syncthreads();
        const int cnt = min(kChunk, x1 - xb);
        const double ma = (i0 + ti < kh) ? mean[i0 + ti] : 0.0;
        const double mb = (j0 + tj < k) ? mean[kh + j0 + tj] : 0.0;
        for (int cc = 0; cc < cnt; ++cc) {
            const double a = sa[ti][cc], b = sb[tj][cc];
            c += (a - ma) * (b - mb);
            l += fabs(a - b);
        }
        __syncthreads();
    }
    const int i = i0 + ti, j = j0 + tj;
    if (i < kh && j < k) {
        cross[((size_t)z * kh + i) * k + j] = c;
        l1[((size_t)z * kh + i) * k + j] = l;
    }
}

// log of the regularized incomplete beta's prefactor x^a (1-x)^b / B(a, b),
// with log x and log(1-x) given (they come from log1p of the t statistic)
__device__ double log_front(double a, double b, double lx, double l1x) {
    return a * lx + b * l1x - (lgamma(a) + lgamma(b) - lgamma(a + b));
}

// 1 + d1/(1 + d2/(1 + ...)) for the incomplete beta's continued fraction
// (terms d_(2m+1) = -(a+m)(a+b+m)x / ((a+2m)(a+2m+1)),
//        d_(2m)   = m(b-m)x / ((a+2m-1)(a+2m))), by Lentz's method
__device__ double ibeta_fraction(double a, double b, double x) {
    const double tiny = 1e-300, eps = 1e-16;
    double f = 1.0, C = 1.0, D = 0.0;
    for (int j = 1; j <= 40000; ++j) {
        const int m = j / 2;
        double d;
        if (j & 1)
            d = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
        else
            d = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
        D = 1.0 + d * D;
        if (fabs(D) < tiny) D = tiny;
        C = 1.0 + d / C;
        if (fabs(C) < tiny) C = tiny;
        D = 1.0 / D;
        const double delta = C * D;
        f *= delta;
        if (fabs(delta - 1.0) < eps) break;
    }
    return f;
}

// P(t_nu > T)
__device__ double student_right_tail(double T, double nu) {
    if (isinf(T)) return T > 0 ? 0.0 : 1.0;
    if (T == 0.0) return 0.5;
    const double a = 0.5 * nu, b = 0.5;
    const double r = T * T / nu;
    const double x = 1.0 / (1.0 + r);                 // nu / (nu + T^2)
    const double lx = -log1p(r);                       // log x
    const double l1x = log(r) - log1p(r);              // log (1 - x)
    double I;                                          // I_x(a, b)
    if (x < (a + 1.0) / (a + b + 2.0))
        I = exp(log_front(a, b, lx, l1x)) / (a * ibeta_fraction(a, b, x));
    else
        I = 1.0 - exp(log_front(a, b, lx, l1x)) / (b * ibeta_fraction(b, a, 1.0 - x));
    const double half = 0.5 * I;
    return T > 0 ? half : 1.0 - half;
}

__global__ void finalize_kernel(const double* __restrict__ cross, const double* __restrict__ l1p, int nz, int kh, int k,
                                int n, const double* __restrict__ ss, double* __restrict__ rho,
                                double* __restrict__ pval, double* __restrict__ l1) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kh * k) return;
    const int i = e / k, j = e % k;
    double c = 0.0, l = 0.0;
    for (int z = 0; z < nz; ++z) {
        c += cross[(size_t)z * kh * k + e];
        l += l1p[(size_t)z * kh * k + e];
    }
    const double den = sqrt(ss[i]) * sqrt(ss[kh + j]);
    const double r = den > 0.0 ? c / den : 0.0;
    const double rc = fmax(-1.0, fmin(1.0, r));
    const double nu = n - 2.0;
    double T;
    if (fabs(rc) >= 1.0)
        T = rc > 0 ? INFINITY : -INFINITY;
    else
        T = rc * sqrt(nu) / sqrt(1.0 - rc * rc);
    rho[e] = r;
    pval[e] = student_right_tail(T, nu);
    l1[e] = l / n;
}

// rank of p[e] among the m values (ties: lower position first)
constexpr int kRankThreads = 256;
__global__ __launch_bounds__(kRankThreads) void rank_kernel(const double* __restrict__ p, int m, int* __restrict__ rank) {
    __shared__ double sp[kRankThreads];
    const int e = blockIdx.x * kRankThreads + threadIdx.x;
    const double pe = e < m ? p[e] : 0.0;
    int r = 0;
    for (int b = 0; b < m; b += kRankThreads) {
        const int f = b + threadIdx.x;
        sp[threadIdx.x] = f < m ? p[f] : 0.0;
        __syncthreads();
        const int cnt = min(kRankThreads, m - b);
        for (int t = 0; t < cnt; ++t) {
            const double q = sp[t];
            const int f2 = b + t;
            r += (q < pe || (q == pe && f2 < e)) ? 1 : 0;
        }
        __syncthreads();
    }
    if (e < m) rank[e] = r;
}

// One workgroup: BH adjustment, edges, recovery ratio and error.
constexpr int kBhThreads = 1024;
__global__ __launch_bounds__(kBhThreads) void bh_scores_kernel(const double* __restrict__ p, const int* __restrict__ rank,
                                                               int kh, int k, double threshold,
                                                               const double* __restrict__ l1, double* __restrict__ padj,
                                                               int32_t* __restrict__ edges, double* __restrict__ scores) {
    __shared__ double q[kMaxTests];
    __shared__ double bmin[kBhThreads];
    __shared__ double red[kBhThreads];
    __shared__ int cnt[kBhThreads];
    const int m = kh * k, t = threadIdx.x;
    for (int e = t; e < m; e += kBhThreads) {
        const int r = rank[e];
        q[r] = p[e] * m / (r + 1.0);
    }
    __syncthreads();
    // suffix minimum: thread t owns the contiguous ranks [t*per, (t+1)*per)
    const int per = (m + kBhThreads - 1) / kBhThreads;
    const int lo = t * per, hi = min(m, lo + per);
    double run = INFINITY;
    for (int r = hi - 1; r >= lo; --r) {
        run = fmin(run, q[r]);
        q[r] = run;
    }
    bmin[t] = run;
    __syncthreads();
    if (t == 0) {   // minimum of the later segments, from the last down
        double acc = INFINITY;
        for (int u = kBhThreads - 1; u >= 0; --u) {
            const double v = bmin[u];
            bmin[u] = acc;
            acc = fmin(acc, v);
        }
    }
    __syncthreads();
    const double later = bmin[t];
    for (int r = lo; r < hi; ++r) q[r] = fmin(q[r], later);
    __syncthreads();
    for (int e = t; e < m; e += kBhThreads) {
        const double v = fmin(1.0, q[rank[e]]);
        padj[e] = v;
        edges[e] = v <= threshold ? 1 : 0;
    }
    __syncthreads();
    // recovery ratio: true communities j with an edge; error: sum of l1 over edges / k
    double err = 0.0;
    int matched = 0;
    for (int j = t; j < k; j += kBhThreads) {
        bool any = false;
        double s = 0.0;
        for (int i = 0; i < kh; ++i) {
            const int e = i * k + j;
            const bool on = fmin(1.0, q[rank[e]]) <= threshold;
            any = any || on;
            if (on) s += l1[e];
        }
        matched += any ? 1 : 0;
        err += s;
    }
    red[t] = err;
    cnt[t] = matched;
    __syncthreads();
    for (int s = kBhThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[t] += red[t + s];
            cnt[t] += cnt[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        scores[0] = (double)cnt[0] / k;
        scores[1] = red[0] / k;
    }
}

__global__ void bridgeness_kernel(const float* __restrict__ Ph, int kh, int n, otm_csr G, int has_g,
                                  double* __restrict__ b, double* __restrict__ Bd) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    double s = 0.0;
    const double u = 1.0 / kh;
    for (int j = 0; j < kh; ++j) {
        const double d = Ph[(size_t)j * n + x] - u;
        s += d * d;
    }
    const double bx = 1.0 - sqrt(kh / (kh - 1.0) * s);
    b[x] = bx;
    if (Bd) {
        double deg = 0.0;
        if (has_g) {
            int64_t p0 = G.rowptr[x], p1 = G.rowptr[x + 1];
            p0 = p0 < 0 ? 0 : (p0 > G.nnz ? G.nnz : p0);
            p1 = p1 < p0 ? p0 : (p1 > G.nnz ? G.nnz : p1);
            for (int64_t p = p0; p < p1; ++p) deg += G.vals ? (double)G.vals[p] : 1.0;
        }
        Bd[x] = deg * bx;
    }
}

int n_splits(int n) { return (n + kNodesPerBlock - 1) / kNodesPerBlock; }

}  // namespace
}  // namespace otm

using namespace otm;

extern "C" size_t otm_validate_workspace(int32_t k_hat, int32_t k, int32_t n) {
    if (k_hat < 1 || k < 1 || n < 3) return 0;
    const size_t m = (size_t)k_hat * k;
    size_t b = ws_round(sizeof(double) * (k_hat + k)) * 2;            // means, sums of squares
    b += ws_round(sizeof(double) * m * n_splits(n)) * 2;              // partial cross and l1 sums
    b += ws_round(sizeof(int) * m);                                   // ranks
    return b;
}

extern "C" int otm_validate(const float* Pi_hat, int32_t k_hat, const float* Pi, int32_t k, int32_t n, double threshold,
                            double* rho, double* pval, double* padj, int32_t* edges, double* l1, double* scores,
                            void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(Pi_hat && Pi && rho && pval && padj && edges && l1 && scores, OTM_EINVAL,
                "no array argument may be NULL");
    OTM_REQUIRE(k_hat >= 1 && k >= 1 && (int64_t)k_hat * k <= kMaxTests, OTM_ECAPACITY,
                "need k_hat * k <= 16384 tests");
    OTM_REQUIRE(n >= 3, OTM_ESHAPE, "need n >= 3 nodes (n - 2 degrees of freedom)");
    OTM_REQUIRE(std::isfinite(threshold) && threshold >= 0.0, OTM_EINVAL, "threshold must be finite and >= 0");
    OTM_REQUIRE(ws && ws_bytes >= otm_validate_workspace(k_hat, k, n), OTM_EWORKSPACE, "validate workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    const int m = k_hat * k, nz = n_splits(n);
    double* mean = wc.take<double>(k_hat + k);
    double* ss = wc.take<double>(k_hat + k);
    double* cross = wc.take<double>((size_t)m * nz);
    double* l1p = wc.take<double>((size_t)m * nz);
    int* rank = wc.take<int>(m);
    int st;
    hipLaunchKernelGGL(row_stats_kernel, dim3(k_hat + k), dim3(kStatThreads), 0, s, Pi_hat, k_hat, Pi, n, mean, ss);
    if ((st = check_launch("row_stats_kernel")) != OTM_OK) return st;
    dim3 grid((k_hat + kTile - 1) / kTile, (k + kTile - 1) / kTile, nz);
    hipLaunchKernelGGL(pair_stats_kernel, grid, dim3(kTile * kTile), 0, s, Pi_hat, k_hat, Pi, k, n, mean, cross, l1p);
    if ((st = check_launch("pair_stats_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(finalize_kernel, dim3((m + 255) / 256), dim3(256), 0, s, cross, l1p, nz, k_hat, k, n, ss, rho,
                       pval, l1);
    if ((st = check_launch("finalize_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(rank_kernel, dim3((m + kRankThreads - 1) / kRankThreads), dim3(kRankThreads), 0, s, pval, m, rank);
    if ((st = check_launch("rank_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(bh_scores_kernel, dim3(1), dim3(kBhThreads), 0, s, pval, rank, k_hat, k, threshold, l1, padj,
                       edges, scores);
    return check_launch("bh_scores_kernel");
}

extern "C" int otm_bridgeness(const float* Pi_hat, int32_t k_hat, int32_t n, const otm_csr* G, double* b,
                              double* b_degree, otm_stream stream) {
    OTM_REQUIRE(Pi_hat && b, OTM_EINVAL, "Pi_hat and b must not be NULL");
    OTM_REQUIRE(k_hat >= 2 && n >= 0, OTM_ESHAPE, "need k_hat >= 2");
    otm_csr g{};
    int has_g = 0;
    if (G) {
        int st = validate_csr_header(G, "G");
        if (st != OTM_OK) return st;
        OTM_REQUIRE(G->n_rows == n, OTM_ESHAPE, "G must have one row per node");
        g = *G;
        has_g = 1;
    }
    OTM_REQUIRE(b_degree == nullptr || has_g, OTM_EINVAL, "the degree-corrected form needs the graph G");
    if (n == 0) return OTM_OK;
    hipLaunchKernelGGL(bridgeness_kernel, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), Pi_hat, k_hat, n, g,
                       has_g, b, b_degree);
    return check_launch("bridgeness_kernel");
}
