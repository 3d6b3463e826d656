// FP64 dense linear algebra of the whitening and post-processing steps.
//
//  * gemm_tn: C = A^T B for tall A, B (d x p, d x q): split-K partials over row
//    chunks, then a fixed-order reduction.
//  * gemm_nn: C = A B with A tall (d x p) and B small (p x q).
//  * eigenproblems of the small symmetric matrices go to the Jacobi solver of
//    jacobi.hip.
//  * whitener (Section 3.1; Section 4.2, randomized tall-thin SVD with the
//    projected matrix truncated to its top k eigenpairs):
//      Omega = sym(S^T O) -> eig -> B = O U_k sigma_k^(-1/2)
//      B^T B = V_B diag(s^2) V_B^T -> W = B V_B diag(s^-2) = U_B diag(s)^-1
//      and every column of W turned so that its largest |entry| is positive.
//  * orthonormalize: an orthonormal basis Q of span(Y) for the power iterations
//    of the sketch, by Cholesky QR applied twice (m <= 200), else
//    Y (Y^T Y)^(-1/2) through the eigensolver.
//  * unwhiten_topics (Lemma postprocessing).
#include <cmath>

#include "otm_internal.h"

namespace otm {
namespace {

// ------------------------------------------------------------------ gemm_tn
constexpr int kTnRows = 16;

// A block owns a TILE x TILE tile of C and one chunk of rows; a thread owns
// the (TILE/16)^2 entries (p0 + ty + 16 i, q0 + tx + 16 j), TILE/32
// multiply-adds per LDS read (64-tiles for the wide sketch products, 32-tiles
// where 64 would leave most of a tile empty).  Each entry sums its chunk's
// rows in order.
template <int kTnTile>
__global__ __launch_bounds__(256) void gemm_tn_partial_kernel(const double* __restrict__ A, int lda,
                                                              const double* __restrict__ B, int ldb, int d, int p,
                                                              int q, int chunk, double* __restrict__ part) {
    constexpr int PT = kTnTile / 16;
    __shared__ double sA[kTnRows][kTnTile + 1];
    __shared__ double sB[kTnRows][kTnTile + 1];
    const int p0 = blockIdx.x * kTnTile, q0 = blockIdx.y * kTnTile;
    const int r0 = blockIdx.z * chunk, r1 = min(d, r0 + chunk);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[PT][PT];
#pragma unroll
    for (int i = 0; i < PT; ++i)
#pragma unroll
        for (int j = 0; j < PT; ++j) acc[i][j] = 0.0;
    for (int rb = r0; rb < r1; rb += kTnRows) {
        for (int e = threadIdx.x; e < kTnRows * kTnTile; e += 256) {
            const int rr = e / kTnTile, cc = e % kTnTile;
            const int r = rb + rr;
            sA[rr][cc] = (r < r1 && p0 + cc < p) ? A[(size_t)r * lda + p0 + cc] : 0.0;
            sB[rr][cc] = (r < r1 && q0 + cc < q) ? B[(size_t)r * ldb + q0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < kTnRows; ++rr) {
            double a[PT], b[PT];
#pragma unroll
            for (int i = 0; i < PT; ++i) a[i] = sA[rr][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < PT; ++j) b[j] = sB[rr][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < PT; ++i)
#pragma unroll
                for (int j = 0; j < PT; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
    double* out = part + (size_t)blockIdx.z * p * q;
#pragma unroll
    for (int i = 0; i < PT; ++i)
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            const int pi = p0 + ty + 16 * i, qj = q0 + tx + 16 * j;
            if (pi < p && qj < q) out[(size_t)pi * q + qj] = acc[i][j];
        }
}

__global__ void reduce_parts_kernel(const double* __restrict__ part, int nparts, int64_t m, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[(size_t)b * m + i];
    out[i] = s;
}

int tn_chunks(int d) {
    int c = (d + 511) / 512;
    return c < 1 ? 1 : (c > 64 ? 64 : c);
}

size_t gemm_tn_ws(int d, int p, int q) { return ws_round(sizeof(double) * (size_t)tn_chunks(d) * p * q); }

int gemm_tn(const double* A, int lda, const double* B, int ldb, int d, int p, int q, double* C, double* part,
            hipStream_t s) {
    const int nch = tn_chunks(d);
    const int chunk = (d + nch - 1) / nch;
    if (p > 128 && q > 128)
        hipLaunchKernelGGL(gemm_tn_partial_kernel<64>, dim3((p + 63) / 64, (q + 63) / 64, nch), dim3(256), 0, s, A, lda,
                           B, ldb, d, p, q, chunk, part);
    else
        hipLaunchKernelGGL(gemm_tn_partial_kernel<32>, dim3((p + 31) / 32, (q + 31) / 32, nch), dim3(256), 0, s, A, lda,
                           B, ldb, d, p, q, chunk, part);
    int st = check_launch("gemm_tn_partial_kernel");
    if (st != OTM_OK) return st;
    const int64_t m = (int64_t)p * q;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, part, nch, m, C);
    return check_launch("reduce_parts_kernel");
}

// ------------------------------------------------------------------ gemm_nn
constexpr int kNnM = 64, kNnN = 64, kNnK = 16;

__global__ __launch_bounds__(256) void gemm_nn_kernel(const double* __restrict__ A, int lda, const double* __restrict__ B,
                                                      int ldb, double* __restrict__ C, int ldc, int d, int p, int q) {
    __shared__ double sA[kNnK][kNnM + 1];
    __shared__ double sB[kNnK][kNnN + 1];
    const int r0 = blockIdx.x * kNnM, c0 = blockIdx.y * kNnN;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;   // rows r0+ty+16i, cols c0+tx+16j
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < p; k0 += kNnK) {
        for (int e = threadIdx.x; e < kNnK * kNnM; e += 256) {
            const int rr = e / kNnK, kk = e % kNnK;
            const int r = r0 + rr, kx = k0 + kk;
            sA[kk][rr] = (r < d && kx < p) ? A[(size_t)r * lda + kx] : 0.0;
        }
        for (int e = threadIdx.x; e < kNnK * kNnN; e += 256) {
            const int kk = e / kNnN, cc = e % kNnN;
            const int kx = k0 + kk, c = c0 + cc;
            sB[kk][cc] = (kx < p && c < q) ? B[(size_t)kx * ldb + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kNnK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sB[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
            if (r < d && c < q) C[(size_t)r * ldc + c] = acc[i][j];
        }
}

int gemm_nn(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int d, int p, int q,
            hipStream_t s) {
    dim3 grid((d + kNnM - 1) / kNnM, (q + kNnN - 1) / kNnN);
    hipLaunchKernelGGL(gemm_nn_kernel, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, d, p, q);
    return check_launch("gemm_nn_kernel");
}

constexpr int kJacMaxN = 256;

// ---------------------------------------------------------------- whitener
__global__ void symmetrize_kernel(double* __restrict__ A, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int i = e / n, j = e % n;
    if (i < j) {
        const double m = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
        A[(size_t)i * n + j] = m;
        A[(size_t)j * n + i] = m;
    }
}

// Pk[:, j] = V[:, order[j]] / sqrt(sigma_order[j]), j < k;  info = 1 if sigma_k not positive enough
__global__ void top_k_scale_kernel(const double* __restrict__ V, const double* __restrict__ ev,
                                   const int* __restrict__ order, int n, int k, double* __restrict__ Pk,
                                   int32_t* info) {
    const double s1 = ev[order[0]], sk = ev[order[k - 1]];
    const bool ok = (sk > 0.0) && (sk > 1e-12 * fmax(s1, 0.0));
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = ok ? 0 : 1;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int r = e / k, j = e % k;
    const int src = order[j];
    Pk[e] = ok ? V[(size_t)r * n + src] / sqrt(ev[src]) : 0.0;
}

// Pw[:, j] = V[:, order[j]] / ev[order[j]];  evals_out[j] = ev[order[j]]
__global__ void whiten_scale_kernel(const double* __restrict__ V, const double* __restrict__ ev,
                                    const int* __restrict__ order, int k, const int32_t* info,
                                    double* __restrict__ Pw, double* __restrict__ evals_out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * k) return;
    const int r = e / k, j = e % k;
    const int src = order[j];
    const double v = ev[src];
    Pw[e] = (*info == 0 && v > 0.0) ? V[(size_t)r * k + src] / v : 0.0;
    if (r == 0) evals_out[j] = v;
}

// per column: (max |W[r][j]|, first row reaching it) over a block of rows
constexpr int kSignBlocks = 128;
__global__ void colmax_partial_kernel(const double* __restrict__ W, int d, int k, double* __restrict__ pval,
                                      int* __restrict__ pidx) {
    const int per = (d + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(d, r0 + per);
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double best = -1.0;
        int bi = r0;
        for (int r = r0; r < r1; ++r) {
            const double v = fabs(W[(size_t)r * k + j]);
            if (v > best) { best = v; bi = r; }
        }
        pval[(size_t)blockIdx.x * k + j] = best;
        pidx[(size_t)blockIdx.x * k + j] = bi;
    }
}

__global__ void colsign_kernel(const double* __restrict__ W, const double* __restrict__ pval,
                               const int* __restrict__ pidx, int nparts, int k, double* __restrict__ sign) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    double best = -1.0;
    int bi = 0;
    for (int b = 0; b < nparts; ++b) {
        const double v = pval[(size_t)b * k + j];
        if (v > best) { best = v; bi = pidx[(size_t)b * k + j]; }
    }
    sign[j] = (W[(size_t)bi * k + j] < 0.0) ? -1.0 : 1.0;
}

// W *= sign per column; W_lo (row stride ldw_lo, or ldw_lo = k when absent)
// gets the rounded copy and zeros in its padding columns k..ldw_lo-1.
__global__ void apply_sign_kernel(double* __restrict__ W, const double* __restrict__ sign, int d, int k,
                                  void* __restrict__ W_lo, int lo_dtype, int ldw_lo) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * ldw_lo) return;
    const int64_t row = e / ldw_lo;
    const int col = static_cast<int>(e - row * ldw_lo);
    double v = 0.0;
    if (col < k) {
        v = W[row * k + col] * sign[col];
        W[row * k + col] = v;
    }
    if (W_lo) {
        if (lo_dtype == OTM_F32) static_cast<float*>(W_lo)[e] = static_cast<float>(v);
        else static_cast<__bf16*>(W_lo)[e] = f32_to_bf16(static_cast<float>(v));
    }
}

// Pq[:, j] = V[:, j] / sqrt(ev[j]) for the orthonormal basis Y (Y^T Y)^(-1/2);
// info = 1 if an eigenvalue of the Gram is not positive enough (rank deficient);
// written on pass 0, or-ed on pass 1
__global__ void orth_scale_kernel(const double* __restrict__ V, const double* __restrict__ ev, int m,
                                  double* __restrict__ Pq, int32_t* info, int pass) {
    double emax = 0.0;
    for (int j = 0; j < m; ++j) emax = fmax(emax, ev[j]);
    bool ok = emax > 0.0;
    for (int j = 0; j < m; ++j) ok = ok && (ev[j] > 1e-14 * emax);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && (pass == 0 || !ok)) *info = ok ? 0 : 1;
    if (e >= m * m) return;
    const int j = e % m;
    Pq[e] = ok ? V[e] / sqrt(ev[j]) : 0.0;
}

// Cholesky of an m x m Gram G = L L^T held in LDS (packed lower triangle,
// m <= 200) and Rinv = (L^T)^(-1), upper triangular, m x m row-major, so that
// Y Rinv has orthonormal columns.  info = 1 (pass 0) or |= 1 (pass 1) when a
// pivot is not above 1e-14 of the largest diagonal entry; that pivot is then
// replaced by the largest diagonal entry so the results stay finite.
//
// Blocked by panels of kCholNB columns, three barriers per panel in each
// half instead of two per column:
//  * factorization, per panel J = [j0, j1): wave 0 factors the diagonal block
//    in registers (one lane per packed entry, columns exchanged by
//    shuffles); every row below solves its kCholNB entries against it; the
//    trailing rows take the rank-kCholNB update.  The updates of an entry
//    are applied column by column in the same order as the unblocked
//    right-looking algorithm.
//  * inverse X = L^-1 in place, panels from the last: X[i][c] for the rows
//    below the panel from (X L)[i][c] = 0, i.e.
//    X[i][c] = -(1/L_cc) sum_{c < l <= i} X[i][l] L[l][c], whose terms with
//    l past the panel are split over S lanes of a wave; then one thread per
//    column inverts the diagonal block from (L X)[r][c] = 0.  The new entries
//    are held in registers (or a small LDS block) until every read of the
//    panel's L entries is done.  The reciprocals 1/L_jj are kept from the
//    factorization, so the inverse divides nowhere.
constexpr int kCholN = 200;
constexpr int kCholThreads = 1024;
constexpr int kCholNB = 8;
constexpr int kCholLoads = 8;      // global loads in flight per thread while filling LDS

__device__ __forceinline__ int low_idx(int i, int j) { return i * (i + 1) / 2 + j; }

// lane p of the packed nb x nb block: (r, c) with p = r (r + 1) / 2 + c, c <= r
__device__ __forceinline__ bool block_entry(int p, int nb, int& r, int& c) {
    r = 0;
    c = 0;
    if (p >= nb * (nb + 1) / 2) return false;
    while ((r + 1) * (r + 2) / 2 <= p) ++r;
    c = p - r * (r + 1) / 2;
    return true;
}

__global__ __launch_bounds__(kCholThreads) void chol_rinv_kernel(const double* __restrict__ G, int m,
                                                                 double* __restrict__ Rinv, int32_t* info, int pass) {
    __shared__ double sL[kCholN * (kCholN + 1) / 2];
    __shared__ double s_rdiag[kCholN];                 // 1 / L_jj
    __shared__ double s_xblk[kCholNB * kCholNB];       // inverse of a diagonal block, column-major
    __shared__ double s_dmax;
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // symmetrized lower triangle 0.5 (G[i][j] + G[j][i]) from coalesced reads
    // of G in two passes (the lower entries, then the upper ones added); a
    // thread's loads of a pass are issued together
    for (int half = 0; half < 2; ++half) {
        for (int base = 0; base < m * m; base += kCholThreads * kCholLoads) {
            double g[kCholLoads];
#pragma unroll
            for (int u = 0; u < kCholLoads; ++u) {
                const int e = base + u * kCholThreads + tid;
                g[u] = (e < m * m) ? G[e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kCholLoads; ++u) {
                const int e = base + u * kCholThreads + tid;
                if (e < m * m) {
                    const int i = e / m, j = e % m;
                    if (half == 0 && j <= i) sL[low_idx(i, j)] = (j == i) ? g[u] : 0.5 * g[u];
                    if (half == 1 && j > i) sL[low_idx(j, i)] += 0.5 * g[u];
                }
            }
        }
        __syncthreads();
    }
    if (tid < 64) {
        double dm = 0.0;
        for (int i = lane; i < m; i += 64) dm = fmax(dm, sL[low_idx(i, i)]);
        for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o));
        if (lane == 0) {
            s_dmax = dm;
            s_bad = 0;
        }
    }
    __syncthreads();
    const double dmax = s_dmax;
    const double dfix = dmax > 0.0 ? dmax : 1.0;

    for (int j0 = 0; j0 < m; j0 += kCholNB) {
        const int nb = min(kCholNB, m - j0), j1 = j0 + nb;
        // diagonal block, wave 0
        if (tid < 64) {
            int r, c;
            const bool live = block_entry(lane, nb, r, c);
            double v = live ? sL[low_idx(j0 + r, j0 + c)] : 0.0;
            bool bad = false;
            for (int cc = 0; cc < nb; ++cc) {
                double d = __shfl(v, cc * (cc + 1) / 2 + cc);
                if (!(d > 1e-14 * dmax)) {   // not positive definite to working precision: reported, pivot replaced
                    bad = true;
                    d = dfix;
                }
                const double sq = sqrt(d), inv = 1.0 / sq;
                if (lane == 0) s_rdiag[j0 + cc] = inv;
                if (live && c == cc) v = (r == cc) ? sq : v * inv;
                const double lr = __shfl(v, r * (r + 1) / 2 + cc);   // L[r][cc]
                const double lc = __shfl(v, c * (c + 1) / 2 + cc);   // L[c][cc]
                if (live && c > cc) v -= lr * lc;
            }
            if (live) sL[low_idx(j0 + r, j0 + c)] = v;
            if (bad && lane == 0) s_bad = 1;
        }
        __syncthreads();
        // the panel's rows below the block.  Only the last panel can be
        // narrower than kCholNB, and it has no rows below it, so this phase
        // and the trailing update always work on full panels.
        for (int i = j1 + tid; i < m; i += kCholThreads) {
            double x[kCholNB];
#pragma unroll
            for (int c = 0; c < kCholNB; ++c) x[c] = sL[low_idx(i, j0 + c)];
#pragma unroll
            for (int c = 0; c < kCholNB; ++c) {
                double sacc = x[c];
#pragma unroll
                for (int t = 0; t < c; ++t) sacc -= x[t] * sL[low_idx(j0 + c, j0 + t)];
                x[c] = sacc * s_rdiag[j0 + c];
            }
#pragma unroll
            for (int c = 0; c < kCholNB; ++c) sL[low_idx(i, j0 + c)] = x[c];
        }
        __syncthreads();
        // trailing update A[i][l] -= sum_c L[i][c] L[l][c], j1 <= l <= i.  Rows
        // are taken in pairs (the r-th shortest with the r-th longest), S
        // threads per pair, so every thread has about the same number of
        // entries; two entries per iteration, loaded before either is stored.
        const int w = m - j1;
        if (w > 0) {
            const int pairs = (w + 1) / 2;
            const int S = max(1, kCholThreads / pairs);
            const int pr = tid / S, sub = tid % S;
            if (pr < pairs) {
                const int ia = j1 + pr, ib = m - 1 - pr;   // ia == ib: the middle row of an odd count
                const int la = ia - j1 + 1, lb = (ib != ia) ? ib - j1 + 1 : 0;
                double lia[kCholNB], lib[kCholNB];
#pragma unroll
                for (int c = 0; c < kCholNB; ++c) {
                    lia[c] = sL[low_idx(ia, j0 + c)];
                    lib[c] = sL[low_idx(ib, j0 + c)];
                }
                for (int t = sub; t < la + lb; t += 2 * S) {
                    const int u = t + S;
                    const bool two = u < la + lb;
                    const bool fa = t < la, fb = u < la;
                    const int l1 = j1 + (fa ? t : t - la), l2 = j1 + (fb ? u : u - la);
                    double* p1 = sL + low_idx(fa ? ia : ib, l1);
                    double* p2 = sL + low_idx(fb ? ia : ib, two ? l2 : l1);
                    const double* L1 = sL + low_idx(l1, j0);
                    const double* L2 = sL + low_idx(two ? l2 : l1, j0);
                    double a1 = *p1, a2 = *p2;
                    double x1[kCholNB], x2[kCholNB];
#pragma unroll
                    for (int c = 0; c < kCholNB; ++c) {
                        x1[c] = L1[c];
                        x2[c] = L2[c];
                    }
#pragma unroll
                    for (int c = 0; c < kCholNB; ++c) {
                        a1 -= (fa ? lia[c] : lib[c]) * x1[c];
                        a2 -= (fb ? lia[c] : lib[c]) * x2[c];
                    }
                    *p1 = a1;
                    if (two) *p2 = a2;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && (pass == 0 || s_bad)) *info = s_bad;

    for (int jb = ((m - 1) / kCholNB) * kCholNB; jb >= 0; jb -= kCholNB) {
        const int nb = min(kCholNB, m - jb), j1 = jb + nb;
        const int w = m - j1;
        // four lanes per row (at most 192 rows): measured faster than wider
        // splits, whose shuffle reduction costs more than the shorter loop
        int S = 4;
        while (S > 1 && S * w > kCholThreads) S >>= 1;
        const int row = tid / S, sub = tid % S;
        const bool has_row = w > 0 && row < w;
        const int i = j1 + row;
        double xr[kCholNB];
        if (w > 0) {   // a panel with rows below it is full (nb == kCholNB)
            double z[kCholNB];
#pragma unroll
            for (int c = 0; c < kCholNB; ++c) z[c] = 0.0;
            if (has_row) {
                const double* Xi = sL + low_idx(i, 0);
                for (int l = j1 + sub; l <= i; l += S) {
                    const double xil = Xi[l];
                    const double* Ll = sL + low_idx(l, jb);
#pragma unroll
                    for (int c = 0; c < kCholNB; ++c) z[c] += xil * Ll[c];
                }
            }
            // every lane of a wave takes part (S lanes per row, S a power of two)
#pragma unroll
            for (int c = 0; c < kCholNB; ++c)
                for (int o = S >> 1; o > 0; o >>= 1) z[c] += __shfl_xor(z[c], o);
#pragma unroll
            for (int c = kCholNB - 1; c >= 0; --c) {
                double acc = z[c];
#pragma unroll
                for (int l = c + 1; l < kCholNB; ++l) acc += xr[l] * sL[low_idx(jb + l, jb + c)];
                xr[c] = -acc * s_rdiag[jb + c];
            }
        }
        __syncthreads();   // every read of the panel's L entries is done
        if (has_row && sub == 0) {
#pragma unroll
            for (int c = 0; c < kCholNB; ++c) sL[low_idx(i, jb + c)] = xr[c];
        }
        // the diagonal block's inverse from L X = I: thread c of wave 0 takes
        // column c, X[r][c] = -(1/L_rr) sum_{c <= l < r} L[r][l] X[l][c]; the
        // block is overwritten once every column is done
        if (tid < nb) {
            const int c = tid;
            double xc[kCholNB];
#pragma unroll
            for (int r = 0; r < kCholNB; ++r) {
                xc[r] = 0.0;
                if (r >= c && r < nb) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < r; ++l)
                        if (l >= c) acc += sL[low_idx(jb + r, jb + l)] * xc[l];
                    xc[r] = (r == c) ? s_rdiag[jb + r] : -s_rdiag[jb + r] * acc;
                }
            }
#pragma unroll
            for (int r = 0; r < kCholNB; ++r) s_xblk[c * kCholNB + r] = xc[r];
        }
        __syncthreads();
        if (tid < nb * kCholNB) {
            const int c = tid / kCholNB, r = tid % kCholNB;
            if (r >= c && r < nb) sL[low_idx(jb + r, jb + c)] = s_xblk[c * kCholNB + r];
        }
        __syncthreads();
    }
    for (int e = tid; e < m * m; e += kCholThreads) {
        const int c = e / m, ii = e % m;
        Rinv[e] = (ii >= c) ? sL[low_idx(ii, c)] : 0.0;
    }
}

// ------------------------------------------------------------- unwhitening
// lambda_i = kappa ||phi_i||^3, UL[a][i] = lambda_i u_i[a], alpha_hat
__global__ void factor_stats_kernel(const float* __restrict__ Phi, int k, double kappa, double* __restrict__ lam,
                                    double* __restrict__ UL, double* __restrict__ alpha_hat) {
    __shared__ double s_inv2[kMaxK];
    __shared__ double s_total;
    const int i = threadIdx.x;
    if (i < k) {
        double nn = 0.0;
        for (int a = 0; a < k; ++a) {
            const double v = Phi[(size_t)i * k + a];
            nn += v * v;
        }
        const double nrm = sqrt(nn);
        const double l = kappa * nrm * nn;
        lam[i] = l;
        for (int a = 0; a < k; ++a) UL[(size_t)a * k + i] = l * Phi[(size_t)i * k + a] / nrm;
        s_inv2[i] = 1.0 / (l * l);
    }
    __syncthreads();
    if (i == 0) {
        double t = 0.0;
        for (int j = 0; j < k; ++j) t += s_inv2[j];
        s_total = t;
    }
    __syncthreads();
    if (i < k && alpha_hat) alpha_hat[i] = s_inv2[i] / s_total;
}

// Ginv = V diag(1/ev) V^T (k x k); info = 1 if an eigenvalue is not positive
__global__ void spd_inverse_kernel(const double* __restrict__ V, const double* __restrict__ ev, int k,
                                   double* __restrict__ Ginv, int32_t* info) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = true;
    double emax = 0.0;
    for (int m = 0; m < k; ++m) emax = fmax(emax, ev[m]);
    for (int m = 0; m < k; ++m) ok = ok && (ev[m] > 1e-300) && (ev[m] > 1e-14 * emax);
    if (e == 0) *info = ok ? 0 : 1;
    if (e >= k * k) return;
    const int r = e / k, c = e % k;
    double s = 0.0;
    for (int m = 0; m < k; ++m) s += V[(size_t)r * k + m] * V[(size_t)c * k + m] / ev[m];
    Ginv[e] = ok ? s : 0.0;
}

// per-block column sums of max(mu, 0), clipping mu in place
__global__ void clip_colsum_partial_kernel(double* __restrict__ mu, int d, int k, double* __restrict__ part) {
    const int per = (d + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(d, r0 + per);
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        double s = 0.0;
        for (int r = r0; r < r1; ++r) {
            double v = mu[(size_t)r * k + j];
            if (v < 0.0) { v = 0.0; mu[(size_t)r * k + j] = 0.0; }
            s += v;
        }
        part[(size_t)blockIdx.x * k + j] = s;
    }
}

__global__ void col_normalize_kernel(double* __restrict__ mu, const double* __restrict__ colsum, int d, int k) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * k) return;
    const double s = colsum[e % k];
    mu[e] = (s > 0.0) ? mu[e] / s : 0.0;
}

constexpr int kColBlocks = 128;

}  // namespace

// ------------------------------------------- shared with other translation units
size_t gemm_tn_f64_ws(int d, int p, int q) { return gemm_tn_ws(d, p, q); }
int gemm_tn_f64(const double* A, int lda, const double* B, int ldb, int d, int p, int q, double* C, double* part,
                hipStream_t s) {
    return gemm_tn(A, lda, B, ldb, d, p, q, C, part, s);
}
int gemm_nn_f64(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int d, int p, int q,
                hipStream_t s) {
    return gemm_nn(A, lda, B, ldb, C, ldc, d, p, q, s);
}

size_t cholqr2_ws(int d, int m) {
    size_t b = ws_round(sizeof(double) * (size_t)m * m) * 3;   // Gram, R1inv, R2inv
    b += gemm_tn_ws(d, m, m);
    b += ws_round(sizeof(double) * (size_t)d * m);             // first pass
    return b;
}

int cholqr2(const double* Y, int d, int m, double* Q, double* Rinv, int32_t* info, void* ws, hipStream_t s) {
    if (m > kCholN) return fail(OTM_ECAPACITY, "Cholesky QR needs m <= 200");
    WsCarver wc(ws, cholqr2_ws(d, m));
    double* Gr = wc.take<double>((size_t)m * m);
    double* R1 = wc.take<double>((size_t)m * m);
    double* R2 = wc.take<double>((size_t)m * m);
    double* part = wc.take<double>(gemm_tn_ws(d, m, m) / sizeof(double));
    double* Q1 = wc.take<double>((size_t)d * m);
    int st;
    const double* src = Y;
    for (int pass = 0; pass < 2; ++pass) {
        double* dst = pass == 0 ? Q1 : Q;
        double* Ri = pass == 0 ? R1 : R2;
        if ((st = gemm_tn(src, m, src, m, d, m, m, Gr, part, s)) != OTM_OK) return st;
        hipLaunchKernelGGL(chol_rinv_kernel, dim3(1), dim3(kCholThreads), 0, s, Gr, m, Ri, info, pass);
        if ((st = check_launch("chol_rinv_kernel")) != OTM_OK) return st;
        if ((st = gemm_nn(src, m, Ri, m, dst, m, d, m, m, s)) != OTM_OK) return st;
        src = Q1;
    }
    // Y = Q R2 R1, so R^-1 = R1^-1 R2^-1
    return gemm_nn(R1, m, R2, m, Rinv, m, m, m, m, s);
}

}  // namespace otm

using namespace otm;

extern "C" size_t otm_whitener_workspace(int32_t d, int32_t k_tilde, int32_t k) {
    if (d < 1 || k_tilde < 1 || k < 1) return 0;
    const size_t kt = k_tilde;
    size_t b = 0;
    b += ws_round(sizeof(double) * kt * kt) * 2;                      // Omega, V
    b += ws_round(sizeof(double) * kt) + ws_round(sizeof(int) * kt);  // ev, order
    b += ws_round(sizeof(double) * kt * k);                           // Pk
    b += ws_round(sizeof(double) * (size_t)d * k);                    // B
    b += ws_round(sizeof(double) * (size_t)k * k) * 3;                // Gram, V_B, Pw
    b += ws_round(sizeof(double) * k) + ws_round(sizeof(int) * k);    // ev_B, order_B
    size_t part = gemm_tn_ws(d, k_tilde, k_tilde);
    const size_t p2 = gemm_tn_ws(d, k, k);
    if (p2 > part) part = p2;
    b += part;
    b += ws_round(sizeof(double) * kSignBlocks * k) + ws_round(sizeof(int) * kSignBlocks * k);
    b += ws_round(sizeof(double) * k);                                // signs
    const size_t j1 = jacobi_ws_bytes(k_tilde), j2 = jacobi_ws_bytes(k);
    b += j1 > j2 ? j1 : j2;                                           // eigensolver log
    return b;
}

extern "C" int otm_whitener(const double* O, const double* S, int32_t d, int32_t k_tilde, int32_t k, double* W,
                            double* evals, void* W_lo, int w_lo_dtype, int32_t ldw_lo, int32_t* info, void* ws,
                            size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(O && S && W && evals && info, OTM_EINVAL, "O, S, W, evals, info must not be NULL");
    OTM_REQUIRE(d >= 1 && k >= 1 && k <= k_tilde && k_tilde <= kJacMaxN && k <= d, OTM_ESHAPE,
                "need 1 <= k <= k_tilde <= 256 and k <= d");
    OTM_REQUIRE(W_lo == nullptr || w_lo_dtype == OTM_F32 || w_lo_dtype == OTM_BF16, OTM_EDTYPE,
                "W_lo must be F32 or BF16");
    OTM_REQUIRE(W_lo == nullptr || ldw_lo >= k, OTM_ESHAPE, "need ldw_lo >= k");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_whitener_workspace(d, k_tilde, k), OTM_EWORKSPACE,
                "whitener workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    const int kt = k_tilde;
    double* Om = wc.take<double>((size_t)kt * kt);
    double* Vo = wc.take<double>((size_t)kt * kt);
    double* ev = wc.take<double>(kt);
    int* ord = wc.take<int>(kt);
    double* Pk = wc.take<double>((size_t)kt * k);
    double* Bm = wc.take<double>((size_t)d * k);
    double* Gr = wc.take<double>((size_t)k * k);
    double* Vb = wc.take<double>((size_t)k * k);
    double* Pw = wc.take<double>((size_t)k * k);
    double* evb = wc.take<double>(k);
    int* ordb = wc.take<int>(k);
    size_t part_bytes = gemm_tn_ws(d, kt, kt);
    if (gemm_tn_ws(d, k, k) > part_bytes) part_bytes = gemm_tn_ws(d, k, k);
    double* part = wc.take<double>(part_bytes / sizeof(double));
    double* pval = wc.take<double>((size_t)kSignBlocks * k);
    int* pidx = wc.take<int>((size_t)kSignBlocks * k);
    double* sgn = wc.take<double>(k);
    const size_t jb = jacobi_ws_bytes(kt) > jacobi_ws_bytes(k) ? jacobi_ws_bytes(kt) : jacobi_ws_bytes(k);
    void* jws = wc.take<char>(jb);
    int st;
    if ((st = gemm_tn(S, kt, O, kt, d, kt, kt, Om, part, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(symmetrize_kernel, dim3((kt * kt + 255) / 256), dim3(256), 0, s, Om, kt);
    if ((st = check_launch("symmetrize_kernel")) != OTM_OK) return st;
    if ((st = jacobi(Om, Vo, kt, ev, ord, jws, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(top_k_scale_kernel, dim3((kt * k + 255) / 256), dim3(256), 0, s, Vo, ev, ord, kt, k, Pk, info);
    if ((st = check_launch("top_k_scale_kernel")) != OTM_OK) return st;
    if ((st = gemm_nn(O, kt, Pk, k, Bm, k, d, kt, k, s)) != OTM_OK) return st;
    if ((st = gemm_tn(Bm, k, Bm, k, d, k, k, Gr, part, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(symmetrize_kernel, dim3((k * k + 255) / 256), dim3(256), 0, s, Gr, k);
    if ((st = check_launch("symmetrize_kernel")) != OTM_OK) return st;
    if ((st = jacobi(Gr, Vb, k, evb, ordb, jws, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(whiten_scale_kernel, dim3((k * k + 255) / 256), dim3(256), 0, s, Vb, evb, ordb, k, info, Pw,
                       evals);
    if ((st = check_launch("whiten_scale_kernel")) != OTM_OK) return st;
    if ((st = gemm_nn(Bm, k, Pw, k, W, k, d, k, k, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(colmax_partial_kernel, dim3(kSignBlocks), dim3(128), 0, s, W, d, k, pval, pidx);
    if ((st = check_launch("colmax_partial_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(colsign_kernel, dim3((k + 127) / 128), dim3(128), 0, s, W, pval, pidx, kSignBlocks, k, sgn);
    if ((st = check_launch("colsign_kernel")) != OTM_OK) return st;
    const int ld_lo = W_lo ? ldw_lo : k;
    const int64_t total = (int64_t)d * ld_lo;
    hipLaunchKernelGGL(apply_sign_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, W, sgn, d, k, W_lo,
                       w_lo_dtype, ld_lo);
    return check_launch("apply_sign_kernel");
}

extern "C" size_t otm_orthonormalize_workspace(int32_t d, int32_t m) {
    if (d < 1 || m < 1) return 0;
    size_t b = ws_round(sizeof(double) * (size_t)m * m) * 3;   // Gram, V / Rinv, Pq
    b += ws_round(sizeof(double) * m) + ws_round(sizeof(int) * m);
    b += gemm_tn_ws(d, m, m);
    b += ws_round(sizeof(double) * (size_t)d * m);               // first Cholesky-QR pass
    b += jacobi_ws_bytes(m);
    return b;
}

extern "C" int otm_orthonormalize(const double* Y, int32_t d, int32_t m, double* Q, int32_t* info, void* ws,
                                  size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(Y && Q && info, OTM_EINVAL, "Y, Q, info must not be NULL");
    OTM_REQUIRE(d >= 1 && m >= 1 && m <= d && m <= kJacMaxN, OTM_ESHAPE, "need 1 <= m <= min(d, 256)");
    OTM_REQUIRE(Y != Q, OTM_EINVAL, "Y and Q must not alias");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_orthonormalize_workspace(d, m), OTM_EWORKSPACE,
                "orthonormalize workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    double* Gr = wc.take<double>((size_t)m * m);
    double* V = wc.take<double>((size_t)m * m);
    double* Pq = wc.take<double>((size_t)m * m);
    double* ev = wc.take<double>(m);
    int* ord = wc.take<int>(m);
    double* part = wc.take<double>(gemm_tn_ws(d, m, m) / sizeof(double));
    double* Q1 = wc.take<double>((size_t)d * m);
    void* jws = wc.take<char>(jacobi_ws_bytes(m));
    int st;
    if (m <= kCholN) {
        // Cholesky QR twice: Q1 = Y R1^-1, Q = Q1 R2^-1 with R^T R the Gram of each input
        const double* src = Y;
        for (int pass = 0; pass < 2; ++pass) {
            double* dst = pass == 0 ? Q1 : Q;
            if ((st = gemm_tn(src, m, src, m, d, m, m, Gr, part, s)) != OTM_OK) return st;
            hipLaunchKernelGGL(chol_rinv_kernel, dim3(1), dim3(kCholThreads), 0, s, Gr, m, V, info, pass);
            if ((st = check_launch("chol_rinv_kernel")) != OTM_OK) return st;
            if ((st = gemm_nn(src, m, V, m, dst, m, d, m, m, s)) != OTM_OK) return st;
            src = Q1;
        }
        return OTM_OK;
    }
    // larger m: Q = Y (Y^T Y)^(-1/2), also applied twice
    const double* src = Y;
    for (int pass = 0; pass < 2; ++pass) {
        double* dst = pass == 0 ? Q1 : Q;
        if ((st = gemm_tn(src, m, src, m, d, m, m, Gr, part, s)) != OTM_OK) return st;
        hipLaunchKernelGGL(symmetrize_kernel, dim3((m * m + 255) / 256), dim3(256), 0, s, Gr, m);
        if ((st = check_launch("symmetrize_kernel")) != OTM_OK) return st;
        if ((st = jacobi(Gr, V, m, ev, ord, jws, s)) != OTM_OK) return st;
        hipLaunchKernelGGL(orth_scale_kernel, dim3((m * m + 255) / 256), dim3(256), 0, s, V, ev, m, Pq, info, pass);
        if ((st = check_launch("orth_scale_kernel")) != OTM_OK) return st;
        if ((st = gemm_nn(src, m, Pq, m, dst, m, d, m, m, s)) != OTM_OK) return st;
        src = Q1;
    }
    return OTM_OK;
}

extern "C" size_t otm_unwhiten_workspace(int32_t d, int32_t k) {
    if (d < 1 || k < 1) return 0;
    size_t b = 0;
    b += ws_round(sizeof(double) * (size_t)k * k) * 5;   // UL, Gram, V, Ginv, Z
    b += ws_round(sizeof(double) * k) + ws_round(sizeof(int) * k);
    b += gemm_tn_ws(d, k, k);
    b += ws_round(sizeof(double) * (size_t)kColBlocks * k);
    b += ws_round(sizeof(double) * k);
    b += jacobi_ws_bytes(k);
    return b;
}

extern "C" int otm_unwhiten_topics(const double* W, int32_t d, int32_t k, const float* Phi, double theta, double* mu,
                                   double* alpha_hat, double* lambda, int32_t* info, void* ws, size_t ws_bytes,
                                   otm_stream stream) {
    OTM_REQUIRE(W && Phi && mu && alpha_hat && lambda && info, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(d >= 1 && k >= 1 && k <= kMaxK && k <= d, OTM_ESHAPE, "need 1 <= k <= min(d, 128)");
    OTM_REQUIRE(std::isfinite(theta), OTM_EINVAL, "theta must be finite");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_unwhiten_workspace(d, k), OTM_EWORKSPACE,
                "unwhiten workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    double* UL = wc.take<double>((size_t)k * k);
    double* Gr = wc.take<double>((size_t)k * k);
    double* V = wc.take<double>((size_t)k * k);
    double* Gi = wc.take<double>((size_t)k * k);
    double* Z = wc.take<double>((size_t)k * k);
    double* ev = wc.take<double>(k);
    int* ord = wc.take<int>(k);
    double* part = wc.take<double>(gemm_tn_ws(d, k, k) / sizeof(double));
    double* cpart = wc.take<double>((size_t)kColBlocks * k);
    double* csum = wc.take<double>(k);
    void* jws = wc.take<char>(jacobi_ws_bytes(k));
    int st;
    hipLaunchKernelGGL(factor_stats_kernel, dim3(1), dim3(kMaxK), 0, s, Phi, k, 0.5 * (1.0 + theta), lambda, UL,
                       alpha_hat);
    if ((st = check_launch("factor_stats_kernel")) != OTM_OK) return st;
    if ((st = gemm_tn(W, k, W, k, d, k, k, Gr, part, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(symmetrize_kernel, dim3((k * k + 255) / 256), dim3(256), 0, s, Gr, k);
    if ((st = check_launch("symmetrize_kernel")) != OTM_OK) return st;
    if ((st = jacobi(Gr, V, k, ev, ord, jws, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(spd_inverse_kernel, dim3((k * k + 255) / 256), dim3(256), 0, s, V, ev, k, Gi, info);
    if ((st = check_launch("spd_inverse_kernel")) != OTM_OK) return st;
    if ((st = gemm_nn(Gi, k, UL, k, Z, k, k, k, k, s)) != OTM_OK) return st;
    if ((st = gemm_nn(W, k, Z, k, mu, k, d, k, k, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(clip_colsum_partial_kernel, dim3(kColBlocks), dim3(128), 0, s, mu, d, k, cpart);
    if ((st = check_launch("clip_colsum_partial_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3((k + 255) / 256), dim3(256), 0, s, cpart, kColBlocks, (int64_t)k, csum);
    if ((st = check_launch("reduce_parts_kernel")) != OTM_OK) return st;
    const int64_t total = (int64_t)d * k;
    hipLaunchKernelGGL(col_normalize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, mu, csum, d, k);
    return check_launch("col_normalize_kernel");
}
