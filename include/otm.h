/*
 * otm.h -- C ABI of the MI355X (gfx950) hot path of the online tensor method
 * for latent variable models (Huang, Niranjan, Hakeem, Anandkumar, "Online
 * Tensor Methods for Learning Latent Variable Models").
 *
 * Path: M2 operator -> randomized whitener -> whitening SpMM -> stochastic
 * tensor gradient descent (STGD) on the implicit whitened third moment ->
 * post-processing (topics / memberships).
 *
 * Conventions (every entry point):
 *  - Array arguments are DEVICE pointers owned by the caller, unless noted.
 *    The library never allocates device memory: scratch space comes from the
 *    caller through (ws, ws_bytes); query its size with the matching
 *    *_workspace function.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    the call returns after host-side validation; results are visible after
 *    the stream is synchronised.  Conditions that depend on device data (an
 *    indefinite moment, a non-finite update) are reported through device
 *    flags named in each entry point.
 *  - Return value: OTM_OK or a negative otm_status; otm_last_error() then
 *    holds a message (thread-local).  No exception crosses the ABI and the
 *    library never aborts the process.
 *  - Dense row-major layout.  A factor matrix Phi (k x k) stores phi_i, the
 *    i-th estimated eigenvector, contiguously at Phi + i*k.
 *  - Results do not depend on run-to-run scheduling: all reductions use a
 *    fixed order and no floating-point atomics.
 */
#ifndef OTM_H
#define OTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OTM_OK = 0,
    OTM_EINVAL = -1,      /* null pointer or invalid scalar argument */
    OTM_ESHAPE = -2,      /* inconsistent sizes */
    OTM_EDTYPE = -3,      /* unsupported element type for this entry point */
    OTM_ENOTPSD = -4,     /* projected second moment has no k positive eigenvalues */
    OTM_ENONFINITE = -5,  /* a non-finite value was produced */
    OTM_EHIP = -6,        /* HIP runtime error */
    OTM_EWORKSPACE = -7,  /* workspace missing or too small */
    OTM_ECAPACITY = -8    /* size beyond the compiled capacity (see otm_max_k) */
} otm_status;

typedef enum { OTM_F64 = 0, OTM_F32 = 1, OTM_BF16 = 2 } otm_dtype;

typedef void* otm_stream; /* hipStream_t */

/* Sparse observations in CSR form (Sections 2.1-2.2: word counts c_t of a
 * document, or the adjacency row G[x, A] of a node).  Device arrays:
 * rowptr (n_rows + 1), colidx (nnz, each < n_cols), vals (nnz; NULL means
 * every stored entry is 1).  Kernels skip entries whose column is out of
 * range and clamp row ranges to [0, nnz], so malformed input cannot make
 * them read out of bounds; otm_csr_check reports it. */
typedef struct {
    int32_t n_rows;
    int32_t n_cols;
    int64_t nnz;
    const int32_t* rowptr;
    const int32_t* colidx;
    const float* vals;
} otm_csr;

const char* otm_status_string(int status);
const char* otm_last_error(void);
int otm_version(void);
/* Largest k (number of components) the STGD kernels are compiled for. */
int otm_max_k(void);
/* Largest mini-batch of the STGD kernels. */
int otm_max_batch(void);

/* Validates a CSR on the device and synchronises `stream`: rowptr[0] == 0,
 * non-decreasing, rowptr[n_rows] == nnz, every colidx in [0, n_cols).
 * *bad_count receives the number of violations (0 = valid).  ws must hold
 * otm_csr_check_workspace() bytes. */
size_t otm_csr_check_workspace(void);
int otm_csr_check(const otm_csr* C, int64_t* bad_count, void* ws, size_t ws_bytes, otm_stream stream);

/* ---- a1: second-moment operator (Section 2, Eq. 2moment; Section 4.2) -----
 * O = M2 S for the n x d observations C, without forming M2:
 *   M2 = (alpha0+1)/n sum_t w2_t (c_t c_t^T - diag c_t) - alpha0 M1 M1^T,
 *   M1 = (1/n) sum_t w1_t c_t.
 * normalize != 0 (documents): w1_t = 1/l_t, w2_t = 1/(l_t (l_t - 1)) with l_t
 * the row sum (every row needs l_t >= 2, else *info = 1 and O is undefined);
 * normalize == 0 (graph rows): w1 = w2 = 1.
 * C: n x d; CT: its transpose (d x n) with the same entries.
 * S: d x k_tilde FP64 row-major (the random projection).  O: d x k_tilde FP64.
 * info: device int32, set to 0 on success.  FP64 throughout. */
size_t otm_m2_apply_workspace(int32_t n, int32_t d, int32_t k_tilde);
int otm_m2_apply(const otm_csr* C, const otm_csr* CT, int normalize, double alpha0,
                 const double* S, int32_t k_tilde, double* O, int32_t* info,
                 void* ws, size_t ws_bytes, otm_stream stream);

/* M2 applied to a column-selection projection with random signs (Section
 * 4.2: for a sparse M2 the projection S in {0, +-1}^(d x k_tilde) selects
 * k_tilde columns): S[r_j, j] = s_j, so
 *   O[:, j] = s_j M2[:, r_j]
 *           = s_j [(alpha0+1)/n (sum_t w2_t c_t[r_j] c_t - u[r_j] e_(r_j)) - alpha0 M1 M1[r_j]],
 * u = C^T w2, M1 and w1, w2 as in otm_m2_apply.  Only the samples with
 * c_t[r_j] != 0 (row r_j of CT) and their rows are read.  sel_rows: k_tilde
 * int32 rows in [0, d); sel_signs: k_tilde FP64 (+-1).  O: d x k_tilde FP64.
 * info: device int32, 0 on success, 1 as in otm_m2_apply, 2 when a selected
 * row lies outside [0, d) (that column is left 0).  Deterministic: each
 * column's sums run over the samples in their stored order. */
size_t otm_m2_apply_select_workspace(int32_t n, int32_t d);
int otm_m2_apply_select(const otm_csr* C, const otm_csr* CT, int normalize, double alpha0, const int32_t* sel_rows,
                        const double* sel_signs, int32_t k_tilde, double* O, int32_t* info, void* ws, size_t ws_bytes,
                        otm_stream stream);
/* The d x k_tilde FP64 matrix of a column selection (for otm_whitener's S). */
int otm_selection_dense(const int32_t* sel_rows, const double* sel_signs, int32_t d, int32_t k_tilde, double* S,
                        otm_stream stream);

/* ---- a2: randomized whitener (Section 3.1; Section 4.2, "Randomized
 * Tall-thin SVD" and its tall-thin QR variant) -----------------------------
 * From O = M2 S (d x k_tilde) and S (d x k_tilde), FP64:
 *   Omega = sym(S^T O) = U diag(sigma) U^T (sigma descending),
 *   B = O U_k diag(sigma_k)^(-1/2),   B = U_B diag(s) V_B^T,
 *   W = U_B diag(s)^(-1)     so that W^T (B B^T) W = I,
 * columns sign-fixed so that each column's largest-magnitude entry is
 * positive (ties: lowest row).  W: d x k FP64; evals: k FP64 (s^2, the top
 * eigenvalues of the low-rank M2).  W_lo: optional (may be NULL) copy of W in
 * w_lo_dtype (OTM_F32 or OTM_BF16, round-to-nearest-even) for otm_whiten,
 * d x ldw_lo row-major (ldw_lo >= k; columns k..ldw_lo-1 written with 0;
 * ignored when W_lo is NULL).  A row stride that is a multiple of 16 bytes
 * lets otm_whiten gather W rows as 16-byte vectors.
 * info: device int32, 0 on success, 1 if sigma_k <= 1e-12 sigma_1 or
 * sigma_k <= 0 (OTM_ENOTPSD condition; W undefined).  k <= k_tilde <= 256. */
size_t otm_whitener_workspace(int32_t d, int32_t k_tilde, int32_t k);
int otm_whitener(const double* O, const double* S, int32_t d, int32_t k_tilde, int32_t k,
                 double* W, double* evals, void* W_lo, int w_lo_dtype, int32_t ldw_lo,
                 int32_t* info, void* ws, size_t ws_bytes, otm_stream stream);

/* Orthonormal basis of the sketch for power iterations (READING of Section
 * 4.2 for sampled data: the projected moment S^T M2 S is indefinite at
 * k_tilde = 2k when M2's noise directions dominate the sketch, so the sketch
 * is refined by q steps Q <- orth(M2 Q) before the whitener, as in the power
 * method sketches of the cited Nystrom analysis; q = 0 is the paper's
 * algorithm).  Q (d x m FP64) is an orthonormal basis of span(Y): Cholesky
 * QR applied twice for m <= 200 (Q = Y R1^-1 R2^-1), else Y (Y^T Y)^(-1/2)
 * through a Jacobi eigensolver of the m x m Gram, also applied twice.  info: device int32, 0 on
 * success, 1 if Y is rank deficient (a pivot or eigenvalue <= 1e-14 of the
 * largest).  m <= min(d, 256); Y, Q must not alias. */
size_t otm_orthonormalize_workspace(int32_t d, int32_t m);
int otm_orthonormalize(const double* Y, int32_t d, int32_t m, double* Q, int32_t* info,
                       void* ws, size_t ws_bytes, otm_stream stream);

/* ---- four-partition graph moments (Section 2.2: transition matrices of
 * Eq. transitionMat, moments of Eqs. 1moment_graph / 2moment_graph; Section
 * 4.1: products in factored form; Section 4.2: algorithm "Randomized
 * Pseudoinverse") ----------------------------------------------------------
 * The nodes are split into the samples X and the leaf sets A, B, C;
 * Pairs(Y1, Y2) = (1/n_X) G[X, Y1]^T G[X, Y2].  The blocks of the adjacency
 * matrix the estimator reads, each a CSR with its transpose: */
typedef struct {
    otm_csr XA, XB, XC;   /* G[X, A], G[X, B], G[X, C]: n_X x n_A, n_X x n_B, n_X x n_C */
    otm_csr AX, BX, CX;   /* G[A, X], G[B, X], G[C, X]: the transposes, same entries */
} otm_partition;

/* out (n1 x m) = Pairs(Y1, Y2) V = (1/n_X) G1T (G2 V) for G1T = G[Y1, X]
 * (n1 x n_X), G2 = G[X, Y2] (n_X x n2) and V (n2 x m FP64 row-major),
 * 1 <= m <= 256.  ws: otm_pairs_apply_workspace(n_X, m) bytes. */
size_t otm_pairs_apply_workspace(int32_t n_x, int32_t m);
int otm_pairs_apply(const otm_csr* G1T, const otm_csr* G2, const double* V, int32_t m, double* out, void* ws,
                    size_t ws_bytes, otm_stream stream);

/* Rank-k randomized pseudo-inverse of P (n1 x n2) in factored form, from its
 * sketches J = P S_right (n1 x m) and K = P^T S_left (n2 x m), both FP64
 * row-major, and S_left (n1 x m).  The algorithm "Randomized Pseudoinverse"
 * of Section 4.2 is printed for a symmetric P and one sketch; it is taken here
 * from both sides (it reduces to the printed form when P is symmetric and
 * S_left = S_right):
 *   Psi = S_left^T J, its top-k singular triplets (U_k, s, V_k) from the
 *   eigenpairs of Psi^T Psi; J V_k = Q_J R_J and K U_k = Q_K R_K (Cholesky QR
 *   twice); core = R_K^-T diag(s) R_J^-1;  P^+ ~ Q_K core Q_J^T (n2 x n1).
 * Outputs QJ (n1 x k), QK (n2 x k), core (k x k), sv (k singular values of
 * Psi, descending; NULL allowed).  info: device int32, 0 on success, 1 when
 * s_k <= 1e-12 s_1 or a QR pivot vanishes (results then undefined).
 * 1 <= k <= m <= 256, k <= min(n1, n2, 200). */
size_t otm_pinv_factors_workspace(int32_t n1, int32_t n2, int32_t m, int32_t k);
int otm_pinv_factors(const double* J, const double* K, const double* S_left, int32_t n1, int32_t n2, int32_t m,
                     int32_t k, double* QJ, double* QK, double* core, double* sv, int32_t* info, void* ws,
                     size_t ws_bytes, otm_stream stream);

/* Y (n_out x m) = Q_out M (Q_in^T X), M = core (trans == 0) or core^T
 * (trans != 0): a low-rank factored product (Section 4.1).  Q_in: n_in x k,
 * Q_out: n_out x k, core: k x k, X: n_in x m, all FP64 row-major. */
size_t otm_factored_apply_workspace(int32_t n_in, int32_t k, int32_t m);
int otm_factored_apply(const double* Q_in, int32_t n_in, const double* core, int trans, const double* Q_out,
                       int32_t n_out, int32_t k, const double* X, int32_t m, double* Y, void* ws, size_t ws_bytes,
                       otm_stream stream);

/* Transposed transition products (Section 4.1: y_B = W^T Z_B G[x, B]^T,
 * y_C = W^T Z_C G[x, C]^T) with Z_B = Pairs(A, C) Pairs(B, C)^+ and
 * Z_C = Pairs(A, B) Pairs(C, B)^+, Pairs(B, C)^+ ~ QK core QJ^T from
 * otm_pinv_factors(J = Pairs(B, C) S_C, K = Pairs(C, B) S_B, S_left = S_B):
 *   view 1: out (n_B x m) = Z_B^T V = QJ core^T QK^T Pairs(C, A) V
 *   view 2: out (n_C x m) = Z_C^T V = QK core QJ^T Pairs(B, A) V
 * V: n_A x m FP64 (for W_B = Z_B^T W, W_C = Z_C^T W: V = W, m = k). */
size_t otm_transition_t_workspace(const otm_partition* G, int32_t k, int32_t m);
int otm_transition_t_apply(const otm_partition* G, const double* QJ, const double* QK, const double* core, int32_t k,
                           int view, const double* V, int32_t m, double* out, void* ws, size_t ws_bytes,
                           otm_stream stream);

/* O (n_A x m) = M2 S for the second moment of Eq. 2moment_graph, without
 * forming it:  M2 = (alpha0+1)/n_X sum_x Z_C G[x, C]^T G[x, B] Z_B^T
 * - alpha0 M1 M1^T,  M1 = (1/n_X) sum_x G[x, A]^T, applied right to left:
 * (alpha0+1) Z_C Pairs(C, B) (Z_B^T S) - alpha0 M1 (M1^T S).  S: n_A x m FP64. */
size_t otm_m2_apply_four_workspace(const otm_partition* G, int32_t k, int32_t m);
int otm_m2_apply_four(const otm_partition* G, const double* QJ, const double* QK, const double* core, int32_t k,
                      double alpha0, const double* S, int32_t m, double* O, void* ws, size_t ws_bytes,
                      otm_stream stream);

/* FP64 rows X (rows x cols, row stride ldx) to out (rows x ldo) in OTM_F32 or
 * OTM_BF16 (round to nearest even), columns cols..ldo-1 written with 0: the
 * low-precision copy the whitening SpMM gathers (W_B, W_C). */
int otm_cast_rows(const double* X, int32_t rows, int32_t cols, int32_t ldx, void* out, int dtype, int32_t ldo,
                  otm_stream stream);

/* ---- a3: whitening SpMM (Section 3.1 whitened data; Appendix A) ----------
 * Y[t, :] = r_t * sum_j C[t, j] W[j, :],  r_t = 1 / (row sum) if normalize
 * (document views) else 1.  W: n_cols x k in w_dtype (OTM_F32 or OTM_BF16),
 * row-major with row stride ldw >= k elements; the padding columns k..ldw-1
 * must be readable but do not change the result.  Rows are gathered as
 * 16-byte vectors when ldw is a multiple of 16 bytes and W is 16-byte aligned
 * (for instance ldw = k rounded up to 4 in FP32, to 8 in BF16), narrower ones
 * otherwise; k <= 64 * vector width.  Y: n_rows x ldy row-major in y_dtype (OTM_F32 or OTM_BF16,
 * round-to-nearest-even), FP32 accumulation; columns k..ldy-1 are written
 * with 0.  ldy >= k; ldy % 8 == 0 for OTM_BF16, ldy % 4 == 0 for OTM_F32.
 * ybar: optional (NULL allowed) k floats, the mean of Y's rows computed from
 * the FP32 accumulators (Appendix A: ybar = E_t[y_t]), fixed-order sum.
 * A row with sum 0 under normalize gives a zero row. */
size_t otm_whiten_workspace(int32_t n_rows, int32_t k);
int otm_whiten(const otm_csr* C, int normalize, const void* W, int w_dtype, int32_t k, int32_t ldw,
               void* Y, int y_dtype, int32_t ldy, float* ybar,
               void* ws, size_t ws_bytes, otm_stream stream);

/* The whitening SpMM of otm_whiten for callers that cannot allocate (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results (Y and ybar bit-identical to otm_whiten's),
 * with the per-block partial column sums in a library-owned device array of
 * otm_whiten_noalloc_capacity() floats (4 MiB, one copy per device, held until
 * the process ends) instead of a caller workspace.  The call allocates
 * nothing and takes no workspace; it returns OTM_EWORKSPACE when the partial
 * sums (up to 8192 blocks x k) exceed the array, which never happens for
 * k <= 128.  The first call on a device resolves the array's address there
 * (make that call outside a graph capture).  All calls on one device share
 * the array: calls that overlap on one device (several streams or host
 * threads at once) race and give wrong ybar. */
size_t otm_whiten_noalloc_capacity(void);
int otm_whiten_noalloc(const otm_csr* C, int normalize, const void* W, int w_dtype, int32_t k, int32_t ldw,
                       void* Y, int y_dtype, int32_t ldy, float* ybar, otm_stream stream);

/* ---- a4 / a5: stochastic tensor gradient descent (Section 3.2, Lemma
 * "update"; stacked form of Section 4.3) -----------------------------------
 * For a batch of rows t with whitened views yA_t, yB_t, yC_t (rows of YA,
 * YB, YC; n x ldy row-major, y_dtype OTM_F32 or OTM_BF16; the three may alias)
 * and global means ybar (3 x k FP32: ybar_A, ybar_B, ybar_C), every phi_i
 * moves by beta * Delta_i where Delta_i is the batch mean of
 *   -kappa sum_j <phi_j,phi_i>^2 phi_j
 *   + a <phi_i,yA><phi_i,yB> yC + c <phi_i,ybarA><phi_i,ybarB> ybarC
 *   - b (<phi_i,yA><phi_i,yB> ybarC + <phi_i,yA><phi_i,ybarB> yC
 *        + <phi_i,ybarA><phi_i,yB> yC),
 * a = (alpha0+1)(alpha0+2)/2, b = alpha0(alpha0+1)/2, c = alpha0^2,
 * kappa = (1+theta)/2.  All k components update from the same old Phi.
 * Contractions run on the matrix cores: FP32 inputs in FP32, BF16 inputs in
 * BF16 with FP32 accumulation; the FP32 master copy of Phi is updated with
 * compensated (Kahan) summation when compensated != 0.
 * Capacity: k <= otm_max_k(), batch <= otm_max_batch(). */
typedef struct {
    int32_t k;          /* components */
    int32_t batch;      /* mini-batch size B */
    int32_t passes;     /* passes over the data (rows of perms) */
    int32_t ldy;        /* row stride of YA/YB/YC in elements */
    int32_t y_dtype;    /* OTM_F32 or OTM_BF16 */
    int32_t compensated;
    double alpha0;
    double theta;       /* orthogonality weight, 1 in the paper's experiments */
    double beta0;       /* beta_t = beta0 / (1 + t / beta_tau), t the global step */
    double beta_tau;
} otm_sgd_params;

/* One step on the first `rows` rows of YA/YB/YC (1 <= rows <= batch) with
 * rate beta.  Phi (k x k FP32) is updated in place; Phi_comp: NULL or the
 * k x k compensation terms, read and written. */
int otm_sgd_step(const otm_sgd_params* p, int32_t rows, const void* YA, const void* YB,
                 const void* YC, const float* ybar, double beta, float* Phi, float* Phi_comp,
                 otm_stream stream);

/* Global steps [start_step, end_step) of an online run over n rows:
 * step t is pass t / S, batch t % S, S = ceil(n / batch); pass p visits rows
 * perms[p*n + 0 .. n-1] (perms: passes x n int32, a permutation of 0..n-1 per
 * pass; NULL visits rows in order), the last batch of a pass holding the
 * remaining n - (S-1)*batch rows.  end_step < 0 means passes * S.
 * `restarts` independent runs execute concurrently, one per workgroup: run r
 * uses Phi + r*k*k, Phi_comp + r*k*k (if not NULL), perms + r*perm_stride and
 * writes snapshots + r*passes*k*k.  snapshots: NULL or restarts x passes x
 * k x k, Phi after the last step of each pass.  nonfinite: NULL or a device
 * int32 that is set to 1 (never cleared) if an update is not finite or a
 * permutation entry lies outside [0, n) (that entry then reads row 0). */
int otm_sgd_run(const otm_sgd_params* p, int32_t n, const void* YA, const void* YB,
                const void* YC, const float* ybar, const int32_t* perms, int64_t perm_stride,
                int32_t restarts, int64_t start_step, int64_t end_step, float* Phi,
                float* Phi_comp, float* snapshots, int32_t* nonfinite, otm_stream stream);

/* ---- restart score (Section 3.2 objective; selection among restarts) -----
 * score_r = sum_ij (phi_i^T phi_j)^3 - 2 sum_i T(phi_i, phi_i, phi_i)
 *         = ||sum_i phi_i^(x3) - T||_F^2 - ||T||_F^2
 * for each of `restarts` factor matrices Phi + r*k*k (k x k FP32, phi_i
 * contiguous), with T the whitened, Dirichlet-corrected tensor of the n rows
 * of YA/YB/YC (the tensor the update of Lemma "update" descends on, with the
 * global means ybar).  The lowest score is the lowest residual.  One pass over
 * the rows, the same contractions as a step, no update; FP32 products summed
 * in FP64 across batches.  y_dtype must be OTM_F32; p->passes is ignored.
 * score: restarts FP64 (device).  ws: otm_sgd_score_workspace(restarts). */
size_t otm_sgd_score_workspace(int32_t restarts);
int otm_sgd_score(const otm_sgd_params* p, int32_t n, const void* YA, const void* YB, const void* YC,
                  const float* ybar, const float* Phi, int32_t restarts, double* score,
                  void* ws, size_t ws_bytes, otm_stream stream);

/* ---- batched STGD: many decompositions with restarts in one persistent
 * launch (the per-problem computation is otm_sgd_run with a scoring pass) ---
 * A problem is one decomposition: whitened views of n rows, k components,
 * `restarts` runs from the initial factors Phi0 + r*k*k, results Phi + r*k*k,
 * scores score[r] as in otm_sgd_score of the final factors.  perms: NULL
 * (rows in order) or, per run r, passes x n int32 at perms + r*perm_stride
 * (perm_stride 0: every run of the problem visits the rows in the same order).
 * Every pointer is device memory owned by the caller. */
typedef struct {
    const void* YA;
    const void* YB;
    const void* YC;
    const float* ybar;        /* 3 x k */
    const int32_t* perms;
    int64_t perm_stride;
    const float* Phi0;        /* restarts x k x k, read only */
    float* Phi;               /* restarts x k x k, written */
    double* score;            /* restarts, written */
    int32_t n, k, ldy;
    int32_t pad_;
    double alpha0;
} otm_problem;

/* Host-only planning (no GPU call): one job per (problem, restart).  Each
 * job's kernel variant (padded k, tile layout, view staging) comes from the
 * tuning cache file (NULL or a missing entry: the default layout); jobs are
 * grouped by variant, longest first inside a group (estimated from the steps
 * and the tuned cost per step).  The shared settings (batch, passes,
 * y_dtype = OTM_F32, compensated, theta, beta0, beta_tau) come from p; p->k,
 * p->ldy and p->alpha0 are ignored.  best: device int32 per problem, the
 * lowest-score restart (ties to the lower index), written by the run.
 * nonfinite: NULL or device int32, cleared at the start of each run and set
 * as in otm_sgd_run.  *plan receives a host object (free it with
 * otm_plan_free); its device image (otm_plan_image, otm_plan_size bytes) is
 * plain data that the caller copies to device memory for the runs. */
typedef struct otm_plan_s* otm_plan;
int otm_sgd_batched_plan(const otm_problem* problems, int32_t n_problems, int32_t restarts,
                         const otm_sgd_params* p, const char* tune_cache, int32_t* best,
                         int32_t* nonfinite, otm_plan* plan);
size_t otm_plan_size(otm_plan plan);
const void* otm_plan_image(otm_plan plan);
int32_t otm_plan_groups(otm_plan plan);   /* kernel variants the plan uses */
/* Variant of group g (in launch order): padded k, tile layout (0 or 1), views
 * (1 = one aliased view, 3 = three views) and its number of jobs. */
int otm_plan_group_info(otm_plan plan, int32_t group, int32_t* kp, int32_t* layout, int32_t* views,
                        int32_t* jobs);
int otm_plan_free(otm_plan plan);

/* Runs a plan whose image is at `image` (device memory): a kernel clears the
 * queue counters and the nonfinite flag; one persistent kernel per variant
 * group runs on library-owned branch streams forked from `stream` (all
 * concurrent; each group's workgroups, sized by its share of the estimated
 * work, pull jobs until the group's queue is empty); the branches join back
 * into `stream`, and a last kernel writes best.  The image must stay
 * unchanged while the run is in flight.  ws: otm_sgd_batched_workspace(plan)
 * bytes.  No device allocation, no memset node: the call can be captured into
 * a graph (otm_sgd_batched_graph).  Runs on one device must not be issued
 * from several host threads at once (they share the branch streams). */
size_t otm_sgd_batched_workspace(otm_plan plan);
int otm_sgd_batched(otm_plan plan, const void* image, void* ws, size_t ws_bytes, otm_stream stream);

/* The same launch sequence captured into a graph on `stream` (not the null
 * stream) and instantiated; replays compute the same results (every output
 * is overwritten, Phi0 is only read).  otm_graph_launch replays it on a
 * stream; otm_graph_destroy frees it. */
typedef struct otm_graph_s* otm_graph;
int otm_sgd_batched_graph(otm_plan plan, const void* image, void* ws, size_t ws_bytes, otm_stream stream,
                          otm_graph* graph);
int otm_graph_launch(otm_graph graph, otm_stream stream);
int otm_graph_destroy(otm_graph graph);

/* Tile-layout autotuner for the batched kernel: for each padded k of ks and
 * each view layout (one aliased view, three views) it times the kernel
 * variants on a full device of synthetic probe jobs (batch rows of random
 * whitened data, one pass), and records the fastest in the text file
 * cache_path (merged with its existing entries).  Allocates and frees its own
 * probe buffers (setup time, not for capture); synchronises the stream. */
int otm_sgd_autotune(const int32_t* ks, int32_t n_k, int32_t batch, const char* cache_path, otm_stream stream);

/* ---- learned warm start of the stochastic updates (an addition: the paper
 * starts them at random, Section 3.2) ----------------------------------------
 * Sizes: P = 100 (largest k the network takes), 4 sketches, n_in = 4 P^2 +
 * 4 P, hidden 512, n_out = P^2; the parameters are one flat FP32 buffer
 * [W1 (hidden x n_in), b1 (hidden), W2 (n_out x hidden), b2 (n_out)],
 * row-major. */
int otm_ws_dims(int32_t* n_in, int32_t* n_hidden, int32_t* n_out, int32_t* p, int64_t* n_params);

/* Sketch of the whitened third moment: S_r = T(I, I, theta_r), r = 0..3, the
 * tensor T of Lemma "update" (global means ybar, coefficients of alpha0)
 * contracted along its third (view C) mode, from the rows without forming T:
 *   S_r = (1/n) YA^T diag(a z_r - b (ybarC . theta_r)) YB - b ybarA (YB^T z_r / n)^T
 *         - b (YA^T z_r / n) ybarB^T + c (ybarC . theta_r) ybarA ybarB^T,  z_r = YC theta_r.
 * Rows n x ldy in y_dtype (F32 or BF16); ybar 3 x k FP32; Theta k x 4 FP32
 * row-major; S: 4 blocks of lds x lds FP32 (S_r[i][j] at S + (r*lds + i)*lds
 * + j; entries outside the k x k block untouched).  FP64 sums, FP32 output. */
size_t otm_ws_sketch_workspace(int32_t n, int32_t k);
int otm_ws_sketch(const void* YA, const void* YB, const void* YC, int y_dtype, int32_t ldy, int32_t n, int32_t k,
                  const float* ybar, double alpha0, const float* Theta, float* S, int32_t lds, void* ws,
                  size_t ws_bytes, otm_stream stream);

/* Canonical frames and network inputs for `count` instances (one workgroup
 * each): ks[i] (device int32, 1 <= k <= P); S: count x 4 x P x P sketches
 * (live k x k blocks); Theta: count x P x 4.  Q (count x P x P): the
 * eigenvectors of sym(S_0) as columns (FP32 Jacobi), by decreasing
 * |eigenvalue| (ties: lower index), each oriented so that its contraction with
 * the theta_r of largest |q . theta_r| has the sign of q^T S_r q; zero
 * outside k x k.  sigma: sqrt(mean_r ||S_r||_F^2).  X (count x n_in):
 * [Q^T S_r Q / sigma padded to P x P for r = 0..3, Q^T theta_r padded to P].
 * info[i]: Jacobi sweeps used, -1 if not converged in 15, -2 if k is out of
 * range (then X = 0, Q = I).  ws: otm_ws_frames_workspace(count). */
size_t otm_ws_frames_workspace(int32_t count);
int otm_ws_frames(int32_t count, const int32_t* ks, const float* S, const float* Theta, float* Q, float* sigma,
                  float* X, int32_t* info, void* ws, size_t ws_bytes, otm_stream stream);

/* Training targets: with the planted directions U (count x P x P, column j =
 * u_j) and lambda (count x P), C = Q^T U, perm = greedy matching by
 * decreasing |C| (ties: lower row, then lower column), target (count x P^2,
 * row-major P x P) column l = lambda_perm[l]^(1/3) C[:, perm[l]] / sigma^(1/3). */
int otm_ws_target(int32_t count, const int32_t* ks, const float* Q, const float* sigma, const float* U,
                  const float* lam, float* target, otm_stream stream);

/* Perceptron on the matrix cores.  Forward (FP32): H = relu(X W1^T + b1)
 * (batch x hidden), out = H W2^T + b2 (batch x n_out).  Backward from dout:
 * grads (flat, as the parameters) of W2, b2, W1, b1.  Adam (Kingma and Ba,
 * Algorithm 1) over the flat buffers, step t >= 1.  BF16 inference: weights
 * converted once (otm_mlp_to_bf16), inputs and the hidden layer rounded to
 * BF16, FP32 accumulation and FP32 biases (the FP32 parameter buffer). */
size_t otm_mlp_workspace(int32_t batch);
int otm_mlp_forward(const float* params, int32_t batch, const float* X, float* H, float* out, void* ws,
                    size_t ws_bytes, otm_stream stream);
int otm_mlp_backward(const float* params, int32_t batch, const float* X, const float* H, const float* dout,
                     float* grads, void* ws, size_t ws_bytes, otm_stream stream);
int otm_mlp_adam(float* params, const float* grads, float* m, float* v, int32_t t, double lr, double beta1,
                 double beta2, double eps, otm_stream stream);
int otm_mlp_to_bf16(const float* params, void* params_bf16, otm_stream stream);
size_t otm_mlp_bf16_workspace(int32_t batch);
int otm_mlp_forward_bf16(const void* params_bf16, const float* params, int32_t batch, const float* X, float* out,
                         void* ws, size_t ws_bytes, otm_stream stream);

/* Squared error over the live k x k blocks: *loss (device FP64) = sum / live,
 * dout = 2 (out - target) / live inside the blocks, 0 outside; live = sum of
 * k_i^2.  ws: otm_ws_mse_workspace(count). */
size_t otm_ws_mse_workspace(int32_t count);
int otm_ws_mse(int32_t count, const int32_t* ks, int64_t live, const float* out, const float* target, double* loss,
               float* dout, void* ws, size_t ws_bytes, otm_stream stream);

/* Initial factors V0 = Q out[:k, :k] sigma^(1/3): instance i writes phi_j
 * (length k, contiguous) at Phi + i*P*P + j*k. */
int otm_ws_factors(int32_t count, const int32_t* ks, const float* out, const float* Q, const float* sigma,
                   float* Phi, otm_stream stream);

/* ---- a6: post-processing (Section 3.3, Lemma "postprocessing") -----------
 * lambda_i = kappa ||phi_i||^3, u_i = phi_i / ||phi_i||,
 * mu_i = lambda_i (W^T)^+ u_i with (W^T)^+ = W (W^T W)^(-1), negatives
 * clipped to 0, columns normalised to sum 1 (a zero column stays 0);
 * alpha_hat_i = lambda_i^(-2) / sum_j lambda_j^(-2).
 * W: d x k FP64; Phi: k x k FP32; mu: d x k FP64 row-major; alpha_hat, lambda:
 * k FP64.  info: device int32, 0 on success, 1 if W^T W is not positive
 * definite.  FP64 throughout. */
size_t otm_unwhiten_workspace(int32_t d, int32_t k);
int otm_unwhiten_topics(const double* W, int32_t d, int32_t k, const float* Phi, double theta,
                        double* mu, double* alpha_hat, double* lambda, int32_t* info,
                        void* ws, size_t ws_bytes, otm_stream stream);

/* Memberships of the n samples (Lemma postprocessing with unit eigenvectors):
 * Pi[:, x] = diag(lambda)^(-1) U^T y_x, then negatives clipped to 0, column
 * normalised to sum 1, entries < tau set to 0, normalised again (a column
 * summing to 0 stays 0).  Y: n x ldy in y_dtype (OTM_F32 or OTM_BF16);
 * Phi: k x k FP32; Pi: k x n FP32 row-major.  FP64 arithmetic. */
size_t otm_recover_pi_workspace(int32_t k);
int otm_recover_pi(const void* Y, int y_dtype, int32_t ldy, int32_t n, int32_t k,
                   const float* Phi, double theta, double tau, float* Pi,
                   void* ws, size_t ws_bytes, otm_stream stream);

/* ---- validation against ground truth (Section 5.1, p-value testing;
 * Section 5.2, evaluation metrics) ------------------------------------------
 * Pi_hat: k_hat x n estimated memberships (rows = communities, FP32), Pi:
 * k x n true memberships of the same n nodes (FP32).  FP64 arithmetic:
 *   rho (k_hat x k): Pearson correlation of row i of Pi_hat with row j of Pi
 *     (0 when either row is constant);
 *   pval: right p-value P(t_(n-2) > T), T = rho sqrt(n-2) / sqrt(1-rho^2)
 *     (READING: the printed 1 - P(t > T) contradicts the stated right tail);
 *   padj: Benjamini-Hochberg adjusted p-values over all k_hat * k tests
 *     (READING of the false-discovery-rate adjustment), ties by position;
 *   edges (int32 0/1): padj <= threshold (the paper uses 0.01);
 *   l1: (1/n) sum_x |Pi_hat_i(x) - Pi_j(x)|;
 *   scores[0] = recovery ratio R = (1/k) #{j with an edge},
 *   scores[1] = error E = (1/k) sum over the edges of l1.
 * k_hat * k <= 16384, n >= 3.  Fixed-order sums; deterministic. */
size_t otm_validate_workspace(int32_t k_hat, int32_t k, int32_t n);
int otm_validate(const float* Pi_hat, int32_t k_hat, const float* Pi, int32_t k, int32_t n, double threshold,
                 double* rho, double* pval, double* padj, int32_t* edges, double* l1, double* scores, void* ws,
                 size_t ws_bytes, otm_stream stream);

/* Bridgeness of every node (Eq. bridgeness):
 * b_x = 1 - sqrt(k_hat/(k_hat-1) sum_j (Pi_hat_j(x) - 1/k_hat)^2), k_hat >= 2;
 * with the graph G (one row per node, NULL allowed) also the degree-corrected
 * b_degree_x = D_x b_x (Eq. degreebridgeness), D_x the row's sum of values
 * (its degree).  b, b_degree: n FP64 (b_degree NULL allowed; needs G). */
int otm_bridgeness(const float* Pi_hat, int32_t k_hat, int32_t n, const otm_csr* G, double* b, double* b_degree,
                   otm_stream stream);

/* ---- loss (measurement only; the hot path never forms the tensor) --------
 * T (k x k x k FP64, T[(a*k + b)*k + c]) = the whitened tensor of Section
 * 3.2:  a/n sum_t yA x yB x yC - b/n sum_t (yA x yB x ybarC + yA x ybarB x yC
 * + ybarA x yB x yC) + c ybarA x ybarB x ybarC, over all n rows. */
int otm_tensor_form(const void* YA, const void* YB, const void* YC, int y_dtype, int32_t ldy,
                    int32_t n, int32_t k, const float* ybar, double alpha0, double* T,
                    otm_stream stream);
/* R[j] = ||sum_i phi_i^(x3) - T||_F^2 / ||T||_F^2 for `count` factor
 * matrices Phi + j*k*k (FP32), FP64 arithmetic.  R: count doubles. */
size_t otm_residual_workspace(int32_t k, int32_t count);
int otm_residual(const double* T, int32_t k, const float* Phi, int32_t count, double* R,
                 void* ws, size_t ws_bytes, otm_stream stream);

/* ---- measurement probes: the device's own rates, beside the datasheet
 * figures the roofline fractions use ------------------------------------------
 * otm_probe_copy: dst = src over `bytes` (a positive multiple of 16, both
 * 16-byte aligned, not overlapping) with 16-byte vectors on `blocks`
 * workgroups of 256 threads, grid-stride: HBM bandwidth = 2 bytes / time.
 * otm_probe_mfma: every wave of `blocks` workgroups (four waves each) runs
 * `iters` rounds of eight independent matrix-core chains of dtype OTM_BF16
 * (16x16x32), OTM_F32 or OTM_F64 (16x16x4); out: blocks x 256 floats (sums that
 * keep the work alive).  otm_probe_mfma_flops gives the flops of such a launch. */
int otm_probe_copy(const void* src, void* dst, int64_t bytes, int32_t blocks, otm_stream stream);
int64_t otm_probe_mfma_flops(int dtype, int64_t iters, int32_t blocks);
int otm_probe_mfma(int dtype, int64_t iters, int32_t blocks, float* out, otm_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* OTM_H */
