// Four-partition graph moments (Section 2.2, Eq. transitionMat and Eqs.
// 1moment_graph / 2moment_graph; Section 4.1, the factored products; Section
// 4.2, algorithm "Randomized Pseudoinverse").  FP64 throughout.
//
//  * pairs_apply: Pairs(Y1, Y2) V = (1/n_X) G[X, Y1]^T (G[X, Y2] V), two
//    sparse passes (the second over the transposed block).
//  * pinv_factors: the rank-k pseudo-inverse of P from its sketches
//    J = P S_right, K = P^T S_left: Psi = S_left^T J, its top-k singular
//    triplets from the eigenpairs of Psi^T Psi, J' = J V_k = Q_J R_J,
//    K' = K U_k = Q_K R_K (Cholesky QR twice), Core = R_K^-T diag(s) R_J^-1,
//    so that P^+ ~ Q_K Core Q_J^T (n2 x n1).
//  * factored_apply: Q_out M (Q_in^T X) with M = Core or Core^T.
//  * transition_t_apply: Z_B^T V = Q_J Core^T Q_K^T Pairs(C, A) V and
//    Z_C^T V = Q_K Core Q_J^T Pairs(B, A) V (the matrices that whiten views B
//    and C), with Z_B = Pairs(A, C) Pairs(B, C)^+, Z_C = Pairs(A, B) Pairs(C, B)^+.
//  * m2_apply_four: O = (alpha0+1) Z_C Pairs(C, B) (Z_B^T S) - alpha0 M1 (M1^T S).
#include <cmath>

#include "otm_internal.h"

namespace otm {
namespace {

constexpr int kMaxM = 256;    // sketch columns of the FP64 sparse passes
constexpr int kMaxRank = 200; // Cholesky QR bound

// Top-k singular triplets of Psi (m x m) from the eigenpairs of Psi^T Psi:
// Vk[:, j] = v_j, VkS[:, j] = v_j / s_j (so Psi VkS = U_k), sk[j] = s_j.
// info = 1 when s_k <= 1e-12 s_1 (no rank-k part to invert).
__global__ void svd_topk_kernel(const double* __restrict__ V, const double* __restrict__ ev,
                                const int* __restrict__ order, int m, int k, double* __restrict__ Vk,
                                double* __restrict__ VkS, double* __restrict__ sk, int32_t* info) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const double s1 = sqrt(fmax(ev[order[0]], 0.0));
    const double sK = sqrt(fmax(ev[order[k - 1]], 0.0));
    const bool ok = sK > 1e-12 * s1 && sK > 0.0;
    if (e == 0) *info = ok ? 0 : 1;
    if (e >= m * k) return;
    const int row = e / k, j = e % k;
    const int col = order[j];
    const double sj = sqrt(fmax(ev[col], 0.0));
    const double v = V[(size_t)row * m + col];
    Vk[e] = v;
    VkS[e] = ok ? v / sj : 0.0;
    if (row == 0) sk[j] = sj;
}

// Core (k x k) = RKinv^T diag(s) RJinv; info |= the QR passes' status words
__global__ void pinv_core_kernel(const double* __restrict__ RKinv, const double* __restrict__ s,
                                 const double* __restrict__ RJinv, int k, const int32_t* __restrict__ qinfo,
                                 double* __restrict__ core, int32_t* info) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && (qinfo[0] | qinfo[1])) *info = 1;
    if (e >= k * k) return;
    const int i = e / k, j = e % k;
    double acc = 0.0;
    for (int l = 0; l < k; ++l) acc += RKinv[(size_t)l * k + i] * s[l] * RJinv[(size_t)l * k + j];
    core[e] = acc;
}

// T2 (k x m) = M T1 with M = core (trans = 0) or core^T (trans = 1)
__global__ void small_mm_kernel(const double* __restrict__ core, int trans, const double* __restrict__ T1, int k,
                                int m, double* __restrict__ T2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * m) return;
    const int i = e / m, c = e % m;
    double acc = 0.0;
    for (int l = 0; l < k; ++l) {
        const double a = trans ? core[(size_t)l * k + i] : core[(size_t)i * k + l];
        acc += a * T1[(size_t)l * m + c];
    }
    T2[e] = acc;
}

// out[r] = scale * (sum of the stored values of row r), one wave per row
__global__ void row_sum_kernel(otm_csr C, double scale, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int row = wave; row < C.n_rows; row += nwaves) {
        int64_t b = C.rowptr[row], e = C.rowptr[row + 1];
        b = b < 0 ? 0 : (b > C.nnz ? C.nnz : b);
        e = e < b ? b : (e > C.nnz ? C.nnz : e);
        double acc = 0.0;
        for (int64_t p = b + lane; p < e; p += 64) {
            const int32_t c = C.colidx[p];
            if (c < 0 || c >= C.n_cols) continue;
            acc += C.vals ? static_cast<double>(C.vals[p]) : 1.0;
        }
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) out[row] = scale * acc;
    }
}

// O = a Z - b M1 v^T  (d x m)
__global__ void rank1_epilogue_kernel(const double* __restrict__ Z, const double* __restrict__ M1,
                                      const double* __restrict__ v, int64_t d, int m, double a, double b,
                                      double* __restrict__ O) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * m) return;
    const int64_t r = e / m;
    const int c = static_cast<int>(e % m);
    O[e] = a * Z[e] - b * M1[r] * v[c];
}

// FP64 rows to FP32 or BF16 (round to nearest even), columns cols..ldo-1 zero
__global__ void cast_rows_kernel(const double* __restrict__ X, int64_t rows, int cols, int ldx, void* __restrict__ out,
                                 int dtype, int ldo) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * ldo) return;
    const int64_t r = e / ldo;
    const int c = static_cast<int>(e % ldo);
    const double v = c < cols ? X[r * ldx + c] : 0.0;
    if (dtype == OTM_F32)
        static_cast<float*>(out)[e] = static_cast<float>(v);
    else
        static_cast<__bf16*>(out)[e] = f32_to_bf16(static_cast<float>(v));
}

unsigned grid_for(int64_t n, int threads = 256) { return static_cast<unsigned>((n + threads - 1) / threads); }

// --------------------------------------------------------------- building blocks
size_t pairs_ws(int n_x, int m) { return ws_round(sizeof(double) * (size_t)n_x * m); }

int pairs_apply_impl(const otm_csr& G1T, const otm_csr& G2, const double* V, int m, double* out, double* tmp,
                     hipStream_t s) {
    int st = spmm64(G2, V, m, 1.0, tmp, s);
    if (st != OTM_OK) return st;
    return spmm64(G1T, tmp, m, 1.0 / G2.n_rows, out, s);
}

size_t factored_ws(int n_in, int k, int m) {
    return ws_round(sizeof(double) * (size_t)k * m) * 2 + gemm_tn_f64_ws(n_in, k, m);
}

int factored_apply_impl(const double* Qin, int n_in, const double* core, int trans, const double* Qout, int n_out,
                        int k, const double* X, int m, double* Y, void* ws, hipStream_t s) {
    WsCarver wc(ws, factored_ws(n_in, k, m));
    double* T1 = wc.take<double>((size_t)k * m);
    double* T2 = wc.take<double>((size_t)k * m);
    double* part = wc.take<double>(gemm_tn_f64_ws(n_in, k, m) / sizeof(double));
    int st = gemm_tn_f64(Qin, k, X, m, n_in, k, m, T1, part, s);
    if (st != OTM_OK) return st;
    hipLaunchKernelGGL(small_mm_kernel, dim3(grid_for((int64_t)k * m)), dim3(256), 0, s, core, trans, T1, k, m, T2);
    if ((st = check_launch("small_mm_kernel")) != OTM_OK) return st;
    return gemm_nn_f64(Qout, k, T2, m, Y, m, n_out, k, m, s);
}

int check_partition(const otm_partition* G) {
    OTM_REQUIRE(G != nullptr, OTM_EINVAL, "partition must not be NULL");
    const otm_csr* all[6] = {&G->XA, &G->XB, &G->XC, &G->AX, &G->BX, &G->CX};
    const char* names[6] = {"XA", "XB", "XC", "AX", "BX", "CX"};
    for (int i = 0; i < 6; ++i) {
        int st = validate_csr_header(all[i], names[i]);
        if (st != OTM_OK) return st;
    }
    const int nx = G->XA.n_rows;
    OTM_REQUIRE(nx >= 1 && G->XB.n_rows == nx && G->XC.n_rows == nx, OTM_ESHAPE,
                "XA, XB, XC must have the same n_X >= 1 rows");
    OTM_REQUIRE(G->AX.n_rows == G->XA.n_cols && G->AX.n_cols == nx && G->AX.nnz == G->XA.nnz, OTM_ESHAPE,
                "AX must be the transpose of XA");
    OTM_REQUIRE(G->BX.n_rows == G->XB.n_cols && G->BX.n_cols == nx && G->BX.nnz == G->XB.nnz, OTM_ESHAPE,
                "BX must be the transpose of XB");
    OTM_REQUIRE(G->CX.n_rows == G->XC.n_cols && G->CX.n_cols == nx && G->CX.nnz == G->XC.nnz, OTM_ESHAPE,
                "CX must be the transpose of XC");
    return OTM_OK;
}

size_t transition_ws(const otm_partition* G, int k, int m) {
    const int nx = G->XA.n_rows, nB = G->XB.n_cols, nC = G->XC.n_cols;
    const int nmax = nB > nC ? nB : nC;
    size_t f = factored_ws(nB, k, m);
    if (factored_ws(nC, k, m) > f) f = factored_ws(nC, k, m);
    return pairs_ws(nx, m) + ws_round(sizeof(double) * (size_t)nmax * m) + f;
}

// out = Z_B^T V (view 1, n_B x m) or Z_C^T V (view 2, n_C x m), V: n_A x m
int transition_t_impl(const otm_partition* G, const double* QJ, const double* QK, const double* core, int k, int view,
                      const double* V, int m, double* out, void* ws, hipStream_t s) {
    WsCarver wc(ws, transition_ws(G, k, m));
    const int nx = G->XA.n_rows, nB = G->XB.n_cols, nC = G->XC.n_cols;
    double* tmp = wc.take<double>((size_t)nx * m);
    double* X = wc.take<double>((size_t)(nB > nC ? nB : nC) * m);
    void* fws = wc.take<char>(factored_ws(nB > nC ? nB : nC, k, m));
    int st;
    if (view == 1) {   // Pairs(C, A) V = (1/n_X) G[C, X] (G[X, A] V), then Q_J Core^T Q_K^T
        if ((st = pairs_apply_impl(G->CX, G->XA, V, m, X, tmp, s)) != OTM_OK) return st;
        return factored_apply_impl(QK, nC, core, 1, QJ, nB, k, X, m, out, fws, s);
    }
    if ((st = pairs_apply_impl(G->BX, G->XA, V, m, X, tmp, s)) != OTM_OK) return st;   // Pairs(B, A) V
    return factored_apply_impl(QJ, nB, core, 0, QK, nC, k, X, m, out, fws, s);
}

}  // namespace
}  // namespace otm

using namespace otm;

extern "C" size_t otm_pairs_apply_workspace(int32_t n_x, int32_t m) {
    if (n_x < 1 || m < 1) return 0;
    return pairs_ws(n_x, m);
}

extern "C" int otm_pairs_apply(const otm_csr* G1T, const otm_csr* G2, const double* V, int32_t m, double* out, void* ws,
                               size_t ws_bytes, otm_stream stream) {
    int st = validate_csr_header(G1T, "G1T");
    if (st != OTM_OK) return st;
    if ((st = validate_csr_header(G2, "G2")) != OTM_OK) return st;
    OTM_REQUIRE(V && out, OTM_EINVAL, "V and out must not be NULL");
    OTM_REQUIRE(G2->n_rows >= 1 && G1T->n_cols == G2->n_rows, OTM_ESHAPE,
                "G1T (n1 x n_X) and G2 (n_X x n2) must share n_X >= 1 samples");
    OTM_REQUIRE(m >= 1 && m <= kMaxM, OTM_ECAPACITY, "need 1 <= m <= 256");
    OTM_REQUIRE(ws && ws_bytes >= otm_pairs_apply_workspace(G2->n_rows, m), OTM_EWORKSPACE,
                "pairs_apply workspace too small");
    return pairs_apply_impl(*G1T, *G2, V, m, out, static_cast<double*>(ws), as_stream(stream));
}

extern "C" size_t otm_pinv_factors_workspace(int32_t n1, int32_t n2, int32_t m, int32_t k) {
    if (n1 < 1 || n2 < 1 || m < 1 || k < 1) return 0;
    size_t b = 0;
    b += ws_round(sizeof(double) * (size_t)m * m) * 3;                 // Psi, Gram, V
    b += ws_round(sizeof(double) * m) + ws_round(sizeof(int) * m);     // ev, order
    b += ws_round(sizeof(double) * (size_t)m * k) * 3;                 // Vk, VkS, Uk
    b += ws_round(sizeof(double) * k);                                 // s_k
    size_t part = gemm_tn_f64_ws(n1, m, m);
    if (gemm_tn_f64_ws(m, m, m) > part) part = gemm_tn_f64_ws(m, m, m);
    b += part;
    b += ws_round(sizeof(double) * (size_t)n1 * k) + ws_round(sizeof(double) * (size_t)n2 * k);   // J', K'
    b += ws_round(sizeof(double) * (size_t)k * k) * 2;                 // RJinv, RKinv
    b += ws_round(sizeof(int32_t) * 2);                                // QR status words
    const size_t q1 = cholqr2_ws(n1, k), q2 = cholqr2_ws(n2, k);
    b += q1 > q2 ? q1 : q2;
    b += jacobi_ws_bytes(m);
    return b;
}

extern "C" int otm_pinv_factors(const double* J, const double* K, const double* S_left, int32_t n1, int32_t n2,
                                int32_t m, int32_t k, double* QJ, double* QK, double* core, double* sv, int32_t* info,
                                void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(J && K && S_left && QJ && QK && core && info, OTM_EINVAL,
                "J, K, S_left, QJ, QK, core, info must not be NULL");
    OTM_REQUIRE(m >= 1 && m <= kMaxM && k >= 1 && k <= m, OTM_ECAPACITY, "need 1 <= k <= m <= 256");
    OTM_REQUIRE(k <= kMaxRank && k <= n1 && k <= n2, OTM_ESHAPE, "need k <= min(n1, n2, 200)");
    OTM_REQUIRE(ws && ws_bytes >= otm_pinv_factors_workspace(n1, n2, m, k), OTM_EWORKSPACE,
                "pinv_factors workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    double* Psi = wc.take<double>((size_t)m * m);
    double* Gr = wc.take<double>((size_t)m * m);
    double* V = wc.take<double>((size_t)m * m);
    double* ev = wc.take<double>(m);
    int* ord = wc.take<int>(m);
    double* Vk = wc.take<double>((size_t)m * k);
    double* VkS = wc.take<double>((size_t)m * k);
    double* Uk = wc.take<double>((size_t)m * k);
    double* sk = wc.take<double>(k);
    size_t part_bytes = gemm_tn_f64_ws(n1, m, m);
    if (gemm_tn_f64_ws(m, m, m) > part_bytes) part_bytes = gemm_tn_f64_ws(m, m, m);
    double* part = wc.take<double>(part_bytes / sizeof(double));
    double* Jk = wc.take<double>((size_t)n1 * k);
    double* Kk = wc.take<double>((size_t)n2 * k);
    double* RJi = wc.take<double>((size_t)k * k);
    double* RKi = wc.take<double>((size_t)k * k);
    int32_t* qinfo = wc.take<int32_t>(2);
    const size_t qb = cholqr2_ws(n1, k) > cholqr2_ws(n2, k) ? cholqr2_ws(n1, k) : cholqr2_ws(n2, k);
    void* qws = wc.take<char>(qb);
    void* jws = wc.take<char>(jacobi_ws_bytes(m));
    int st;
    if ((st = gemm_tn_f64(S_left, m, J, m, n1, m, m, Psi, part, s)) != OTM_OK) return st;   // Psi = S_left^T J
    if ((st = gemm_tn_f64(Psi, m, Psi, m, m, m, m, Gr, part, s)) != OTM_OK) return st;      // Psi^T Psi
    if ((st = jacobi(Gr, V, m, ev, ord, jws, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(svd_topk_kernel, dim3(grid_for((int64_t)m * k)), dim3(256), 0, s, V, ev, ord, m, k, Vk, VkS, sk,
                       info);
    if ((st = check_launch("svd_topk_kernel")) != OTM_OK) return st;
    if ((st = gemm_nn_f64(Psi, m, VkS, k, Uk, k, m, m, k, s)) != OTM_OK) return st;          // U_k = Psi V_k / s
    if ((st = gemm_nn_f64(J, m, Vk, k, Jk, k, n1, m, k, s)) != OTM_OK) return st;            // J' = J V_k
    if ((st = gemm_nn_f64(K, m, Uk, k, Kk, k, n2, m, k, s)) != OTM_OK) return st;            // K' = K U_k
    // each QR writes its own status word (its first pass stores, the second
    // or-s); the core kernel or-s both into info after the rank test's value
    if ((st = cholqr2(Jk, n1, k, QJ, RJi, qinfo, qws, s)) != OTM_OK) return st;
    if ((st = cholqr2(Kk, n2, k, QK, RKi, qinfo + 1, qws, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(pinv_core_kernel, dim3(grid_for((int64_t)k * k)), dim3(256), 0, s, RKi, sk, RJi, k, qinfo, core,
                       info);
    if ((st = check_launch("pinv_core_kernel")) != OTM_OK) return st;
    if (sv) {
        hipError_t e = hipMemcpyAsync(sv, sk, sizeof(double) * k, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "pinv_factors singular values");
    }
    return OTM_OK;
}

extern "C" size_t otm_factored_apply_workspace(int32_t n_in, int32_t k, int32_t m) {
    if (n_in < 1 || k < 1 || m < 1) return 0;
    return factored_ws(n_in, k, m);
}

extern "C" int otm_factored_apply(const double* Q_in, int32_t n_in, const double* core, int trans, const double* Q_out,
                                  int32_t n_out, int32_t k, const double* X, int32_t m, double* Y, void* ws,
                                  size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(Q_in && core && Q_out && X && Y, OTM_EINVAL, "Q_in, core, Q_out, X, Y must not be NULL");
    OTM_REQUIRE(n_in >= 1 && n_out >= 1 && k >= 1 && m >= 1, OTM_ESHAPE, "need positive sizes");
    OTM_REQUIRE(ws && ws_bytes >= otm_factored_apply_workspace(n_in, k, m), OTM_EWORKSPACE,
                "factored_apply workspace too small");
    return factored_apply_impl(Q_in, n_in, core, trans ? 1 : 0, Q_out, n_out, k, X, m, Y, ws, as_stream(stream));
}

extern "C" size_t otm_transition_t_workspace(const otm_partition* G, int32_t k, int32_t m) {
    if (!G || k < 1 || m < 1 || G->XA.n_rows < 1) return 0;
    return transition_ws(G, k, m);
}

extern "C" int otm_transition_t_apply(const otm_partition* G, const double* QJ, const double* QK, const double* core,
                                      int32_t k, int view, const double* V, int32_t m, double* out, void* ws,
                                      size_t ws_bytes, otm_stream stream) {
    int st = check_partition(G);
    if (st != OTM_OK) return st;
    OTM_REQUIRE(QJ && QK && core && V && out, OTM_EINVAL, "QJ, QK, core, V, out must not be NULL");
    OTM_REQUIRE(view == 1 || view == 2, OTM_EINVAL, "view must be 1 (B) or 2 (C)");
    OTM_REQUIRE(m >= 1 && m <= kMaxM && k >= 1, OTM_ECAPACITY, "need k >= 1 and 1 <= m <= 256");
    OTM_REQUIRE(ws && ws_bytes >= otm_transition_t_workspace(G, k, m), OTM_EWORKSPACE,
                "transition_t_apply workspace too small");
    return transition_t_impl(G, QJ, QK, core, k, view, V, m, out, ws, as_stream(stream));
}

extern "C" size_t otm_m2_apply_four_workspace(const otm_partition* G, int32_t k, int32_t m) {
    if (!G || k < 1 || m < 1 || G->XA.n_rows < 1) return 0;
    const int nx = G->XA.n_rows, nA = G->XA.n_cols, nB = G->XB.n_cols, nC = G->XC.n_cols;
    size_t b = transition_ws(G, k, m);                            // u = Z_B^T S (scratch reused below)
    b += ws_round(sizeof(double) * (size_t)nB * m) * 2;           // u, Z_C's inner factored product
    b += ws_round(sizeof(double) * (size_t)nC * m);               // w
    b += ws_round(sizeof(double) * (size_t)nA * m);               // z
    b += ws_round(sizeof(double) * (size_t)nA) + ws_round(sizeof(double) * m);   // M1, v
    b += gemm_tn_f64_ws(nA, 1, m);
    (void)nx;
    return b;
}

extern "C" int otm_m2_apply_four(const otm_partition* G, const double* QJ, const double* QK, const double* core,
                                 int32_t k, double alpha0, const double* S, int32_t m, double* O, void* ws,
                                 size_t ws_bytes, otm_stream stream) {
    int st = check_partition(G);
    if (st != OTM_OK) return st;
    OTM_REQUIRE(QJ && QK && core && S && O, OTM_EINVAL, "QJ, QK, core, S, O must not be NULL");
    OTM_REQUIRE(m >= 1 && m <= kMaxM && k >= 1, OTM_ECAPACITY, "need k >= 1 and 1 <= m <= 256");
    OTM_REQUIRE(std::isfinite(alpha0) && alpha0 >= 0.0, OTM_EINVAL, "alpha0 must be finite and >= 0");
    OTM_REQUIRE(ws && ws_bytes >= otm_m2_apply_four_workspace(G, k, m), OTM_EWORKSPACE,
                "m2_apply_four workspace too small");
    hipStream_t s = as_stream(stream);
    const int nx = G->XA.n_rows, nA = G->XA.n_cols, nB = G->XB.n_cols, nC = G->XC.n_cols;
    WsCarver wc(ws, ws_bytes);
    void* tws = wc.take<char>(transition_ws(G, k, m));
    double* u = wc.take<double>((size_t)nB * m);
    double* zin = wc.take<double>((size_t)nB * m);
    double* w = wc.take<double>((size_t)nC * m);
    double* z = wc.take<double>((size_t)nA * m);
    double* M1 = wc.take<double>(nA);
    double* v = wc.take<double>(m);
    double* part = wc.take<double>(gemm_tn_f64_ws(nA, 1, m) / sizeof(double));
    // u = Z_B^T S
    if ((st = transition_t_impl(G, QJ, QK, core, k, 1, S, m, u, tws, s)) != OTM_OK) return st;
    // w = Pairs(C, B) u = (1/n_X) G[C, X] (G[X, B] u); the transition scratch holds n_X x m first
    WsCarver tc(tws, transition_ws(G, k, m));
    double* tmp = tc.take<double>((size_t)nx * m);
    double* X2 = tc.take<double>((size_t)(nB > nC ? nB : nC) * m);
    void* fws = tc.take<char>(factored_ws(nB > nC ? nB : nC, k, m));
    (void)X2;
    if ((st = pairs_apply_impl(G->CX, G->XB, u, m, w, tmp, s)) != OTM_OK) return st;
    // z = Z_C w = Pairs(A, B) (Q_J Core^T Q_K^T w)
    if ((st = factored_apply_impl(QK, nC, core, 1, QJ, nB, k, w, m, zin, fws, s)) != OTM_OK) return st;
    if ((st = pairs_apply_impl(G->AX, G->XB, zin, m, z, tmp, s)) != OTM_OK) return st;
    // M1 = (1/n_X) G[A, X] 1, v = M1^T S
    hipLaunchKernelGGL(row_sum_kernel, dim3(grid_for((int64_t)nA * 64)), dim3(256), 0, s, G->AX, 1.0 / nx, M1);
    if ((st = check_launch("row_sum_kernel")) != OTM_OK) return st;
    if ((st = gemm_tn_f64(M1, 1, S, m, nA, 1, m, v, part, s)) != OTM_OK) return st;
    hipLaunchKernelGGL(rank1_epilogue_kernel, dim3(grid_for((int64_t)nA * m)), dim3(256), 0, s, z, M1, v, (int64_t)nA,
                       m, alpha0 + 1.0, alpha0, O);
    return check_launch("rank1_epilogue_kernel");
}

extern "C" int otm_cast_rows(const double* X, int32_t rows, int32_t cols, int32_t ldx, void* out, int dtype,
                             int32_t ldo, otm_stream stream) {
    OTM_REQUIRE(X && out, OTM_EINVAL, "X and out must not be NULL");
    OTM_REQUIRE(rows >= 0 && cols >= 1 && ldx >= cols && ldo >= cols, OTM_ESHAPE, "need ldx, ldo >= cols >= 1");
    OTM_REQUIRE(dtype == OTM_F32 || dtype == OTM_BF16, OTM_EDTYPE, "out must be F32 or BF16");
    if (rows == 0) return OTM_OK;
    const int64_t total = (int64_t)rows * ldo;
    hipLaunchKernelGGL(cast_rows_kernel, dim3(grid_for(total)), dim3(256), 0, as_stream(stream), X, (int64_t)rows, cols,
                       ldx, out, dtype, ldo);
    return check_launch("cast_rows_kernel");
}
