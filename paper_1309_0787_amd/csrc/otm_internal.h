// Internal declarations shared by the translation units of libotm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/otm.h"

namespace otm {

// ---------------------------------------------------------------- errors
int fail(int status, const std::string& msg);   // records msg, returns status
int hip_fail(hipError_t e, const char* where);  // OTM_EHIP with the HIP message
int check_launch(const char* where);            // hipGetLastError after a launch

#define OTM_REQUIRE(cond, status, msg)                     \
    do {                                                   \
        if (!(cond)) return ::otm::fail((status), (msg));  \
    } while (0)

inline hipStream_t as_stream(otm_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------ workspace
// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct WsCarver {
    char* base;
    size_t cap;
    size_t off = 0;
    WsCarver(void* p, size_t bytes) : base(static_cast<char*>(p)), cap(bytes) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
    bool ok() const { return off <= cap; }
};

inline size_t ws_round(size_t bytes) { return (bytes + 255) & ~size_t(255); }

int validate_csr_header(const otm_csr* C, const char* name);

// Symmetric FP64 eigensolver for n <= 256 (jacobi.hip): A (n x n, overwritten),
// V (n x n, eigenvectors as columns), evals[i] = eigenvalue of column i,
// order[j] = column of the j-th largest eigenvalue.  ws: jacobi_ws_bytes(n).
size_t jacobi_ws_bytes(int n);
int jacobi(double* A, double* V, int n, double* evals, int* order, void* ws, hipStream_t s);

// FP64 dense products (dense64.hip): C (p x q) = A^T B for tall A (d x p),
// B (d x q), split over row chunks into `part` (gemm_tn_f64_ws bytes), then a
// fixed-order reduction; C (d x q) = A B for tall A (d x p), small B (p x q).
size_t gemm_tn_f64_ws(int d, int p, int q);
int gemm_tn_f64(const double* A, int lda, const double* B, int ldb, int d, int p, int q, double* C, double* part,
                hipStream_t s);
int gemm_nn_f64(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int d, int p, int q,
                hipStream_t s);
// Cholesky QR applied twice (m <= 200): Q (d x m) orthonormal with Y = Q R,
// and Rinv = R^-1 (m x m, upper triangular).  info as in otm_orthonormalize.
size_t cholqr2_ws(int d, int m);
int cholqr2(const double* Y, int d, int m, double* Q, double* Rinv, int32_t* info, void* ws, hipStream_t s);

// FP64 sparse-dense product (spmm.hip): Y[r, :] = scale sum_j C[r, j] X[j, :]
// for m <= 256 columns, rows of X and Y m apart.  Out-of-range columns are
// skipped as in every kernel of the library.
int spmm64(const otm_csr& C, const double* X, int m, double scale, double* Y, hipStream_t s);

// ------------------------------------------------------------- numerics
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf16_to_f32(__bf16 x) { return static_cast<float>(x); }
__device__ __forceinline__ __bf16 f32_to_bf16(float x) { return static_cast<__bf16>(x); }

constexpr int kMaxK = 128;       // STGD capacity (components)
constexpr int kMaxBatch = 128;   // STGD capacity (mini-batch rows)

}  // namespace otm
