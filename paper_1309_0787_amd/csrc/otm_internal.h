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
