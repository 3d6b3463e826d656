// Status handling, CSR validation and small entry points of libotm.
#include <cstdio>
#include <string>

#include "otm_internal.h"

namespace otm {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return OTM_EHIP;
}

int check_launch(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, where);
    return OTM_OK;
}

int validate_csr_header(const otm_csr* C, const char* name) {
    if (C == nullptr) return fail(OTM_EINVAL, std::string(name) + " is NULL");
    if (C->n_rows < 0 || C->n_cols < 0 || C->nnz < 0)
        return fail(OTM_ESHAPE, std::string(name) + ": negative size");
    if (C->rowptr == nullptr) return fail(OTM_EINVAL, std::string(name) + ": rowptr is NULL");
    if (C->nnz > 0 && C->colidx == nullptr) return fail(OTM_EINVAL, std::string(name) + ": colidx is NULL");
    if (C->nnz >= (int64_t(1) << 31)) return fail(OTM_ECAPACITY, std::string(name) + ": nnz must be < 2^31");
    return OTM_OK;
}

namespace {

// Counts CSR violations: rowptr[0] != 0, decreasing rowptr, rowptr[n] != nnz,
// column indices outside [0, n_cols).  One partial count per block.
__global__ void csr_check_kernel(otm_csr C, unsigned long long* partial) {
    __shared__ unsigned long long red[256];
    unsigned long long bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t r = start; r < C.n_rows; r += stride)
        if (C.rowptr[r + 1] < C.rowptr[r]) ++bad;
    for (int64_t e = start; e < C.nnz; e += stride) {
        const int32_t c = C.colidx[e];
        if (c < 0 || c >= C.n_cols) ++bad;
    }
    if (start == 0) {
        if (C.rowptr[0] != 0) ++bad;
        if ((int64_t)C.rowptr[C.n_rows] != C.nnz) ++bad;
    }
    red[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

constexpr int kCheckBlocks = 256;

}  // namespace
}  // namespace otm

extern "C" {

const char* otm_status_string(int status) {
    switch (status) {
        case OTM_OK: return "ok";
        case OTM_EINVAL: return "invalid argument";
        case OTM_ESHAPE: return "inconsistent shape";
        case OTM_EDTYPE: return "unsupported dtype";
        case OTM_ENOTPSD: return "second moment not positive definite on the projection";
        case OTM_ENONFINITE: return "non-finite value";
        case OTM_EHIP: return "HIP runtime error";
        case OTM_EWORKSPACE: return "workspace missing or too small";
        case OTM_ECAPACITY: return "size beyond compiled capacity";
        default: return "unknown status";
    }
}

const char* otm_last_error(void) { return otm::g_last_error.c_str(); }

int otm_version(void) { return 1; }
int otm_max_k(void) { return otm::kMaxK; }
int otm_max_batch(void) { return otm::kMaxBatch; }

size_t otm_csr_check_workspace(void) { return otm::kCheckBlocks * sizeof(unsigned long long); }

int otm_csr_check(const otm_csr* C, int64_t* bad_count, void* ws, size_t ws_bytes, otm_stream stream) {
    int st = otm::validate_csr_header(C, "C");
    if (st != OTM_OK) return st;
    if (bad_count == nullptr) return otm::fail(OTM_EINVAL, "bad_count is NULL");
    if (ws == nullptr || ws_bytes < otm_csr_check_workspace())
        return otm::fail(OTM_EWORKSPACE, "csr_check workspace too small");
    hipStream_t s = otm::as_stream(stream);
    auto* partial = static_cast<unsigned long long*>(ws);
    hipLaunchKernelGGL(otm::csr_check_kernel, dim3(otm::kCheckBlocks), dim3(256), 0, s, *C, partial);
    st = otm::check_launch("csr_check_kernel");
    if (st != OTM_OK) return st;
    unsigned long long host[otm::kCheckBlocks];
    hipError_t e = hipMemcpyAsync(host, partial, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return otm::hip_fail(e, "csr_check copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return otm::hip_fail(e, "csr_check sync");
    unsigned long long total = 0;
    for (int i = 0; i < otm::kCheckBlocks; ++i) total += host[i];
    *bad_count = static_cast<int64_t>(total);
    return OTM_OK;
}

}  // extern "C"
