// Measurement probes: the rates that the roofline fractions are taken against,
// measured on the device at hand beside the datasheet figures.
//
//  * copy: dst = src over `bytes` (16-byte vectors, grid-stride), for HBM
//    bandwidth (read + write bytes over the time);
//  * matrix cores: every wave of a whole-device grid issues `iters` rounds of
//    eight independent 16x16 MFMA chains (BF16 16x16x32, FP32 16x16x4 or FP64
//    16x16x4), for the dense matrix-core rate of that type.
#include "otm_internal.h"

namespace otm {
namespace {

__global__ __launch_bounds__(256) void probe_copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                         int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void probe_mfma_bf16_kernel(int64_t iters, float* __restrict__ out) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = f32_to_bf16(1.0f + 1e-3f * (threadIdx.x & 7));
        b[e] = f32_to_bf16(1e-3f);
    }
    f32x4 c[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) c[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[j], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_mfma_f32_kernel(int64_t iters, float* __restrict__ out) {
    const float a = 1.0f + 1e-3f * (threadIdx.x & 7), b = 1e-3f;
    f32x4 c[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) c[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[j], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void probe_mfma_f64_kernel(int64_t iters, float* __restrict__ out) {
    const double a = 1.0 + 1e-3 * (threadIdx.x & 7), b = 1e-3;
    f64x4 c[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) c[j] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[j], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = static_cast<float>(s);
}

}  // namespace
}  // namespace otm

using namespace otm;

extern "C" int otm_probe_copy(const void* src, void* dst, int64_t bytes, int32_t blocks, otm_stream stream) {
    OTM_REQUIRE(src && dst && src != dst, OTM_EINVAL, "src and dst must be distinct and not NULL");
    OTM_REQUIRE(bytes > 0 && bytes % 16 == 0, OTM_ESHAPE, "bytes must be a positive multiple of 16");
    OTM_REQUIRE((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 == 0, OTM_EINVAL,
                "src and dst must be 16-byte aligned");
    OTM_REQUIRE(blocks >= 1, OTM_EINVAL, "blocks must be >= 1");
    hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks), dim3(256), 0, as_stream(stream),
                       static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), bytes / 16);
    return check_launch("probe_copy_kernel");
}

extern "C" int64_t otm_probe_mfma_flops(int dtype, int64_t iters, int32_t blocks) {
    // 2 m n k flops per instruction: BF16 16x16x32, FP32 and FP64 16x16x4
    const int64_t per = dtype == OTM_BF16 ? 2 * 16 * 16 * 32 : 2 * 16 * 16 * 4;
    return per * kChains * iters * (int64_t)blocks * 4;   // four waves per block
}

extern "C" int otm_probe_mfma(int dtype, int64_t iters, int32_t blocks, float* out, otm_stream stream) {
    OTM_REQUIRE(out != nullptr, OTM_EINVAL, "out must not be NULL");
    OTM_REQUIRE(iters >= 1 && blocks >= 1, OTM_EINVAL, "iters and blocks must be >= 1");
    hipStream_t s = as_stream(stream);
    if (dtype == OTM_BF16)
        hipLaunchKernelGGL(probe_mfma_bf16_kernel, dim3(blocks), dim3(256), 0, s, iters, out);
    else if (dtype == OTM_F32)
        hipLaunchKernelGGL(probe_mfma_f32_kernel, dim3(blocks), dim3(256), 0, s, iters, out);
    else if (dtype == OTM_F64)
        hipLaunchKernelGGL(probe_mfma_f64_kernel, dim3(blocks), dim3(256), 0, s, iters, out);
    else
        return fail(OTM_EDTYPE, "dtype must be F64, F32 or BF16");
    return check_launch("probe_mfma_kernel");
}
