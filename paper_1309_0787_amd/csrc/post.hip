// Post-processing (Section 3.3, Lemma "postprocessing") and the loss used only
// for measurement (the residual of the decomposition against the explicitly
// formed whitened tensor of Section 3.2).
#include <cmath>

#include "otm_internal.h"

namespace otm {
namespace {

template <class T>
__device__ __forceinline__ double ld64(const T* p) { return static_cast<double>(static_cast<float>(*p)); }

// UlT[a*k + i] = u_i[a] / lambda_i with lambda_i = kappa ||phi_i||^3
__global__ void pi_prep_kernel(const float* __restrict__ Phi, int k, double kappa, double* __restrict__ UlT) {
    const int i = threadIdx.x;
    if (i >= k) return;
    double nn = 0.0;
    for (int a = 0; a < k; ++a) {
        const double v = Phi[(size_t)i * k + a];
        nn += v * v;
    }
    const double nrm = sqrt(nn);
    const double lam = kappa * nrm * nn;
    for (int a = 0; a < k; ++a) UlT[(size_t)a * k + i] = static_cast<double>(Phi[(size_t)i * k + a]) / nrm / lam;
}

constexpr int kPiSamples = 32;
constexpr int kPiThreads = 256;

template <class TY>
__global__ __launch_bounds__(kPiThreads) void recover_pi_kernel(const TY* __restrict__ Y, int ldy, int n, int k,
                                                                const double* __restrict__ UlT, double tau,
                                                                float* __restrict__ Pi) {
    __shared__ double sY[kPiSamples][kMaxK + 1];
    __shared__ double sR[kPiSamples][kMaxK + 1];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kPiSamples;
    for (int e = tid; e < kPiSamples * k; e += kPiThreads) {
        const int xs = e / k, a = e % k;
        const int x = x0 + xs;
        sY[xs][a] = (x < n) ? ld64(Y + (size_t)x * ldy + a) : 0.0;
    }
    __syncthreads();
    const int i = tid % 128, half = tid / 128;   // rows i, samples half*16 .. half*16+15
    if (i < k) {
        double acc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.0;
        for (int a = 0; a < k; ++a) {
            const double w = UlT[(size_t)a * k + i];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] += w * sY[half * 16 + u][a];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) sR[half * 16 + u][i] = acc[u];
    }
    __syncthreads();
    if (tid < kPiSamples) {
        const int x = x0 + tid;
        if (x < n) {
            double s = 0.0;
            for (int r = 0; r < k; ++r) {
                const double v = fmax(sR[tid][r], 0.0);
                sR[tid][r] = v;
                s += v;
            }
            double s2 = 0.0;
            for (int r = 0; r < k; ++r) {
                double v = (s > 0.0) ? sR[tid][r] / s : 0.0;
                if (v < tau) v = 0.0;
                sR[tid][r] = v;
                s2 += v;
            }
            for (int r = 0; r < k; ++r)
                Pi[(size_t)r * n + x] = static_cast<float>((s2 > 0.0) ? sR[tid][r] / s2 : 0.0);
        }
    }
}

// ---------------------------------------------------------------- tensor form
constexpr int kTfThreads = 256;
constexpr int kTfRows = 16;
constexpr int kTfB = 16;                                        // b values per block
constexpr int kTfPer = (kTfB * kMaxK + kTfThreads - 1) / kTfThreads;   // (b, c) pairs per thread

// Block (a, bc) forms T[a, b, :] for b in [16 bc, 16 bc + 16).
template <class TY>
__global__ __launch_bounds__(kTfThreads) void tensor_form_kernel(const TY* __restrict__ YA, const TY* __restrict__ YB,
                                                                 const TY* __restrict__ YC, int ldy, int n, int k,
                                                                 const float* __restrict__ ybar, double ca, double cb,
                                                                 double cc, double* __restrict__ T) {
    __shared__ double sA[kTfRows];
    __shared__ double sB[kTfRows][kTfB];
    __shared__ double sC[kTfRows][kMaxK];
    __shared__ double sAB[kTfB], sAC[kMaxK];
    const int a = blockIdx.x;
    const int b0 = blockIdx.y * kTfB;
    const int nb = min(kTfB, k - b0);
    const int tid = threadIdx.x;
    const int pairs = nb * k;
    double acc[kTfPer], accbc[kTfPer];
#pragma unroll
    for (int j = 0; j < kTfPer; ++j) { acc[j] = 0.0; accbc[j] = 0.0; }
    double s_ab = 0.0, s_ac = 0.0;
    for (int t0 = 0; t0 < n; t0 += kTfRows) {
        const int rows = min(kTfRows, n - t0);
        for (int e = tid; e < rows * k; e += kTfThreads) {
            const int r = e / k, c = e % k;
            sC[r][c] = ld64(YC + (size_t)(t0 + r) * ldy + c);
        }
        for (int e = tid; e < rows * nb; e += kTfThreads) {
            const int r = e / nb, c = e % nb;
            sB[r][c] = ld64(YB + (size_t)(t0 + r) * ldy + b0 + c);
        }
        if (tid < rows) sA[tid] = ld64(YA + (size_t)(t0 + tid) * ldy + a);
        __syncthreads();
        for (int r = 0; r < rows; ++r) {
            const double ya = sA[r];
#pragma unroll
            for (int j = 0; j < kTfPer; ++j) {
                const int e = tid + j * kTfThreads;
                if (e < pairs) {
                    const double bc = sB[r][e / k] * sC[r][e % k];
                    acc[j] += ya * bc;
                    accbc[j] += bc;
                }
            }
            if (tid < nb) s_ab += ya * sB[r][tid];
            if (tid < k) s_ac += ya * sC[r][tid];
        }
        __syncthreads();
    }
    if (tid < nb) sAB[tid] = s_ab;
    if (tid < k) sAC[tid] = s_ac;
    __syncthreads();
    const double inv_n = 1.0 / n;
    const double ybA = ybar[a];
#pragma unroll
    for (int j = 0; j < kTfPer; ++j) {
        const int e = tid + j * kTfThreads;
        if (e >= pairs) continue;
        const int bl = e / k, c = e % k, b = b0 + bl;
        const double ybB = ybar[k + b], ybC = ybar[2 * k + c];
        const double v = ca * inv_n * acc[j] - cb * inv_n * (sAB[bl] * ybC + sAC[c] * ybB + ybA * accbc[j]) +
                         cc * ybA * ybB * ybC;
        T[((size_t)a * k + b) * k + c] = v;
    }
}

// part[(j*k + i)*2 + 0] = sum_l (phi_i . phi_l)^3 ; part[.. + 1] = T(phi_i, phi_i, phi_i)
__global__ __launch_bounds__(256) void residual_part_kernel(const double* __restrict__ T, int k,
                                                            const float* __restrict__ Phi, double* __restrict__ part) {
    __shared__ double sphi[kMaxK];
    __shared__ double sred[256];
    const int j = blockIdx.x, i = blockIdx.y, tid = threadIdx.x;
    const float* P = Phi + (size_t)j * k * k;
    if (tid < k) sphi[tid] = P[(size_t)i * k + tid];
    __syncthreads();
    double self = 0.0;
    for (int l = tid; l < k; l += 256) {
        double dot = 0.0;
        for (int a = 0; a < k; ++a) dot += sphi[a] * static_cast<double>(P[(size_t)l * k + a]);
        self += dot * dot * dot;
    }
    double cross = 0.0;
    for (int e = tid; e < k * k; e += 256) {
        const int a = e / k, b = e % k;
        const double* tr = T + (size_t)e * k;
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += tr[c] * sphi[c];
        cross += sphi[a] * sphi[b] * s;
    }
    for (int pass = 0; pass < 2; ++pass) {
        sred[tid] = pass == 0 ? self : cross;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) sred[tid] += sred[tid + s];
            __syncthreads();
        }
        if (tid == 0) part[((size_t)j * k + i) * 2 + pass] = sred[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void residual_final_kernel(const double* __restrict__ T, int k,
                                                             const double* __restrict__ part, double* __restrict__ R) {
    __shared__ double sred[256];
    const int j = blockIdx.x, tid = threadIdx.x;
    const int64_t m = (int64_t)k * k * k;
    double tt = 0.0;
    for (int64_t e = tid; e < m; e += 256) tt += T[e] * T[e];
    sred[tid] = tt;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) sred[tid] += sred[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        const double tsum = sred[0];
        double self = 0.0, cross = 0.0;
        for (int i = 0; i < k; ++i) {
            self += part[((size_t)j * k + i) * 2];
            cross += part[((size_t)j * k + i) * 2 + 1];
        }
        R[j] = (self - 2.0 * cross + tsum) / tsum;
    }
}

}  // namespace
}  // namespace otm

using namespace otm;

extern "C" size_t otm_recover_pi_workspace(int32_t k) {
    if (k < 1) return 0;
    return ws_round(sizeof(double) * (size_t)k * k);
}

extern "C" int otm_recover_pi(const void* Y, int y_dtype, int32_t ldy, int32_t n, int32_t k, const float* Phi,
                              double theta, double tau, float* Pi, void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(Y && Phi && Pi, OTM_EINVAL, "Y, Phi, Pi must not be NULL");
    OTM_REQUIRE(n >= 0 && k >= 1 && k <= kMaxK && ldy >= k, OTM_ESHAPE, "need n >= 0, 1 <= k <= 128, ldy >= k");
    OTM_REQUIRE(y_dtype == OTM_F32 || y_dtype == OTM_BF16, OTM_EDTYPE, "Y must be F32 or BF16");
    OTM_REQUIRE(std::isfinite(theta) && std::isfinite(tau), OTM_EINVAL, "theta and tau must be finite");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_recover_pi_workspace(k), OTM_EWORKSPACE, "recover_pi workspace too small");
    if (n == 0) return OTM_OK;
    hipStream_t s = as_stream(stream);
    double* UlT = static_cast<double*>(ws);
    hipLaunchKernelGGL(pi_prep_kernel, dim3(1), dim3(kMaxK), 0, s, Phi, k, 0.5 * (1.0 + theta), UlT);
    int st = check_launch("pi_prep_kernel");
    if (st != OTM_OK) return st;
    const dim3 grid((n + kPiSamples - 1) / kPiSamples);
    if (y_dtype == OTM_F32)
        hipLaunchKernelGGL(recover_pi_kernel<float>, grid, dim3(kPiThreads), 0, s, static_cast<const float*>(Y), ldy, n,
                           k, UlT, tau, Pi);
    else
        hipLaunchKernelGGL(recover_pi_kernel<__bf16>, grid, dim3(kPiThreads), 0, s, static_cast<const __bf16*>(Y), ldy,
                           n, k, UlT, tau, Pi);
    return check_launch("recover_pi_kernel");
}

extern "C" int otm_tensor_form(const void* YA, const void* YB, const void* YC, int y_dtype, int32_t ldy, int32_t n,
                               int32_t k, const float* ybar, double alpha0, double* T, otm_stream stream) {
    OTM_REQUIRE(YA && YB && YC && ybar && T, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(n >= 1 && k >= 1 && k <= kMaxK && ldy >= k, OTM_ESHAPE, "need n >= 1, 1 <= k <= 128, ldy >= k");
    OTM_REQUIRE(y_dtype == OTM_F32 || y_dtype == OTM_BF16, OTM_EDTYPE, "Y must be F32 or BF16");
    OTM_REQUIRE(std::isfinite(alpha0) && alpha0 >= 0.0, OTM_EINVAL, "alpha0 must be finite and >= 0");
    hipStream_t s = as_stream(stream);
    const double ca = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0, cb = alpha0 * (alpha0 + 1.0) / 2.0, cc = alpha0 * alpha0;
    if (y_dtype == OTM_F32)
        hipLaunchKernelGGL(tensor_form_kernel<float>, dim3(k, (k + kTfB - 1) / kTfB), dim3(kTfThreads), 0, s, static_cast<const float*>(YA),
                           static_cast<const float*>(YB), static_cast<const float*>(YC), ldy, n, k, ybar, ca, cb, cc, T);
    else
        hipLaunchKernelGGL(tensor_form_kernel<__bf16>, dim3(k, (k + kTfB - 1) / kTfB), dim3(kTfThreads), 0, s, static_cast<const __bf16*>(YA),
                           static_cast<const __bf16*>(YB), static_cast<const __bf16*>(YC), ldy, n, k, ybar, ca, cb, cc,
                           T);
    return check_launch("tensor_form_kernel");
}

extern "C" size_t otm_residual_workspace(int32_t k, int32_t count) {
    if (k < 1 || count < 1) return 0;
    return ws_round(sizeof(double) * 2 * (size_t)k * count);
}

extern "C" int otm_residual(const double* T, int32_t k, const float* Phi, int32_t count, double* R, void* ws,
                            size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(T && Phi && R, OTM_EINVAL, "T, Phi, R must not be NULL");
    OTM_REQUIRE(k >= 1 && k <= kMaxK && count >= 1, OTM_ESHAPE, "need 1 <= k <= 128 and count >= 1");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_residual_workspace(k, count), OTM_EWORKSPACE,
                "residual workspace too small");
    hipStream_t s = as_stream(stream);
    double* part = static_cast<double*>(ws);
    hipLaunchKernelGGL(residual_part_kernel, dim3(count, k), dim3(256), 0, s, T, k, Phi, part);
    int st = check_launch("residual_part_kernel");
    if (st != OTM_OK) return st;
    hipLaunchKernelGGL(residual_final_kernel, dim3(count), dim3(256), 0, s, T, k, part, R);
    return check_launch("residual_final_kernel");
}
