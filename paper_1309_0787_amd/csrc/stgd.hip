// Entry points of the single-problem STGD (the kernel body is in stgd_kernel.h).
#include "stgd_kernel.h"

namespace otm {
namespace {

template <class M, int KP, int NSTAGE, bool COMP, int NTL, bool OV>
__global__ __launch_bounds__(kThreads) void sgd_kernel(SgdArgs g) {
    __shared__ __attribute__((aligned(16))) SgdSmem<M, KP, NSTAGE, 4> sm;
    sgd_body<M, KP, NSTAGE, 4, false, COMP, NTL, OV>(g, blockIdx.x, sm);
}

template <class M, int KP, int NSTAGE, bool COMP, bool OV>
int launch_sgd_v(const SgdArgs& a, int restarts, hipStream_t st) {
    // BF16 pads k to a multiple of 32: when k + 2 (the components and the two
    // folded means) fits in one tile less than KP, the last tile row and
    // column of every k x k product hold only padding and are skipped
    if constexpr (M::EPL == 8) {
        if (a.k + 2 <= KP - 16) {
            hipLaunchKernelGGL((sgd_kernel<M, KP, NSTAGE, COMP, KP / 16 - 1, OV>), dim3(restarts), dim3(kThreads), 0, st, a);
            return check_launch("sgd_kernel");
        }
    }
    hipLaunchKernelGGL((sgd_kernel<M, KP, NSTAGE, COMP, KP / 16, OV>), dim3(restarts), dim3(kThreads), 0, st, a);
    return check_launch("sgd_kernel");
}

// Rows read from global memory (no staging) with the three views aliased:
// the body computes the batch product once (P_B = P_A)
template <class M, int KP, int NSTAGE, bool COMP>
int launch_sgd(const SgdArgs& a, int restarts, bool aliased, hipStream_t st) {
    static_assert(smem_bytes<M, KP, NSTAGE>() <= kLdsLimit, "STGD shared memory exceeds 160 KB");
    if constexpr (NSTAGE == 0) {
        if (aliased) return launch_sgd_v<M, KP, NSTAGE, COMP, true>(a, restarts, st);
    }
    return launch_sgd_v<M, KP, NSTAGE, COMP, false>(a, restarts, st);
}

// Picks the instantiation: the smallest padded k, then the largest batch
// staging that fits in LDS (one view when the three views alias).  BF16 runs
// without compensation take the variant that keeps no compensation terms
// (FP32 keeps them: there they also carry -beta kappa O through the step).
template <class M, int KP>
int dispatch_staging(const SgdArgs& a, int restarts, bool aliased, hipStream_t st) {
    constexpr int s1 = staging_for<M, KP>(true), s3 = staging_for<M, KP>(false);
    if constexpr (M::EPL != 1) {
        if (!a.compensated)
            return aliased ? launch_sgd<M, KP, s1, false>(a, restarts, true, st) : launch_sgd<M, KP, s3, false>(a, restarts, false, st);
    }
    return aliased ? launch_sgd<M, KP, s1, true>(a, restarts, true, st) : launch_sgd<M, KP, s3, true>(a, restarts, false, st);
}

int run_common(const otm_sgd_params* p, int32_t n, const void* YA, const void* YB, const void* YC,
               const float* ybar, const int32_t* perms, int64_t perm_stride, int32_t restarts,
               int64_t start_step, int64_t end_step, float* Phi, float* Phi_comp, float* snapshots,
               int32_t* nonfinite, hipStream_t st) {
    OTM_REQUIRE(p != nullptr, OTM_EINVAL, "params is NULL");
    OTM_REQUIRE(YA && YB && YC && ybar && Phi, OTM_EINVAL, "null data pointer");
    OTM_REQUIRE(restarts >= 1, OTM_ESHAPE, "restarts must be >= 1");
    SgdArgs a{};
    int status = fill_scalars(n, p->k, p->ldy, p->alpha0, p, start_step, end_step, a);
    if (status != OTM_OK) return status;
    a.YA = YA; a.YB = YB; a.YC = YC; a.ybar = ybar; a.perms = perms; a.perm_stride = perm_stride;
    a.Phi0 = Phi; a.Phi = Phi; a.Phi_comp = Phi_comp; a.snapshots = snapshots; a.nonfinite = nonfinite;
    a.score = nullptr;
    if (a.start_step == a.end_step && !Phi_comp) return OTM_OK;
    const bool aliased = (YA == YB) && (YB == YC);
    const int k = p->k;
    if (p->y_dtype == OTM_F32) {
        switch ((k + 15) / 16) {
            case 1: return dispatch_staging<MmaF32, 16>(a, restarts, aliased, st);
            case 2: return dispatch_staging<MmaF32, 32>(a, restarts, aliased, st);
            case 3: return dispatch_staging<MmaF32, 48>(a, restarts, aliased, st);
            case 4: return dispatch_staging<MmaF32, 64>(a, restarts, aliased, st);
            case 5: return dispatch_staging<MmaF32, 80>(a, restarts, aliased, st);
            case 6: return dispatch_staging<MmaF32, 96>(a, restarts, aliased, st);
            case 7: return dispatch_staging<MmaF32, 112>(a, restarts, aliased, st);
            default: return dispatch_staging<MmaF32, 128>(a, restarts, aliased, st);
        }
    }
    switch ((k + 31) / 32) {
        case 1: return dispatch_staging<MmaBF16, 32>(a, restarts, aliased, st);
        case 2: return dispatch_staging<MmaBF16, 64>(a, restarts, aliased, st);
        case 3: return dispatch_staging<MmaBF16, 96>(a, restarts, aliased, st);
        default: return dispatch_staging<MmaBF16, 128>(a, restarts, aliased, st);
    }
}

}  // namespace
}  // namespace otm

extern "C" int otm_sgd_run(const otm_sgd_params* p, int32_t n, const void* YA, const void* YB,
                           const void* YC, const float* ybar, const int32_t* perms, int64_t perm_stride,
                           int32_t restarts, int64_t start_step, int64_t end_step, float* Phi,
                           float* Phi_comp, float* snapshots, int32_t* nonfinite, otm_stream stream) {
    return otm::run_common(p, n, YA, YB, YC, ybar, perms, perm_stride, restarts, start_step, end_step,
                           Phi, Phi_comp, snapshots, nonfinite, otm::as_stream(stream));
}

extern "C" int otm_sgd_step(const otm_sgd_params* p, int32_t rows, const void* YA, const void* YB,
                            const void* YC, const float* ybar, double beta, float* Phi, float* Phi_comp,
                            otm_stream stream) {
    if (p == nullptr) return otm::fail(OTM_EINVAL, "params is NULL");
    if (rows < 1 || rows > p->batch) return otm::fail(OTM_ESHAPE, "need 1 <= rows <= batch");
    otm_sgd_params q = *p;
    q.passes = 1;
    q.beta0 = beta;
    q.beta_tau = 1.0;
    return otm::run_common(&q, rows, YA, YB, YC, ybar, nullptr, 0, 1, 0, 1, Phi, Phi_comp, nullptr,
                           nullptr, otm::as_stream(stream));
}
