// Stochastic tensor gradient descent on the implicit whitened third moment
// (Section 3.2, Lemma "update"), in the stacked matrix form of Section 4.3:
//
//   PA = YA Phi, PB = YB Phi                       (batch x k, matrix cores)
//   mA = Phi^T ybarA, mB = Phi^T ybarB             (k, vector ALU)
//   H  = PA * PB,  s = column sums of H            (wave shuffles)
//   Q  = a H - b PA diag(mB) - b diag(mA) PB
//   D  = YC^T Q / B + ybarC (c mA*mB - b s / B)^T  (matrix cores)
//   G  = Phi^T Phi,  O = Phi (G * G)               (matrix cores)
//   Phi <- Phi + beta (D - kappa O)                 (compensated FP32)
//
// One workgroup of 8 waves runs one whole online run (all steps), keeping the
// FP32 master copy of Phi (and its Kahan compensation) in registers.  The
// tensor is never formed.  Wave (wr, wc), wr in 0..3, wc in 0..1, owns the
// 16x16 output tiles (mt, nt) with mt = wr mod 4 and nt = wc mod 2 of every
// product, so the update of a Phi tile needs only the O and D tiles the same
// wave computed.  LDS holds operand copies of Phi (phi_i-major, plus an
// a-major copy for BF16 fragments), a buffer that carries G*G and then Q from
// the accumulator layout to the operand layout, for BF16 the batch of YC
// (a-major, the operand layout of YC^T Q), and small vectors.
// Four workgroup barriers per step: after G*G, after O (the buffer then
// takes Q), after Q, after the update.
#include <cmath>

#include "otm_internal.h"

namespace otm {
namespace {

// ---------------------------------------------------------------------------
// Matrix-core flavours.  Lane l of a 16x16xKI instruction supplies
//   A[l % 16][EPL*(l/16) + e] and B[EPL*(l/16) + e][l % 16], e < EPL,
// and receives C[4*(l/16) + r][l % 16], r < 4.
// ---------------------------------------------------------------------------
struct MmaF32 {
    using Y = float;
    using Op = float;
    using Frag = float;
    static constexpr int KI = 4;
    static constexpr int EPL = 1;
    static constexpr int KMUL = 16;   // padding multiple of k and of the batch
    static constexpr int SPAD = 4;    // LDS row padding (elements)
    static constexpr bool kPhiT = false;
    static constexpr bool kStageC = false;   // YC operand read straight from global memory
    __device__ static f32x4 mma(Frag a, Frag b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static Frag lds(const Op* p) { return *p; }
    __device__ static Op to_op(float x) { return x; }
    __device__ static float op_to_f(Op x) { return x; }
    __device__ static float y_to_f(Y x) { return x; }
    // fragment of EPL consecutive row elements a0.. (masked at k)
    __device__ static Frag yrow(const Y* row, int a0, int k) {
        return (row != nullptr && a0 < k) ? row[a0] : 0.0f;
    }
    __device__ static void store4(Op* p, f32x4 v) {
        *reinterpret_cast<f32x4*>(p) = v;
    }
};

struct MmaBF16 {
    using Y = __bf16;
    using Op = __bf16;
    using Frag = bf16x8;
    static constexpr int KI = 32;
    static constexpr int EPL = 8;
    static constexpr int KMUL = 32;
    static constexpr int SPAD = 8;
    static constexpr bool kPhiT = true;
    static constexpr bool kStageC = true;    // YC batch staged in LDS, a-major
    __device__ static f32x4 mma(Frag a, Frag b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static Frag lds(const Op* p) { return *reinterpret_cast<const bf16x8*>(p); }
    __device__ static Op to_op(float x) { return f32_to_bf16(x); }
    __device__ static float op_to_f(Op x) { return bf16_to_f32(x); }
    __device__ static float y_to_f(Y x) { return bf16_to_f32(x); }
    __device__ static Frag yrow(const Y* row, int a0, int k) {
        bf16x8 v;
        if (row != nullptr && a0 < k) {
            // ldy % 8 == 0 and a0 % 8 == 0: the 16-byte load stays inside the row
            v = *reinterpret_cast<const bf16x8*>(row + a0);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (a0 + e >= k) v[e] = f32_to_bf16(0.0f);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = f32_to_bf16(0.0f);
        }
        return v;
    }
    __device__ static void store4(Op* p, f32x4 v) {
        bf16x4 o;
        o[0] = f32_to_bf16(v[0]);
        o[1] = f32_to_bf16(v[1]);
        o[2] = f32_to_bf16(v[2]);
        o[3] = f32_to_bf16(v[3]);
        *reinterpret_cast<bf16x4*>(p) = o;
    }
};

struct SgdArgs {
    const void* YA;
    const void* YB;
    const void* YC;
    const float* ybar;
    const int32_t* perms;
    int64_t perm_stride;
    float* Phi;
    float* Phi_comp;
    float* snapshots;
    int32_t* nonfinite;
    int32_t n, k, batch, passes, ldy, compensated;
    int64_t start_step, end_step, spp;
    float a, b, c, kappa;
    double beta0, beta_tau;
};

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kTR = 2;  // tile rows per wave (4 wave rows x 2 = 8 tiles = 128)

template <class M, int KPMAX>
__global__ __launch_bounds__(kThreads) void sgd_kernel(SgdArgs g) {
    using Op = typename M::Op;
    using Y = typename M::Y;
    constexpr int TC = KPMAX / 32;                 // tile columns per wave
    constexpr int SP = KPMAX + M::SPAD;            // stride of Phi rows in LDS
    constexpr int SB = kMaxBatch + M::SPAD;        // stride of the exchange buffer rows
    __shared__ __attribute__((aligned(16))) Op sPhi[KPMAX * SP];
    __shared__ __attribute__((aligned(16))) Op sPhiT[M::kPhiT ? KPMAX * SP : 1];
    __shared__ __attribute__((aligned(16))) Op sBuf[KPMAX * SB];
    __shared__ __attribute__((aligned(16))) Op sYC[M::kStageC ? KPMAX * SB : 1];
    __shared__ int32_t sIdx[kMaxBatch];
    __shared__ float sYbar[3 * KPMAX];
    __shared__ float sM[2 * KPMAX];
    __shared__ float sS[4 * KPMAX];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int l16 = lane & 15, q = lane >> 4;

    const int k = g.k;
    const int KP = (k + M::KMUL - 1) / M::KMUL * M::KMUL;
    const int MB = (g.batch + M::KMUL - 1) / M::KMUL * M::KMUL;
    const int NTK = KP / 16, NTM = MB / 16;
    const int n = g.n, B = g.batch, ldy = g.ldy;
    const int r_id = blockIdx.x;
    float* Phi = g.Phi + (size_t)r_id * k * k;
    float* Comp = g.Phi_comp ? g.Phi_comp + (size_t)r_id * k * k : nullptr;
    float* Snap = g.snapshots ? g.snapshots + (size_t)r_id * g.passes * k * k : nullptr;
    const int32_t* perms = g.perms ? g.perms + (size_t)r_id * g.perm_stride : nullptr;
    const Y* YA = static_cast<const Y*>(g.YA);
    const Y* YB = static_cast<const Y*>(g.YB);
    const Y* YC = static_cast<const Y*>(g.YC);

    // ---- master copy of Phi in registers: tile (mt, nt) holds a = row, i = column
    f32x4 phi[kTR][TC], comp[kTR][TC];
#pragma unroll
    for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
        for (int tj = 0; tj < TC; ++tj) {
            const int mt = wr + 4 * ti, nt = wc + 2 * tj;
            f32x4 v = {0.f, 0.f, 0.f, 0.f}, cv = {0.f, 0.f, 0.f, 0.f};
            if (mt < NTK && nt < NTK) {
                const int i = nt * 16 + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = mt * 16 + 4 * q + r;
                    if (a < k && i < k) {
                        v[r] = Phi[(size_t)i * k + a];
                        if (Comp && g.compensated) cv[r] = Comp[(size_t)i * k + a];
                    }
                }
                M::store4(&sPhi[i * SP + mt * 16 + 4 * q], v);
                if constexpr (M::kPhiT) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sPhiT[(mt * 16 + 4 * q + r) * SP + i] = M::to_op(v[r]);
                }
            }
            phi[ti][tj] = v;
            comp[ti][tj] = cv;
        }
    for (int e = tid; e < 3 * KPMAX; e += kThreads) {
        const int v = e / KPMAX, a = e % KPMAX;
        sYbar[e] = (a < k) ? g.ybar[v * k + a] : 0.0f;
    }
    __syncthreads();

    bool bad = false;
    for (int64_t t = g.start_step; t < g.end_step; ++t) {
        const int64_t pass = t / g.spp;
        const int s = static_cast<int>(t - pass * g.spp);
        const int row0 = s * B;
        const int nb = min(B, n - row0);
        const float beta = static_cast<float>(g.beta0 / (1.0 + static_cast<double>(t) / g.beta_tau));

        // ================= phase 1: batch rows, mA/mB, G = Phi^T Phi -> G*G
        if (tid < nb) {
            int32_t r = perms ? perms[(size_t)pass * n + row0 + tid] : row0 + tid;
            if (r < 0 || r >= n) {   // a permutation entry out of range reads row 0 and is reported
                r = 0;
                bad = true;
            }
            sIdx[tid] = r;
        }
        {
            const int v = tid >> 8, rem = tid & 255, i = rem >> 1, h = rem & 1;
            float acc = 0.f;
            if (i < KP) {
                const int half = KP >> 1;
                for (int a = h * half; a < (h + 1) * half; ++a)
                    acc += M::op_to_f(sPhi[i * SP + a]) * sYbar[v * KPMAX + a];
            }
            acc += __shfl_xor(acc, 1);
            if (h == 0 && i < KP) sM[v * KPMAX + i] = acc;
        }
        {
            f32x4 acc[kTR][TC];
#pragma unroll
            for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < KP; k0 += M::KI) {
                typename M::Frag fa[kTR], fb[TC];
#pragma unroll
                for (int ti = 0; ti < kTR; ++ti) {
                    const int mt = wr + 4 * ti;
                    if (mt < NTK) fa[ti] = M::lds(&sPhi[(mt * 16 + l16) * SP + k0 + q * M::EPL]);
                }
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int nt = wc + 2 * tj;
                    if (nt < NTK) fb[tj] = M::lds(&sPhi[(nt * 16 + l16) * SP + k0 + q * M::EPL]);
                }
#pragma unroll
                for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj)
                        if (wr + 4 * ti < NTK && wc + 2 * tj < NTK)
                            acc[ti][tj] = M::mma(fa[ti], fb[tj], acc[ti][tj]);
            }
            // G*G into the exchange buffer, column-major: sBuf[i*SB + j] = G[j][i]^2
#pragma unroll
            for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int mt = wr + 4 * ti, nt = wc + 2 * tj;
                    if (mt < NTK && nt < NTK) {
                        f32x4 v = acc[ti][tj] * acc[ti][tj];
                        M::store4(&sBuf[(nt * 16 + l16) * SB + mt * 16 + 4 * q], v);
                    }
                }
        }
        __syncthreads();

        // ================= phase 2: O = Phi (G*G), kept in registers until the update
        f32x4 oacc[kTR][TC];
#pragma unroll
        for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) oacc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < KP; k0 += M::KI) {
            typename M::Frag fa[kTR], fb[TC];
#pragma unroll
            for (int ti = 0; ti < kTR; ++ti) {
                const int mt = wr + 4 * ti;
                if (mt < NTK) {
                    const int a = mt * 16 + l16;
                    if constexpr (M::kPhiT) fa[ti] = M::lds(&sPhiT[a * SP + k0 + q * M::EPL]);
                    else fa[ti] = sPhi[(k0 + q) * SP + a];
                }
            }
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                const int nt = wc + 2 * tj;
                if (nt < NTK) fb[tj] = M::lds(&sBuf[(nt * 16 + l16) * SB + k0 + q * M::EPL]);
            }
#pragma unroll
            for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj)
                    if (wr + 4 * ti < NTK && wc + 2 * tj < NTK)
                        oacc[ti][tj] = M::mma(fa[ti], fb[tj], oacc[ti][tj]);
        }
        __syncthreads();   // every read of G*G is done: the buffer takes Q next

        // ================= phase 3: PA, PB one tile row at a time -> Q into the
        // exchange buffer (sBuf[i*SB + t] = Q[t][i]) and column sums of H
        {
            float colsum[TC];
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) colsum[tj] = 0.f;
#pragma unroll
            for (int ti = 0; ti < kTR; ++ti) {
                const int mt = wr + 4 * ti;
                if (mt >= NTM) continue;
                const int tr = mt * 16 + l16;
                const bool ok = tr < nb;
                const Y* rowA = ok ? YA + (size_t)sIdx[tr] * ldy : nullptr;
                const Y* rowB = ok ? YB + (size_t)sIdx[tr] * ldy : nullptr;
                f32x4 pa[TC], pb[TC];
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    pa[tj] = f32x4{0.f, 0.f, 0.f, 0.f};
                    pb[tj] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
        for (int k0 = 0; k0 < KP; k0 += M::KI) {
                    const typename M::Frag fa = M::yrow(rowA, k0 + q * M::EPL, k);
                    const typename M::Frag fbv = M::yrow(rowB, k0 + q * M::EPL, k);
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) {
                        const int nt = wc + 2 * tj;
                        if (nt < NTK) {
                            const typename M::Frag fphi = M::lds(&sPhi[(nt * 16 + l16) * SP + k0 + q * M::EPL]);
                            pa[tj] = M::mma(fa, fphi, pa[tj]);
                            pb[tj] = M::mma(fbv, fphi, pb[tj]);
                        }
                    }
                }
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int nt = wc + 2 * tj;
                    if (nt >= NTK) continue;
                    const int i = nt * 16 + l16;
                    const float mA = sM[i], mB = sM[KPMAX + i];
                    f32x4 qv;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float xa = pa[tj][r], xb = pb[tj][r];
                        const float h = xa * xb;
                        colsum[tj] += h;
                        qv[r] = g.a * h - g.b * xa * mB - g.b * mA * xb;
                    }
                    M::store4(&sBuf[i * SB + mt * 16 + 4 * q], qv);
                }
            }
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                const int nt = wc + 2 * tj;
                if (nt >= NTK) continue;
                colsum[tj] += __shfl_xor(colsum[tj], 16);
                colsum[tj] += __shfl_xor(colsum[tj], 32);
                if (q == 0) sS[wr * KPMAX + nt * 16 + l16] = colsum[tj];
            }
        }
        if constexpr (M::kStageC) {
            // YC batch into LDS, a-major: sYC[a*SB + t] (zero outside the batch and k)
            for (int e = tid; e < MB * KP; e += kThreads) {
                const int tr = e / KP, a = e % KP;
                const Y v = (tr < nb && a < k) ? YC[(size_t)sIdx[tr] * ldy + a] : M::to_op(0.0f);
                sYC[a * SB + tr] = v;
            }
        }
        __syncthreads();

        // ================= phase 4: D = YC^T Q (+ rank one), update Phi
        {
            f32x4 dacc[kTR][TC];
#pragma unroll
            for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) dacc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < MB; k0 += M::KI) {
                typename M::Frag fa[kTR], fb[TC];
#pragma unroll
                for (int ti = 0; ti < kTR; ++ti) {
                    const int mt = wr + 4 * ti;
                    const int a = mt * 16 + l16;
                    if constexpr (M::kStageC) {
                        if (mt < NTK) fa[ti] = M::lds(&sYC[a * SB + k0 + q * M::EPL]);
                    } else {
                        const int tr = k0 + q;
                        fa[ti] = (mt < NTK && a < k && tr < nb) ? YC[(size_t)sIdx[tr] * ldy + a] : 0.0f;
                    }
                }
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int nt = wc + 2 * tj;
                    if (nt < NTK) fb[tj] = M::lds(&sBuf[(nt * 16 + l16) * SB + k0 + q * M::EPL]);
                }
#pragma unroll
                for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj)
                        if (wr + 4 * ti < NTK && wc + 2 * tj < NTK)
                            dacc[ti][tj] = M::mma(fa[ti], fb[tj], dacc[ti][tj]);
            }
            const float invB = 1.0f / static_cast<float>(nb);
            const bool snap = (Snap != nullptr) && (s == g.spp - 1);
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                const int nt = wc + 2 * tj;
                if (nt >= NTK) continue;
                const int i = nt * 16 + l16;
                const float ssum = sS[i] + sS[KPMAX + i] + sS[2 * KPMAX + i] + sS[3 * KPMAX + i];
                const float rv = g.c * sM[i] * sM[KPMAX + i] - g.b * ssum * invB;
#pragma unroll
                for (int ti = 0; ti < kTR; ++ti) {
                    const int mt = wr + 4 * ti;
                    if (mt >= NTK) continue;
                    f32x4 v = phi[ti][tj], cv = comp[ti][tj];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int a = mt * 16 + 4 * q + r;
                        const float d = dacc[ti][tj][r] * invB + sYbar[2 * KPMAX + a] * rv;
                        const float delta = beta * (d - g.kappa * oacc[ti][tj][r]);
                        if (g.compensated) {
                            const float y = delta - cv[r];
                            const float tt = v[r] + y;
                            cv[r] = (tt - v[r]) - y;
                            v[r] = tt;
                        } else {
                            v[r] += delta;
                        }
                        bad |= !isfinite(v[r]);
                        if (snap && a < k && i < k)
                            Snap[(size_t)pass * k * k + (size_t)i * k + a] = v[r];
                    }
                    phi[ti][tj] = v;
                    comp[ti][tj] = cv;
                    M::store4(&sPhi[i * SP + mt * 16 + 4 * q], v);
                    if constexpr (M::kPhiT) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) sPhiT[(mt * 16 + 4 * q + r) * SP + i] = M::to_op(v[r]);
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- write back the master copy (and compensation)
#pragma unroll
    for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
        for (int tj = 0; tj < TC; ++tj) {
            const int mt = wr + 4 * ti, nt = wc + 2 * tj;
            if (mt >= NTK || nt >= NTK) continue;
            const int i = nt * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = mt * 16 + 4 * q + r;
                if (a < k && i < k) {
                    Phi[(size_t)i * k + a] = phi[ti][tj][r];
                    if (Comp) Comp[(size_t)i * k + a] = g.compensated ? comp[ti][tj][r] : 0.0f;
                }
            }
        }
    if (bad && g.nonfinite) *g.nonfinite = 1;
}

template <class M, int KPMAX>
int launch_sgd(const SgdArgs& a, int restarts, hipStream_t st) {
    hipLaunchKernelGGL((sgd_kernel<M, KPMAX>), dim3(restarts), dim3(kThreads), 0, st, a);
    return check_launch("sgd_kernel");
}

int run_common(const otm_sgd_params* p, int32_t n, const void* YA, const void* YB, const void* YC,
               const float* ybar, const int32_t* perms, int64_t perm_stride, int32_t restarts,
               int64_t start_step, int64_t end_step, float* Phi, float* Phi_comp, float* snapshots,
               int32_t* nonfinite, hipStream_t st) {
    OTM_REQUIRE(p != nullptr, OTM_EINVAL, "params is NULL");
    OTM_REQUIRE(YA && YB && YC && ybar && Phi, OTM_EINVAL, "null data pointer");
    OTM_REQUIRE(p->k >= 1 && p->batch >= 1 && n >= 1 && p->passes >= 1, OTM_ESHAPE,
                "k, batch, n and passes must be positive");
    OTM_REQUIRE(p->k <= kMaxK, OTM_ECAPACITY, "k exceeds the compiled capacity (128)");
    OTM_REQUIRE(p->batch <= kMaxBatch, OTM_ECAPACITY, "batch exceeds the compiled capacity (128)");
    OTM_REQUIRE(restarts >= 1, OTM_ESHAPE, "restarts must be >= 1");
    OTM_REQUIRE(p->ldy >= p->k, OTM_ESHAPE, "ldy < k");
    OTM_REQUIRE(p->y_dtype == OTM_F32 || p->y_dtype == OTM_BF16, OTM_EDTYPE, "y_dtype must be F32 or BF16");
    OTM_REQUIRE(p->y_dtype != OTM_BF16 || p->ldy % 8 == 0, OTM_ESHAPE, "BF16 rows need ldy % 8 == 0");
    OTM_REQUIRE(p->beta_tau > 0.0, OTM_EINVAL, "beta_tau must be positive");
    OTM_REQUIRE(std::isfinite(p->beta0) && std::isfinite(p->alpha0) && std::isfinite(p->theta) && p->alpha0 >= 0.0,
                OTM_EINVAL, "alpha0, beta0, theta must be finite, alpha0 >= 0");
    SgdArgs a{};
    a.YA = YA; a.YB = YB; a.YC = YC; a.ybar = ybar; a.perms = perms; a.perm_stride = perm_stride;
    a.Phi = Phi; a.Phi_comp = Phi_comp; a.snapshots = snapshots; a.nonfinite = nonfinite;
    a.n = n; a.k = p->k; a.batch = p->batch; a.passes = p->passes; a.ldy = p->ldy;
    a.compensated = p->compensated ? 1 : 0;
    a.spp = (n + p->batch - 1) / p->batch;
    const int64_t total = a.spp * p->passes;
    a.start_step = start_step;
    a.end_step = end_step < 0 ? total : end_step;
    OTM_REQUIRE(a.start_step >= 0 && a.start_step <= a.end_step && a.end_step <= total, OTM_ESHAPE,
                "need 0 <= start_step <= end_step <= passes * ceil(n / batch)");
    const double al = p->alpha0;
    a.a = static_cast<float>((al + 1.0) * (al + 2.0) / 2.0);
    a.b = static_cast<float>(al * (al + 1.0) / 2.0);
    a.c = static_cast<float>(al * al);
    a.kappa = static_cast<float>(0.5 * (1.0 + p->theta));
    a.beta0 = p->beta0;
    a.beta_tau = p->beta_tau;
    if (a.start_step == a.end_step && !Phi_comp) return OTM_OK;
    const int k = p->k;
    if (p->y_dtype == OTM_F32) {
        const int kp = (k + 15) / 16 * 16;
        if (kp <= 32) return launch_sgd<MmaF32, 32>(a, restarts, st);
        if (kp <= 64) return launch_sgd<MmaF32, 64>(a, restarts, st);
        return launch_sgd<MmaF32, 128>(a, restarts, st);
    }
    const int kp = (k + 31) / 32 * 32;
    if (kp <= 32) return launch_sgd<MmaBF16, 32>(a, restarts, st);
    if (kp <= 64) return launch_sgd<MmaBF16, 64>(a, restarts, st);
    return launch_sgd<MmaBF16, 128>(a, restarts, st);
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
