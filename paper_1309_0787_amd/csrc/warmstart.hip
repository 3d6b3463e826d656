// Learned warm start of the stochastic updates (an addition to the paper,
// which starts them at random, Section 3.2):
//   sketch   S_r = T(I, I, theta_r), r = 1..4, from the whitened rows
//            (the tensor of Section 3.2 contracted along its third mode);
//   frame    eigenvectors Q of S_1 (FP32 Jacobi in LDS, one workgroup per
//            instance), by decreasing |eigenvalue|, oriented by the theta_r;
//   network  x = [Q^T S_r Q / sigma, Q^T theta_r] -> relu(W1 x + b1) ->
//            W2 h + b2 (P x P), trained in FP32 and run in BF16 on the
//            matrix cores;
//   factors  V0 = Q out[:k, :k] sigma^(1/3).
// The perceptron's products are one tiled matrix-core GEMM (64 x 64 tiles,
// four waves of 32 x 32, split over K when the output has few tiles, with a
// fixed-order reduction that applies bias and ReLU).
#include <algorithm>
#include <cmath>

#include "otm_internal.h"

namespace otm {
namespace {

constexpr int kP = 100;                       // largest k the network takes
constexpr int kSk = 4;                        // sketches
constexpr int kHid = 512;
constexpr int kIn = kSk * kP * kP + kSk * kP; // 40400
constexpr int kOut = kP * kP;                 // 10000
constexpr size_t kParams = (size_t)kHid * kIn + kHid + (size_t)kOut * kHid + kOut;

// ------------------------------------------------------------------ sketch
constexpr int kSkRows = 256;      // rows per partial block

// z[t][r] = yC_t . theta_r
template <class TY>
__global__ void sketch_z_kernel(const TY* __restrict__ YC, int ldy, int n, int k, const float* __restrict__ Theta,
                                float* __restrict__ z) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float acc[kSk] = {0.f, 0.f, 0.f, 0.f};
    const TY* row = YC + (size_t)t * ldy;
    for (int a = 0; a < k; ++a) {
        const float y = static_cast<float>(row[a]);
#pragma unroll
        for (int r = 0; r < kSk; ++r) acc[r] = fmaf(y, Theta[a * kSk + r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < kSk; ++r) z[(size_t)t * kSk + r] = acc[r];
}

// partial[blk][r][i][j] = sum over the block's rows of yA_i * w_r(t) * yB_j, and
// partial vectors sum yA_i z_r, sum yB_j z_r, with w_r = a z_r - b gC_r.
// One workgroup per (row block, 16 x 16 output tile); FP64 accumulation.
template <class TY>
__global__ __launch_bounds__(256) void sketch_partial_kernel(const TY* __restrict__ YA, const TY* __restrict__ YB,
                                                             int ldy, int n, int k, const float* __restrict__ z,
                                                             float a, float b, const float* __restrict__ gC,
                                                             double* __restrict__ part, double* __restrict__ vpart) {
    const int tiles = (k + 15) / 16;
    const int ti = blockIdx.y / tiles, tj = blockIdx.y % tiles;
    const int blk = blockIdx.x;
    const int t0 = blk * kSkRows, t1 = min(n, t0 + kSkRows);
    const int li = threadIdx.x >> 4, lj = threadIdx.x & 15;
    const int i = ti * 16 + li, j = tj * 16 + lj;
    __shared__ float sa[32][16], sb[32][16], sw[32][kSk], sz[32][kSk];
    double acc[kSk] = {0, 0, 0, 0};
    double va[kSk] = {0, 0, 0, 0}, vb[kSk] = {0, 0, 0, 0};
    for (int c0 = t0; c0 < t1; c0 += 32) {
        for (int e = threadIdx.x; e < 32 * 16; e += 256) {
            const int tt = e >> 4, col = e & 15;
            const int t = c0 + tt;
            const bool ok = t < t1;
            sa[tt][col] = (ok && ti * 16 + col < k) ? static_cast<float>(YA[(size_t)t * ldy + ti * 16 + col]) : 0.f;
            sb[tt][col] = (ok && tj * 16 + col < k) ? static_cast<float>(YB[(size_t)t * ldy + tj * 16 + col]) : 0.f;
        }
        if (threadIdx.x < 32 * kSk) {
            const int tt = threadIdx.x / kSk, r = threadIdx.x % kSk;
            const int t = c0 + tt;
            const float zz = t < t1 ? z[(size_t)t * kSk + r] : 0.f;
            sz[tt][r] = zz;
            sw[tt][r] = t < t1 ? a * zz - b * gC[r] : 0.f;
        }
        __syncthreads();
#pragma unroll 4
        for (int tt = 0; tt < 32; ++tt) {
            const double p = static_cast<double>(sa[tt][li]) * sb[tt][lj];
#pragma unroll
            for (int r = 0; r < kSk; ++r) acc[r] += p * sw[tt][r];
            if (tj == 0 && lj == 0) {
#pragma unroll
                for (int r = 0; r < kSk; ++r) va[r] += static_cast<double>(sa[tt][li]) * sz[tt][r];
            }
            if (ti == 0 && li == 0) {
#pragma unroll
                for (int r = 0; r < kSk; ++r) vb[r] += static_cast<double>(sb[tt][lj]) * sz[tt][r];
            }
        }
        __syncthreads();
    }
    const int nb = gridDim.x;
    if (i < k && j < k) {
#pragma unroll
        for (int r = 0; r < kSk; ++r) part[(((size_t)r * nb + blk) * k + i) * k + j] = acc[r];
    }
    // vpart[r][blk][0][i] = sum yA_i z_r, vpart[r][blk][1][j] = sum yB_j z_r
    if (tj == 0 && lj == 0 && i < k) {
#pragma unroll
        for (int r = 0; r < kSk; ++r) vpart[(((size_t)r * nb + blk) * 2 + 0) * k + i] = va[r];
    }
    if (ti == 0 && li == 0 && j < k) {
#pragma unroll
        for (int r = 0; r < kSk; ++r) vpart[(((size_t)r * nb + blk) * 2 + 1) * k + j] = vb[r];
    }
}

// S_r[i][j] = (sum_blk part)/n - b ybarA_i (sum yB_j z_r)/n - b (sum yA_i z_r)/n ybarB_j
//             + c gC_r ybarA_i ybarB_j, written to S + r*lds*lds + i*lds + j
__global__ void sketch_final_kernel(const double* __restrict__ part, const double* __restrict__ vpart, int nb, int n,
                                    int k, const float* __restrict__ ybar, float b, float c,
                                    const float* __restrict__ gC, float* __restrict__ S, int lds) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kSk * k * k) return;
    const int r = e / (k * k), i = (e / k) % k, j = e % k;
    double s = 0.0, va = 0.0, vb = 0.0;
    for (int q = 0; q < nb; ++q) {
        s += part[(((size_t)r * nb + q) * k + i) * k + j];
        va += vpart[(((size_t)r * nb + q) * 2 + 0) * k + i];
        vb += vpart[(((size_t)r * nb + q) * 2 + 1) * k + j];
    }
    const double inv = 1.0 / n;
    const double yA = ybar[i], yB = ybar[k + j];
    const double v = s * inv - b * yA * vb * inv - b * va * inv * yB + (double)c * gC[r] * yA * yB;
    S[((size_t)r * lds + i) * lds + j] = static_cast<float>(v);
}

__global__ void sketch_gc_kernel(const float* __restrict__ ybar, int k, const float* __restrict__ Theta,
                                 float* __restrict__ gC) {
    const int r = threadIdx.x;
    if (r >= kSk) return;
    double s = 0.0;
    for (int a = 0; a < k; ++a) s += (double)ybar[2 * k + a] * Theta[a * kSk + r];
    gC[r] = static_cast<float>(s);
}

// ------------------------------------------------------------------ frames
// One workgroup per instance: cyclic Jacobi on S_1 (round-robin pairs, FP32,
// A and V in LDS), eigenvalues by decreasing magnitude, frame sketches
// F_r = Q^T S_r Q, orientation, features.
constexpr int kFrameMax = 128;
constexpr int kFrameThreads = 256;
constexpr int kFrameSweeps = 15;

struct FrameSmem {
    float A[kFrameMax][kFrameMax + 1];
    float V[kFrameMax][kFrameMax + 1];
    float c[kFrameMax / 2], s[kFrameMax / 2];
    int p[kFrameMax / 2], q[kFrameMax / 2];
    int order[kFrameMax];
    float sign[kFrameMax];
    float red[kFrameThreads];
};

__global__ __launch_bounds__(kFrameThreads) void frames_kernel(const int32_t* __restrict__ ks,
                                                               const float* __restrict__ Sall,
                                                               const float* __restrict__ Thall, float* __restrict__ Qall,
                                                               float* __restrict__ sigall, float* __restrict__ Xall,
                                                               float* __restrict__ Tmp, int32_t* __restrict__ info) {
    __shared__ FrameSmem sm;
    const int inst = blockIdx.x;
    const int tid = threadIdx.x;
    const int k = ks[inst];
    const float* S = Sall + (size_t)inst * kSk * kP * kP;   // 4 x P x P
    const float* Th = Thall + (size_t)inst * kP * kSk;      // P x 4
    float* Qo = Qall + (size_t)inst * kP * kP;
    float* X = Xall + (size_t)inst * kIn;
    float* T1 = Tmp + (size_t)inst * kP * kP;
    if (k < 1 || k > kP) {   // outside the network's range: zero features, identity frame
        for (int e = tid; e < kIn; e += kFrameThreads) X[e] = 0.f;
        for (int e = tid; e < kP * kP; e += kFrameThreads) Qo[e] = (e / kP == e % kP) ? 1.f : 0.f;
        if (tid == 0) {
            sigall[inst] = 0.f;
            info[inst] = -2;
        }
        return;
    }
    // sigma = sqrt(mean_r ||S_r||_F^2)
    float acc = 0.f;
    for (int e = tid; e < kSk * k * k; e += kFrameThreads) {
        const int r = e / (k * k), i = (e / k) % k, j = e % k;
        const float v = S[((size_t)r * kP + i) * kP + j];
        acc = fmaf(v, v, acc);
    }
    sm.red[tid] = acc;
    __syncthreads();
    for (int h = kFrameThreads / 2; h > 0; h >>= 1) {
        if (tid < h) sm.red[tid] += sm.red[tid + h];
        __syncthreads();
    }
    const float sigma = sqrtf(sm.red[0] / kSk);
    __syncthreads();
    // A = sym(S_1), V = I, padded to an even size m with a zero row/column
    const int m = (k + 1) & ~1;
    for (int e = tid; e < m * m; e += kFrameThreads) {
        const int i = e / m, j = e % m;
        sm.A[i][j] = (i < k && j < k) ? 0.5f * (S[(size_t)i * kP + j] + S[(size_t)j * kP + i]) : 0.f;
        sm.V[i][j] = (i == j) ? 1.f : 0.f;
    }
    __syncthreads();
    int sweeps = -1;
    for (int sw = 0; sw < kFrameSweeps; ++sw) {
        // off-diagonal and total Frobenius norms
        float off = 0.f, tot = 0.f;
        for (int e = tid; e < m * m; e += kFrameThreads) {
            const int i = e / m, j = e % m;
            const float v = sm.A[i][j] * sm.A[i][j];
            tot += v;
            if (i != j) off += v;
        }
        sm.red[tid] = off;
        __syncthreads();
        for (int h = kFrameThreads / 2; h > 0; h >>= 1) {
            if (tid < h) sm.red[tid] += sm.red[tid + h];
            __syncthreads();
        }
        const float offn = sm.red[0];
        __syncthreads();
        sm.red[tid] = tot;
        __syncthreads();
        for (int h = kFrameThreads / 2; h > 0; h >>= 1) {
            if (tid < h) sm.red[tid] += sm.red[tid + h];
            __syncthreads();
        }
        const float totn = sm.red[0];
        __syncthreads();
        if (offn <= 1e-12f * totn || totn == 0.f) {
            sweeps = sw;
            break;
        }
        for (int round = 0; round < m - 1; ++round) {
            // round-robin pairs: position 0 fixed, the others rotate
            if (tid < m / 2) {
                auto pos = [&](int x) { return x == 0 ? 0 : 1 + (x - 1 + round) % (m - 1); };
                int p = pos(tid), q = pos(m - 1 - tid);
                if (p > q) { const int t = p; p = q; q = t; }
                const float app = sm.A[p][p], aqq = sm.A[q][q], apq = sm.A[p][q];
                float c = 1.f, s = 0.f;
                if (fabsf(apq) > 1e-30f) {
                    const float th = (aqq - app) / (2.f * apq);
                    const float t = (th >= 0.f ? 1.f : -1.f) / (fabsf(th) + sqrtf(th * th + 1.f));
                    c = 1.f / sqrtf(t * t + 1.f);
                    s = t * c;
                }
                sm.c[tid] = c;
                sm.s[tid] = s;
                sm.p[tid] = p;
                sm.q[tid] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int e = tid; e < (m / 2) * m; e += kFrameThreads) {
                const int w = e / m, j = e % m;
                const int p = sm.p[w], q = sm.q[w];
                const float c = sm.c[w], s = sm.s[w];
                const float ap = sm.A[p][j], aq = sm.A[q][j];
                sm.A[p][j] = c * ap - s * aq;
                sm.A[q][j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int e = tid; e < (m / 2) * m; e += kFrameThreads) {
                const int w = e / m, i = e % m;
                const int p = sm.p[w], q = sm.q[w];
                const float c = sm.c[w], s = sm.s[w];
                const float ap = sm.A[i][p], aq = sm.A[i][q];
                sm.A[i][p] = c * ap - s * aq;
                sm.A[i][q] = s * ap + c * aq;
                const float vp = sm.V[i][p], vq = sm.V[i][q];
                sm.V[i][p] = c * vp - s * vq;
                sm.V[i][q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    // order: rank of |eigenvalue| (descending, ties to the lower index); the
    // padding column (index k when k is odd) is excluded
    for (int i = tid; i < k; i += kFrameThreads) {
        const float ei = fabsf(sm.A[i][i]);
        int rank = 0;
        for (int j = 0; j < k; ++j) {
            const float ej = fabsf(sm.A[j][j]);
            rank += (ej > ei) || (ej == ei && j < i);
        }
        sm.order[rank] = i;
    }
    __syncthreads();
    // T1 = S_r Q for each r, then F_r = Q^T T1 (Q column l = V[:, order[l]])
    for (int r = 0; r < kSk; ++r) {
        const float* Sr = S + (size_t)r * kP * kP;
        for (int e = tid; e < k * k; e += kFrameThreads) {
            const int i = e / k, l = e % k;
            const int col = sm.order[l];
            float acc2 = 0.f;
            for (int a = 0; a < k; ++a) acc2 = fmaf(Sr[(size_t)i * kP + a], sm.V[a][col], acc2);
            T1[(size_t)i * kP + l] = acc2;
        }
        __syncthreads();
        for (int e = tid; e < k * k; e += kFrameThreads) {
            const int l = e / k, j = e % k;
            const int col = sm.order[l];
            float acc2 = 0.f;
            for (int a = 0; a < k; ++a) acc2 = fmaf(sm.V[a][col], T1[(size_t)a * kP + j], acc2);
            X[(size_t)r * kP * kP + (size_t)l * kP + j] = acc2 / sigma;   // unsigned for now
        }
        __syncthreads();
    }
    // orientation: r* = argmax_r |q_l . theta_r| (ties: lowest r); flip if
    // (q_l . theta_r*) and (q_l^T S_r* q_l) have opposite signs
    for (int l = tid; l < k; l += kFrameThreads) {
        const int col = sm.order[l];
        float qt[kSk];
#pragma unroll
        for (int r = 0; r < kSk; ++r) {
            float d = 0.f;
            for (int a = 0; a < k; ++a) d = fmaf(sm.V[a][col], Th[a * kSk + r], d);
            qt[r] = d;
        }
        int rs = 0;
#pragma unroll
        for (int r = 1; r < kSk; ++r)
            if (fabsf(qt[r]) > fabsf(qt[rs])) rs = r;
        const float mu = X[(size_t)rs * kP * kP + (size_t)l * kP + l];
        const float sg = (qt[rs] * mu < 0.f) ? -1.f : 1.f;
        sm.sign[l] = sg;
#pragma unroll
        for (int r = 0; r < kSk; ++r) X[(size_t)kSk * kP * kP + r * kP + l] = sg * qt[r];
    }
    __syncthreads();
    // signs into the frame sketches (d_l d_j), zero padding, Q out
    for (int e = tid; e < kSk * kP * kP; e += kFrameThreads) {
        const int l = (e / kP) % kP, j = e % kP;
        X[e] = (l < k && j < k) ? X[e] * sm.sign[l] * sm.sign[j] : 0.f;
    }
    for (int e = tid; e < kSk * kP; e += kFrameThreads)
        if (e % kP >= k) X[(size_t)kSk * kP * kP + e] = 0.f;
    for (int e = tid; e < kP * kP; e += kFrameThreads) {
        const int a = e / kP, l = e % kP;
        Qo[e] = (a < k && l < k) ? sm.V[a][sm.order[l]] * sm.sign[l] : 0.f;
    }
    if (tid == 0) {
        sigall[inst] = sigma;
        info[inst] = sweeps;
    }
}

// ------------------------------------------------------------------ target
// Per instance: C = Q^T U (frame vectors against planted directions), greedy
// matching by decreasing |C| (ties: lower row, then lower column), target
// column l = lambda_perm[l]^(1/3) C[:, perm[l]] / sigma^(1/3).
__global__ __launch_bounds__(256) void target_kernel(const int32_t* __restrict__ ks, const float* __restrict__ Qall,
                                                     const float* __restrict__ sigall, const float* __restrict__ Uall,
                                                     const float* __restrict__ lamall, float* __restrict__ tgt) {
    __shared__ float C[kP][kP + 1];
    __shared__ int perm[kP];
    __shared__ unsigned char used_r[kP], used_c[kP];
    __shared__ float bv[256];
    __shared__ int bi[256];
    const int inst = blockIdx.x, tid = threadIdx.x;
    const int k = ks[inst];
    float* out = tgt + (size_t)inst * kOut;
    for (int e = tid; e < kOut; e += 256) out[e] = 0.f;
    if (k < 1 || k > kP) return;
    const float* Q = Qall + (size_t)inst * kP * kP;
    const float* U = Uall + (size_t)inst * kP * kP;
    for (int e = tid; e < k * k; e += 256) {
        const int l = e / k, j = e % k;
        float acc = 0.f;
        for (int a = 0; a < k; ++a) acc = fmaf(Q[(size_t)a * kP + l], U[(size_t)a * kP + j], acc);
        C[l][j] = acc;
    }
    for (int e = tid; e < k; e += 256) used_r[e] = used_c[e] = 0;
    __syncthreads();
    for (int round = 0; round < k; ++round) {
        float best = -1.f;
        int bidx = 0x7fffffff;
        for (int e = tid; e < k * k; e += 256) {
            const int l = e / k, j = e % k;
            if (used_r[l] || used_c[j]) continue;
            const float v = fabsf(C[l][j]);
            if (v > best || (v == best && e < bidx)) {   // row-major index order = lower row, then lower column
                best = v;
                bidx = e;
            }
        }
        bv[tid] = best;
        bi[tid] = bidx;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) {
                const float v2 = bv[tid + h];
                const int i2 = bi[tid + h];
                if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) {
                    bv[tid] = v2;
                    bi[tid] = i2;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            const int l = bi[0] / k, j = bi[0] % k;
            perm[l] = j;
            used_r[l] = 1;
            used_c[j] = 1;
        }
        __syncthreads();
    }
    const float sc = 1.f / cbrtf(sigall[inst]);
    for (int e = tid; e < k * k; e += 256) {
        const int a = e / k, l = e % k;
        const int j = perm[l];
        out[(size_t)a * kP + l] = cbrtf(lamall[(size_t)inst * kP + j]) * C[a][j] * sc;
    }
}

// ------------------------------------------------------------------ GEMM
// C (M x N, row-major, ldc) = op(A) op(B) where op(A) is M x K and op(B) is
// K x N; TA: A is stored K x M (lda), else M x K; TB: B is stored N x K (ldb),
// else K x N.  Matrix cores: FP32 (16x16x4) or BF16 (16x16x32, FP32
// accumulation).  Tile 64 x 64 x 32, four waves of 32 x 32.  With splits > 1,
// blockIdx.z takes K range [z*kc, (z+1)*kc) and writes its partial tile to
// part + z*M*N (row-major M x N); else the epilogue writes C (+ bias[n],
// ReLU) directly.
template <class T>
struct MmaT;
template <>
struct MmaT<float> {
    static constexpr int EPL = 1;
    using Frag = float;
    __device__ static f32x4 mma(Frag a, Frag b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static Frag frag(const float* p) { return *p; }
    static constexpr int KI = 4;
};
template <>
struct MmaT<__bf16> {
    static constexpr int EPL = 8;
    using Frag = bf16x8;
    __device__ static f32x4 mma(Frag a, Frag b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
    __device__ static Frag frag(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
    static constexpr int KI = 32;
};

constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

template <class T, bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_kernel(const T* __restrict__ A, int lda, const T* __restrict__ B, int ldb,
                                                   float* __restrict__ C, int ldc, int M, int N, int K, int kc,
                                                   const float* __restrict__ bias, int relu, float* __restrict__ part) {
    using MT = MmaT<T>;
    __shared__ __attribute__((aligned(16))) T As[GBM][GBK + GPAD];
    __shared__ __attribute__((aligned(16))) T Bs[GBN][GBK + GPAD];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6) & 3;
    const int wm = w >> 1, wn = w & 1;
    const int l16 = lane & 15, qd = lane >> 4;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const T zero = static_cast<T>(0.0f);
    for (int k0 = kb; k0 < ke; k0 += GBK) {
        // A tile: As[m][kk] = op(A)[m0+m][k0+kk]
        for (int e = tid; e < GBM * GBK; e += 256) {
            int m, kk;
            if (TA) { kk = e / GBM; m = e % GBM; }    // stored K x M: contiguous in m
            else { m = e / GBK; kk = e % GBK; }       // stored M x K: contiguous in k
            const int gm = m0 + m, gk = k0 + kk;
            T v = zero;
            if (gm < M && gk < ke) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            As[m][kk] = v;
        }
        // B tile: Bs[n][kk] = op(B)[k0+kk][n0+n]
        for (int e = tid; e < GBN * GBK; e += 256) {
            int nn, kk;
            if (TB) { nn = e / GBK; kk = e % GBK; }   // stored N x K: contiguous in k
            else { kk = e / GBN; nn = e % GBN; }      // stored K x N: contiguous in n
            const int gn = n0 + nn, gk = k0 + kk;
            T v = zero;
            if (gn < N && gk < ke) v = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
            Bs[nn][kk] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; kk += MT::KI) {
            typename MT::Frag fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) fa[i] = MT::frag(&As[wm * 32 + i * 16 + l16][kk + qd * MT::EPL]);
#pragma unroll
            for (int j = 0; j < 2; ++j) fb[j] = MT::frag(&Bs[wn * 32 + j * 16 + l16][kk + qd * MT::EPL]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = MT::mma(fa[i], fb[j], acc[i][j]);
        }
        __syncthreads();
    }
    // lane holds rows 4*qd + r of column l16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * 32 + i * 16 + 4 * qd + r;
                const int gn = n0 + wn * 32 + j * 16 + l16;
                if (gm >= M || gn >= N) continue;
                float v = acc[i][j][r];
                if (part != nullptr) {
                    part[((size_t)blockIdx.z * M + gm) * N + gn] = v;
                } else {
                    if (bias) v += bias[gn];
                    if (relu) v = fmaxf(v, 0.f);
                    C[(size_t)gm * ldc + gn] = v;
                }
            }
}

// C = sum_z part[z] (fixed order) + bias, then ReLU, or times the ReLU mask of H
__global__ void split_reduce_kernel(const float* __restrict__ part, int splits, int M, int N, float* __restrict__ C,
                                    int ldc, const float* __restrict__ bias, int relu, const float* __restrict__ mask,
                                    int ldm) {
    const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (e >= (size_t)M * N) return;
    const int m = e / N, n = e % N;
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += part[(size_t)z * M * N + e];
    if (bias) v += bias[n];
    if (relu) v = fmaxf(v, 0.f);
    if (mask) v = mask[(size_t)m * ldm + n] > 0.f ? v : 0.f;
    C[(size_t)m * ldc + n] = v;
}

constexpr int kMaxSplits = 64;

// partial tiles of the perceptron's products for a batch: the split over K
// is at most kMaxSplits, and at most 2 when the output has kOut columns
size_t gemm_ws_bytes(int batch) {
    return ws_round(sizeof(float) * (size_t)batch * std::max((size_t)kMaxSplits * kHid, (size_t)4 * kOut));
}

// picks the split over K so that the grid has at least ~1024 workgroups
template <class T, bool TA, bool TB>
int gemm(const T* A, int lda, const T* B, int ldb, float* C, int ldc, int M, int N, int K, const float* bias, int relu,
         const float* mask, int ldm, float* ws, size_t ws_bytes, hipStream_t st) {
    const int tiles = ((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
    int splits = 1;
    while (splits < kMaxSplits && tiles * splits < 1024 && K / (splits * 2) >= 4 * GBK) splits *= 2;
    const int kc = ((K + splits - 1) / splits + GBK - 1) / GBK * GBK;
    splits = (K + kc - 1) / kc;
    dim3 grid((N + GBN - 1) / GBN, (M + GBM - 1) / GBM, splits);
    if (splits == 1 && mask == nullptr) {   // a mask is applied by the reduction
        hipLaunchKernelGGL((gemm_kernel<T, TA, TB>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, kc, bias,
                           relu, static_cast<float*>(nullptr));
        return check_launch("gemm_kernel");
    }
    OTM_REQUIRE(ws != nullptr && ws_bytes >= sizeof(float) * (size_t)splits * M * N, OTM_EWORKSPACE,
                "GEMM workspace too small");
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, kc,
                       static_cast<const float*>(nullptr), 0, ws);
    int s = check_launch("gemm_kernel");
    if (s != OTM_OK) return s;
    const size_t tot = (size_t)M * N;
    hipLaunchKernelGGL(split_reduce_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, ws, splits, M, N, C, ldc, bias,
                       relu, mask, ldm);
    return check_launch("split_reduce_kernel");
}

// column sums of a batch x N matrix (fixed order)
__global__ void colsum_kernel(const float* __restrict__ X, int rows, int N, float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += X[(size_t)r * N + n];
    out[n] = s;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, size_t count, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, __bf16* __restrict__ y, size_t count) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        y[e] = f32_to_bf16(x[e]);
}

// per instance: squared error over the live k x k block (FP64 partial), and
// dout = 2 (out - target) mask / count
__global__ void mse_kernel(const int32_t* __restrict__ ks, int count, const float* __restrict__ out,
                           const float* __restrict__ tgt, double inv_cnt, float* __restrict__ dout,
                           double* __restrict__ per) {
    __shared__ double red[256];
    const int inst = blockIdx.x, tid = threadIdx.x;
    const int k = ks[inst];
    double s = 0.0;
    for (int e = tid; e < kOut; e += 256) {
        const int i = e / kP, j = e % kP;
        const bool live = i < k && j < k;
        const size_t idx = (size_t)inst * kOut + e;
        const float d = live ? out[idx] - tgt[idx] : 0.f;
        s += (double)d * d;
        dout[idx] = static_cast<float>(2.0 * d * inv_cnt);
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) per[inst] = red[0];
}

__global__ void sum_loss_kernel(const double* __restrict__ per, int count, double inv_cnt, double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < count; ++i) s += per[i];
    *loss = s * inv_cnt;
}

// Phi (instance i at Phi + i*P*P, phi_j contiguous, length k) = rows of
// (Q out[:k, :k] sigma^(1/3))^T
__global__ void factors_kernel(const int32_t* __restrict__ ks, const float* __restrict__ out,
                               const float* __restrict__ Qall, const float* __restrict__ sigall,
                               float* __restrict__ Phi) {
    const int inst = blockIdx.x;
    const int k = ks[inst];
    if (k < 1 || k > kP) return;
    const float* O = out + (size_t)inst * kOut;
    const float* Q = Qall + (size_t)inst * kP * kP;
    const float sc = cbrtf(sigall[inst]);
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int j = e / k, a = e % k;   // phi_j[a] = sum_l Q[a][l] O[l][j]
        float acc = 0.f;
        for (int l = 0; l < k; ++l) acc = fmaf(Q[(size_t)a * kP + l], O[(size_t)l * kP + j], acc);
        Phi[(size_t)inst * kP * kP + (size_t)j * k + a] = acc * sc;
    }
}

// parameter blocks inside the flat buffer
struct ParamView {
    size_t w1, b1, w2, b2;
};
constexpr ParamView kView{0, (size_t)kHid * kIn, (size_t)kHid * kIn + kHid, (size_t)kHid * kIn + kHid + (size_t)kOut * kHid};

}  // namespace
}  // namespace otm

using namespace otm;

extern "C" int otm_ws_dims(int32_t* n_in, int32_t* n_hidden, int32_t* n_out, int32_t* p, int64_t* n_params) {
    OTM_REQUIRE(n_in && n_hidden && n_out && p && n_params, OTM_EINVAL, "null argument");
    *n_in = kIn;
    *n_hidden = kHid;
    *n_out = kOut;
    *p = kP;
    *n_params = static_cast<int64_t>(kParams);
    return OTM_OK;
}

extern "C" size_t otm_ws_sketch_workspace(int32_t n, int32_t k) {
    if (n < 1 || k < 1) return 0;
    const size_t nb = (n + kSkRows - 1) / kSkRows;
    return ws_round(sizeof(float) * (size_t)n * kSk) + ws_round(sizeof(double) * kSk * nb * k * k) +
           ws_round(sizeof(double) * kSk * nb * 2 * k) + ws_round(sizeof(float) * kSk);
}

extern "C" int otm_ws_sketch(const void* YA, const void* YB, const void* YC, int y_dtype, int32_t ldy, int32_t n,
                             int32_t k, const float* ybar, double alpha0, const float* Theta, float* S, int32_t lds,
                             void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(YA && YB && YC && ybar && Theta && S, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(n >= 1 && k >= 1 && k <= kMaxK && ldy >= k && lds >= k, OTM_ESHAPE, "need n >= 1, 1 <= k <= 128, ldy >= k, lds >= k");
    OTM_REQUIRE(y_dtype == OTM_F32 || y_dtype == OTM_BF16, OTM_EDTYPE, "rows must be F32 or BF16");
    OTM_REQUIRE(std::isfinite(alpha0) && alpha0 >= 0.0, OTM_EINVAL, "alpha0 must be finite and >= 0");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_ws_sketch_workspace(n, k), OTM_EWORKSPACE, "sketch workspace too small");
    hipStream_t st = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    const int nb = (n + kSkRows - 1) / kSkRows;
    float* z = wc.take<float>((size_t)n * kSk);
    double* part = wc.take<double>((size_t)kSk * nb * k * k);
    double* vpart = wc.take<double>((size_t)kSk * nb * 2 * k);
    float* gC = wc.take<float>(kSk);
    const float a = static_cast<float>((alpha0 + 1.0) * (alpha0 + 2.0) / 2.0);
    const float b = static_cast<float>(alpha0 * (alpha0 + 1.0) / 2.0);
    const float c = static_cast<float>(alpha0 * alpha0);
    hipLaunchKernelGGL(sketch_gc_kernel, dim3(1), dim3(64), 0, st, ybar, k, Theta, gC);
    int s = check_launch("sketch_gc_kernel");
    if (s != OTM_OK) return s;
    const int tiles = (k + 15) / 16;
    if (y_dtype == OTM_F32) {
        hipLaunchKernelGGL(sketch_z_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, st,
                           static_cast<const float*>(YC), ldy, n, k, Theta, z);
        if ((s = check_launch("sketch_z_kernel")) != OTM_OK) return s;
        hipLaunchKernelGGL(sketch_partial_kernel<float>, dim3(nb, tiles * tiles), dim3(256), 0, st,
                           static_cast<const float*>(YA), static_cast<const float*>(YB), ldy, n, k, z, a, b, gC, part,
                           vpart);
    } else {
        hipLaunchKernelGGL(sketch_z_kernel<__bf16>, dim3((n + 255) / 256), dim3(256), 0, st,
                           static_cast<const __bf16*>(YC), ldy, n, k, Theta, z);
        if ((s = check_launch("sketch_z_kernel")) != OTM_OK) return s;
        hipLaunchKernelGGL(sketch_partial_kernel<__bf16>, dim3(nb, tiles * tiles), dim3(256), 0, st,
                           static_cast<const __bf16*>(YA), static_cast<const __bf16*>(YB), ldy, n, k, z, a, b, gC,
                           part, vpart);
    }
    if ((s = check_launch("sketch_partial_kernel")) != OTM_OK) return s;
    const int tot = kSk * k * k;
    hipLaunchKernelGGL(sketch_final_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, part, vpart, nb, n, k, ybar, b,
                       c, gC, S, lds);
    return check_launch("sketch_final_kernel");
}

extern "C" size_t otm_ws_frames_workspace(int32_t count) {
    if (count < 1) return 0;
    return ws_round(sizeof(float) * (size_t)count * kP * kP);
}

extern "C" int otm_ws_frames(int32_t count, const int32_t* ks, const float* S, const float* Theta, float* Q,
                             float* sigma, float* X, int32_t* info, void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(ks && S && Theta && Q && sigma && X && info, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(count >= 1, OTM_ESHAPE, "count must be >= 1");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_ws_frames_workspace(count), OTM_EWORKSPACE, "frames workspace too small");
    hipLaunchKernelGGL(frames_kernel, dim3(count), dim3(kFrameThreads), 0, as_stream(stream), ks, S, Theta, Q, sigma,
                       X, static_cast<float*>(ws), info);
    return check_launch("frames_kernel");
}

extern "C" int otm_ws_target(int32_t count, const int32_t* ks, const float* Q, const float* sigma, const float* U,
                             const float* lam, float* target, otm_stream stream) {
    OTM_REQUIRE(ks && Q && sigma && U && lam && target, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(count >= 1, OTM_ESHAPE, "count must be >= 1");
    hipLaunchKernelGGL(target_kernel, dim3(count), dim3(256), 0, as_stream(stream), ks, Q, sigma, U, lam, target);
    return check_launch("target_kernel");
}

extern "C" size_t otm_mlp_workspace(int32_t batch) {
    if (batch < 1) return 0;
    return gemm_ws_bytes(batch) + ws_round(sizeof(float) * (size_t)batch * kHid);
}

extern "C" int otm_mlp_forward(const float* params, int32_t batch, const float* X, float* H, float* out, void* ws,
                               size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(params && X && H && out, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(batch >= 1, OTM_ESHAPE, "batch must be >= 1");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_mlp_workspace(batch), OTM_EWORKSPACE, "perceptron workspace too small");
    hipStream_t st = as_stream(stream);
    float* part = static_cast<float*>(ws);
    const size_t pb = gemm_ws_bytes(batch);
    // Z = X W1^T + b1, H = relu(Z);  out = H W2^T + b2
    int s = gemm<float, false, true>(X, kIn, params + kView.w1, kIn, H, kHid, batch, kHid, kIn, params + kView.b1, 1,
                                     nullptr, 0, part, pb, st);
    if (s != OTM_OK) return s;
    return gemm<float, false, true>(H, kHid, params + kView.w2, kHid, out, kOut, batch, kOut, kHid, params + kView.b2, 0,
                                    nullptr, 0, part, pb, st);
}

extern "C" int otm_mlp_backward(const float* params, int32_t batch, const float* X, const float* H, const float* dout,
                                float* grads, void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(params && X && H && dout && grads, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(batch >= 1, OTM_ESHAPE, "batch must be >= 1");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_mlp_workspace(batch), OTM_EWORKSPACE, "perceptron workspace too small");
    hipStream_t st = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    const size_t pb = gemm_ws_bytes(batch);
    float* part = wc.take<float>(pb / sizeof(float));
    float* dZ = wc.take<float>((size_t)batch * kHid);
    // gW2 = dout^T H (out x hidden), gb2 = colsum(dout)
    int s = gemm<float, true, false>(dout, kOut, H, kHid, grads + kView.w2, kHid, kOut, kHid, batch, nullptr, 0,
                                     nullptr, 0, part, pb, st);
    if (s != OTM_OK) return s;
    hipLaunchKernelGGL(colsum_kernel, dim3((kOut + 255) / 256), dim3(256), 0, st, dout, batch, kOut, grads + kView.b2);
    if ((s = check_launch("colsum_kernel")) != OTM_OK) return s;
    // dZ = (dout W2) * (H > 0)
    if ((s = gemm<float, false, false>(dout, kOut, params + kView.w2, kHid, dZ, kHid, batch, kHid, kOut, nullptr, 0, H,
                                       kHid, part, pb, st)) != OTM_OK)
        return s;
    // gW1 = dZ^T X (hidden x in), gb1 = colsum(dZ)
    if ((s = gemm<float, true, false>(dZ, kHid, X, kIn, grads + kView.w1, kIn, kHid, kIn, batch, nullptr, 0, nullptr, 0,
                                      part, pb, st)) != OTM_OK)
        return s;
    hipLaunchKernelGGL(colsum_kernel, dim3((kHid + 255) / 256), dim3(256), 0, st, dZ, batch, kHid, grads + kView.b1);
    return check_launch("colsum_kernel");
}

extern "C" int otm_mlp_adam(float* params, const float* grads, float* m, float* v, int32_t t, double lr, double beta1,
                            double beta2, double eps, otm_stream stream) {
    OTM_REQUIRE(params && grads && m && v, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(t >= 1, OTM_EINVAL, "step t must be >= 1");
    const float c1 = static_cast<float>(1.0 - std::pow(beta1, t)), c2 = static_cast<float>(1.0 - std::pow(beta2, t));
    hipLaunchKernelGGL(adam_kernel, dim3(2048), dim3(256), 0, as_stream(stream), params, grads, m, v, kParams,
                       static_cast<float>(lr), static_cast<float>(beta1), static_cast<float>(beta2),
                       static_cast<float>(eps), c1, c2);
    return check_launch("adam_kernel");
}

extern "C" int otm_mlp_to_bf16(const float* params, void* params_bf16, otm_stream stream) {
    OTM_REQUIRE(params && params_bf16, OTM_EINVAL, "null pointer argument");
    hipLaunchKernelGGL(to_bf16_kernel, dim3(2048), dim3(256), 0, as_stream(stream), params,
                       static_cast<__bf16*>(params_bf16), kParams);
    return check_launch("to_bf16_kernel");
}

extern "C" size_t otm_mlp_bf16_workspace(int32_t batch) {
    if (batch < 1) return 0;
    return gemm_ws_bytes(batch) + ws_round(sizeof(__bf16) * (size_t)batch * kIn) +
           ws_round(sizeof(float) * (size_t)batch * kHid) + ws_round(sizeof(__bf16) * (size_t)batch * kHid);
}

extern "C" int otm_mlp_forward_bf16(const void* params_bf16, const float* bias_f32, int32_t batch, const float* X,
                                    float* out, void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(params_bf16 && bias_f32 && X && out, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(batch >= 1, OTM_ESHAPE, "batch must be >= 1");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_mlp_bf16_workspace(batch), OTM_EWORKSPACE,
                "BF16 perceptron workspace too small");
    hipStream_t st = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    const size_t pb = gemm_ws_bytes(batch);
    float* part = wc.take<float>(pb / sizeof(float));
    __bf16* Xb = wc.take<__bf16>((size_t)batch * kIn);
    float* H = wc.take<float>((size_t)batch * kHid);
    __bf16* Hb = wc.take<__bf16>((size_t)batch * kHid);
    const __bf16* P = static_cast<const __bf16*>(params_bf16);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(256), dim3(256), 0, st, X, Xb, (size_t)batch * kIn);
    int s = check_launch("to_bf16_kernel");
    if (s != OTM_OK) return s;
    if ((s = gemm<__bf16, false, true>(Xb, kIn, P + kView.w1, kIn, H, kHid, batch, kHid, kIn, bias_f32 + kView.b1, 1,
                                       nullptr, 0, part, pb, st)) != OTM_OK)
        return s;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(64), dim3(256), 0, st, H, Hb, (size_t)batch * kHid);
    if ((s = check_launch("to_bf16_kernel")) != OTM_OK) return s;
    return gemm<__bf16, false, true>(Hb, kHid, P + kView.w2, kHid, out, kOut, batch, kOut, kHid, bias_f32 + kView.b2, 0,
                                     nullptr, 0, part, pb, st);
}

extern "C" size_t otm_ws_mse_workspace(int32_t count) { return count < 1 ? 0 : ws_round(sizeof(double) * count); }

extern "C" int otm_ws_mse(int32_t count, const int32_t* ks, int64_t live, const float* out, const float* target,
                          double* loss, float* dout, void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(ks && out && target && loss && dout, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(count >= 1 && live >= 1, OTM_ESHAPE, "count and live must be >= 1");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_ws_mse_workspace(count), OTM_EWORKSPACE, "loss workspace too small");
    hipStream_t st = as_stream(stream);
    const double inv = 1.0 / static_cast<double>(live);
    hipLaunchKernelGGL(mse_kernel, dim3(count), dim3(256), 0, st, ks, count, out, target, inv, dout,
                       static_cast<double*>(ws));
    int s = check_launch("mse_kernel");
    if (s != OTM_OK) return s;
    hipLaunchKernelGGL(sum_loss_kernel, dim3(1), dim3(64), 0, st, static_cast<const double*>(ws), count, inv, loss);
    return check_launch("sum_loss_kernel");
}

extern "C" int otm_ws_factors(int32_t count, const int32_t* ks, const float* out, const float* Q, const float* sigma,
                              float* Phi, otm_stream stream) {
    OTM_REQUIRE(ks && out && Q && sigma && Phi, OTM_EINVAL, "null pointer argument");
    OTM_REQUIRE(count >= 1, OTM_ESHAPE, "count must be >= 1");
    hipLaunchKernelGGL(factors_kernel, dim3(count), dim3(256), 0, as_stream(stream), ks, out, Q, sigma, Phi);
    return check_launch("factors_kernel");
}
