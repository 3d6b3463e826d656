// Symmetric eigensolver (FP64) for the small matrices of the whitening step:
// the projected moment Omega (k_tilde x k_tilde), the Gram of B (k x k) and
// the Gram of a sketch (m x m), all at most 256 x 256.
//
// Cyclic two-sided Jacobi in one workgroup.  Rounds follow the round-robin
// tournament order, so each round applies n/2 disjoint rotations at once:
// every 2x2 block (rows of pair P, columns of pair Q) becomes R_P^T X R_Q with
// R = [[c, s], [-s, c]].  A pair is rotated only while
// |a_pq| > 1e-15 sqrt(|a_pp a_qq|) and |a_pq| > 1e-15 ||A||_F; the sweeps
// stop once no pair passes that test (checked for all pairs at once after
// each sweep, so the last, rotation-free sweep is not run; at most 60).
//
// n <= 200: the matrix lives in LDS as a packed upper triangle (20100
// doubles), so a round never leaves the CU, and every round's rotations are
// written to a log.  A second kernel replays the log onto the rows of the
// eigenvector matrix, a few rows per workgroup held in LDS, all workgroups in
// parallel.  200 < n <= 256 uses the same rotations on a matrix in global
// memory and accumulates the eigenvectors as it goes.
#include <cmath>

#include "otm_internal.h"

namespace otm {
namespace {

constexpr int kJacThreads = 1024;
constexpr int kJacMaxN = 256;
constexpr int kJacLdsN = 200;
constexpr int kJacMaxSweeps = 60;

__device__ __forceinline__ int rr_player(int pos, int round, int N) {
    if (pos == 0) return 0;
    return 1 + (pos - 1 + round) % (N - 1);
}

__device__ __forceinline__ int tri_idx(int i, int j, int n) {
    if (i > j) { const int t = i; i = j; j = t; }
    return i * n - (i * (i - 1)) / 2 + (j - i);
}

struct Rot {
    double c, s;
};

// a pair slot of the current round: its players p < q and the offsets of
// their rows in the packed triangle (element (i, j), i <= j, at roff(i) + j)
struct alignas(8) PairSlot {
    short p, q, rp, rq;
};

__device__ __forceinline__ int roff(int i, int n) { return i * n - (i * (i - 1)) / 2 - i; }

// ------------------------------------------------------------------ LDS form
// log_rot[round * npairs + slot], log_pq[round * npairs + slot] = p | q << 16;
// *rounds = number of rounds performed.
__global__ __launch_bounds__(kJacThreads) void jacobi_lds_kernel(const double* __restrict__ Ain, int n,
                                                                 double* __restrict__ evals, int* __restrict__ order,
                                                                 Rot* __restrict__ log_rot, int* __restrict__ log_pq,
                                                                 int* __restrict__ rounds) {
    __shared__ double sA[kJacLdsN * (kJacLdsN + 1) / 2];
    __shared__ Rot srot[kJacLdsN / 2];
    __shared__ PairSlot spq[kJacLdsN / 2];
    __shared__ double s_red[kJacThreads / 64];
    __shared__ int s_rotated;
    const int tid = threadIdx.x;
    const int N = (n + 1) & ~1;
    const int npairs = N / 2;
    double f = 0.0;
    for (int e = tid; e < n * n; e += kJacThreads) {
        const int i = e / n, j = e % n;
        const double a = Ain[e];
        f += a * a;
        if (i <= j) sA[tri_idx(i, j, n)] = a;
    }
    for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
    if ((tid & 63) == 0) s_red[tid >> 6] = f;
    __syncthreads();
    double fro = 0.0;
    for (int w = 0; w < kJacThreads / 64; ++w) fro += s_red[w];
    const double abs_tol = 1e-15 * sqrt(fro);
    // static list of this thread's off-diagonal blocks (pair slots P < Q);
    // the diagonal block of a pair is rotated by the thread that computes
    // its rotation
    constexpr int kBlk = 5;   // 100 * 99 / 2 <= 5 * 1024
    int blkP[kBlk], blkQ[kBlk];
    const int nblk = npairs * (npairs - 1) / 2;
#pragma unroll
    for (int j = 0; j < kBlk; ++j) {
        int e = tid + j * kJacThreads, P = -1, Q = -1;
        if (e < nblk) {
            P = 0;
            while (e >= npairs - 1 - P) { e -= npairs - 1 - P; ++P; }
            Q = P + 1 + e;
        }
        blkP[j] = P;
        blkQ[j] = Q;
    }
    const bool odd = (n & 1) != 0;   // one player per round is the dummy index n
    int done_rounds = 0;
    for (int sweep = 0; sweep < kJacMaxSweeps; ++sweep) {
        if (tid == 0) s_rotated = 0;
        __syncthreads();
        for (int round = 0; round < N - 1; ++round) {
            if (tid < npairs) {
                int p = rr_player(tid, round, N), q = rr_player(N - 1 - tid, round, N);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                const int rp = roff(p, n), rq = roff(q, n);
                if (q < n) {
                    const int ipp = rp + p, iqq = rq + q, ipq = rp + q;
                    const double app = sA[ipp], aqq = sA[iqq], apq = sA[ipq];
                    const bool small = fabs(apq) <= 1e-15 * sqrt(fabs(app * aqq)) || fabs(apq) <= abs_tol;
                    if (!small) {
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        s_rotated = 1;
                        // the pair's own 2x2 block becomes R^T A R: no other
                        // thread touches these three entries in this round
                        sA[ipp] = c * c * app - 2.0 * c * s * apq + s * s * aqq;
                        sA[iqq] = s * s * app + 2.0 * c * s * apq + c * c * aqq;
                        sA[ipq] = 0.0;
                    }
                }
                srot[tid] = Rot{c, s};
                spq[tid] = PairSlot{static_cast<short>(p), static_cast<short>(q), static_cast<short>(rp),
                                    static_cast<short>(rq)};
                const size_t li = (size_t)(done_rounds + round) * npairs + tid;
                log_rot[li] = Rot{c, s};
                log_pq[li] = p | (q << 16);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kBlk; ++j) {
                const int P = blkP[j], Q = blkQ[j];
                if (P < 0) continue;
                const Rot r1 = srot[P], r2 = srot[Q];
                if (r1.s == 0.0 && r2.s == 0.0) continue;
                const double c1 = r1.c, s1 = r1.s, c2 = r2.c, s2 = r2.s;
                const PairSlot a = spq[P], b = spq[Q];
                // element (x, y) of the symmetric matrix from the packed upper triangle
                auto at = [](int x, int rx, int y, int ry) { return x <= y ? rx + y : ry + x; };
                const int i00 = at(a.p, a.rp, b.p, b.rp);
                int i01 = at(a.p, a.rp, b.q, b.rq), i10 = at(a.q, a.rq, b.p, b.rp), i11 = at(a.q, a.rq, b.q, b.rq);
                if (odd) {   // only q can be the dummy index
                    if (b.q >= n) i01 = i11 = -1;
                    if (a.q >= n) i10 = i11 = -1;
                }
                const double x00 = sA[i00];
                const double x01 = i01 >= 0 ? sA[i01] : 0.0;
                const double x10 = i10 >= 0 ? sA[i10] : 0.0;
                const double x11 = i11 >= 0 ? sA[i11] : 0.0;
                const double y00 = c1 * x00 - s1 * x10, y01 = c1 * x01 - s1 * x11;
                const double y10 = s1 * x00 + c1 * x10, y11 = s1 * x01 + c1 * x11;
                sA[i00] = y00 * c2 - y01 * s2;
                if (i01 >= 0) sA[i01] = y00 * s2 + y01 * c2;
                if (i10 >= 0) sA[i10] = y10 * c2 - y11 * s2;
                if (i11 >= 0) sA[i11] = y10 * s2 + y11 * c2;
            }
            __syncthreads();
        }
        done_rounds += N - 1;
        if (!s_rotated) break;
        // converged when no pair passes the rotation test: the next sweep
        // would leave A as it is, so it is not run
        __syncthreads();
        if (tid == 0) s_rotated = 0;
        __syncthreads();
        for (int e = tid; e < n * n; e += kJacThreads) {
            const int i = e / n, j = e - (e / n) * n;
            if (i < j) {
                const double aij = sA[tri_idx(i, j, n)];
                const double aii = sA[tri_idx(i, i, n)], ajj = sA[tri_idx(j, j, n)];
                if (!(fabs(aij) <= 1e-15 * sqrt(fabs(aii * ajj)) || fabs(aij) <= abs_tol)) s_rotated = 1;
            }
        }
        __syncthreads();
        if (!s_rotated) break;
        __syncthreads();
    }
    if (tid == 0) *rounds = done_rounds;
    for (int i = tid; i < n; i += kJacThreads) evals[i] = sA[tri_idx(i, i, n)];
    __syncthreads();
    for (int i = tid; i < n; i += kJacThreads) {
        const double v = evals[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double u = evals[j];
            if (u > v || (u == v && j < i)) ++rank;
        }
        order[rank] = i;
    }
}

// V = product of the logged rotations: row r of V starts as e_r and every
// round rotates its column pairs.  Rows are independent; a workgroup keeps
// kRowsPerWg rows in LDS and stages the log in chunks of rounds.
constexpr int kApplyThreads = 256;
constexpr int kRowsPerWg = 4;
constexpr int kChunkRounds = 32;

__global__ __launch_bounds__(kApplyThreads) void jacobi_apply_kernel(const Rot* __restrict__ log_rot,
                                                                     const int* __restrict__ log_pq,
                                                                     const int* __restrict__ rounds, int n,
                                                                     double* __restrict__ V) {
    __shared__ double sV[kRowsPerWg][kJacLdsN];
    __shared__ Rot sR[kChunkRounds * (kJacLdsN / 2)];
    __shared__ int sPQ[kChunkRounds * (kJacLdsN / 2)];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * kRowsPerWg;
    const int nrows = min(kRowsPerWg, n - r0);
    const int npairs = ((n + 1) & ~1) / 2;
    for (int e = tid; e < kRowsPerWg * n; e += kApplyThreads) {
        const int rr = e / n, c = e % n;
        sV[rr][c] = (r0 + rr == c) ? 1.0 : 0.0;
    }
    const int total = *rounds;
    for (int base = 0; base < total; base += kChunkRounds) {
        const int nr = min(kChunkRounds, total - base);
        __syncthreads();
        for (int e = tid; e < nr * npairs; e += kApplyThreads) {
            sR[e] = log_rot[(size_t)base * npairs + e];
            sPQ[e] = log_pq[(size_t)base * npairs + e];
        }
        __syncthreads();
        for (int rd = 0; rd < nr; ++rd) {
            for (int e = tid; e < nrows * npairs; e += kApplyThreads) {
                const int rr = e / npairs, P = e % npairs;
                const Rot rot = sR[rd * npairs + P];
                const int pq = sPQ[rd * npairs + P];
                const int p = pq & 0xffff, q = pq >> 16;
                if (rot.s == 0.0 || q >= n) continue;
                const double vp = sV[rr][p], vq = sV[rr][q];
                sV[rr][p] = rot.c * vp - rot.s * vq;
                sV[rr][q] = rot.s * vp + rot.c * vq;
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < nrows * n; e += kApplyThreads) {
        const int rr = e / n, c = e % n;
        V[(size_t)(r0 + rr) * n + c] = sV[rr][c];
    }
}

// ------------------------------------------------------------ global form
__global__ __launch_bounds__(kJacThreads) void jacobi_global_kernel(double* __restrict__ A, double* __restrict__ V,
                                                                    int n, double* __restrict__ evals,
                                                                    int* __restrict__ order) {
    __shared__ double sc[kJacMaxN / 2], ss[kJacMaxN / 2];
    __shared__ int sp[kJacMaxN / 2], sq[kJacMaxN / 2];
    __shared__ double s_red[kJacThreads / 64];
    __shared__ int s_rotated;
    const int tid = threadIdx.x;
    const int N = (n + 1) & ~1;
    const int npairs = N / 2;
    double f = 0.0;
    for (int e = tid; e < n * n; e += kJacThreads) {
        V[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
        f += A[e] * A[e];
    }
    for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
    if ((tid & 63) == 0) s_red[tid >> 6] = f;
    __syncthreads();
    double fro = 0.0;
    for (int w = 0; w < kJacThreads / 64; ++w) fro += s_red[w];
    const double abs_tol = 1e-15 * sqrt(fro);
    for (int sweep = 0; sweep < kJacMaxSweeps; ++sweep) {
        if (tid == 0) s_rotated = 0;
        __syncthreads();
        for (int round = 0; round < N - 1; ++round) {
            if (tid < npairs) {
                int p = rr_player(tid, round, N), q = rr_player(N - 1 - tid, round, N);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q], apq = A[(size_t)p * n + q];
                    const bool small = fabs(apq) <= 1e-15 * sqrt(fabs(app * aqq)) || fabs(apq) <= abs_tol;
                    if (!small) {
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        s_rotated = 1;
                    }
                }
                sp[tid] = p;
                sq[tid] = q;
                sc[tid] = c;
                ss[tid] = s;
            }
            __syncthreads();
            for (int e = tid; e < npairs * npairs; e += kJacThreads) {
                const int P = e / npairs, Q = e % npairs;
                const int p1 = sp[P], q1 = sq[P], p2 = sp[Q], q2 = sq[Q];
                const double c1 = sc[P], s1 = ss[P], c2 = sc[Q], s2 = ss[Q];
                if (s1 == 0.0 && s2 == 0.0) continue;
                const bool r1ok = q1 < n, r2ok = q2 < n;
                const double x00 = A[(size_t)p1 * n + p2];
                const double x01 = r2ok ? A[(size_t)p1 * n + q2] : 0.0;
                const double x10 = r1ok ? A[(size_t)q1 * n + p2] : 0.0;
                const double x11 = (r1ok && r2ok) ? A[(size_t)q1 * n + q2] : 0.0;
                const double y00 = c1 * x00 - s1 * x10, y01 = c1 * x01 - s1 * x11;
                const double y10 = s1 * x00 + c1 * x10, y11 = s1 * x01 + c1 * x11;
                A[(size_t)p1 * n + p2] = y00 * c2 - y01 * s2;
                if (r2ok) A[(size_t)p1 * n + q2] = y00 * s2 + y01 * c2;
                if (r1ok) A[(size_t)q1 * n + p2] = y10 * c2 - y11 * s2;
                if (r1ok && r2ok) A[(size_t)q1 * n + q2] = y10 * s2 + y11 * c2;
            }
            for (int e = tid; e < n * npairs; e += kJacThreads) {
                const int r = e / npairs, P = e % npairs;
                const int p1 = sp[P], q1 = sq[P];
                const double c = sc[P], s = ss[P];
                if (s == 0.0 || q1 >= n) continue;
                const double vp = V[(size_t)r * n + p1], vq = V[(size_t)r * n + q1];
                V[(size_t)r * n + p1] = c * vp - s * vq;
                V[(size_t)r * n + q1] = s * vp + c * vq;
            }
            __threadfence_block();
            __syncthreads();
        }
        if (!s_rotated) break;
        // converged when no pair passes the rotation test (see the LDS form)
        __syncthreads();
        if (tid == 0) s_rotated = 0;
        __syncthreads();
        for (int e = tid; e < n * n; e += kJacThreads) {
            const int i = e / n, j = e - (e / n) * n;
            if (i < j) {
                const double aij = A[(size_t)i * n + j];
                const double aii = A[(size_t)i * n + i], ajj = A[(size_t)j * n + j];
                if (!(fabs(aij) <= 1e-15 * sqrt(fabs(aii * ajj)) || fabs(aij) <= abs_tol)) s_rotated = 1;
            }
        }
        __syncthreads();
        if (!s_rotated) break;
        __syncthreads();
    }
    for (int i = tid; i < n; i += kJacThreads) evals[i] = A[(size_t)i * n + i];
    __syncthreads();
    for (int i = tid; i < n; i += kJacThreads) {
        const double v = evals[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double u = evals[j];
            if (u > v || (u == v && j < i)) ++rank;
        }
        order[rank] = i;
    }
}

size_t log_entries(int n) {
    const int N = (n + 1) & ~1;
    return (size_t)kJacMaxSweeps * (N - 1) * (N / 2);
}

}  // namespace

size_t jacobi_ws_bytes(int n) {
    if (n > kJacLdsN) return 0;
    return ws_round(sizeof(Rot) * log_entries(n)) + ws_round(sizeof(int) * log_entries(n)) + ws_round(sizeof(int));
}

int jacobi(double* A, double* V, int n, double* evals, int* order, void* ws, hipStream_t s) {
    if (n < 1 || n > kJacMaxN) return fail(OTM_ECAPACITY, "eigensolver size must be in [1, 256]");
    if (n <= kJacLdsN) {
        WsCarver wc(ws, jacobi_ws_bytes(n));
        Rot* lr = wc.take<Rot>(log_entries(n));
        int* lp = wc.take<int>(log_entries(n));
        int* rounds = wc.take<int>(1);
        hipLaunchKernelGGL(jacobi_lds_kernel, dim3(1), dim3(kJacThreads), 0, s, A, n, evals, order, lr, lp, rounds);
        int st = check_launch("jacobi_lds_kernel");
        if (st != OTM_OK) return st;
        hipLaunchKernelGGL(jacobi_apply_kernel, dim3((n + kRowsPerWg - 1) / kRowsPerWg), dim3(kApplyThreads), 0, s, lr,
                           lp, rounds, n, V);
        return check_launch("jacobi_apply_kernel");
    }
    hipLaunchKernelGGL(jacobi_global_kernel, dim3(1), dim3(kJacThreads), 0, s, A, V, n, evals, order);
    return check_launch("jacobi_global_kernel");
}

}  // namespace otm
