// Sparse products of the hot path.
//
//  * whitening SpMM (Section 3.1 whitened data, Appendix A):
//      Y[t, :] = r_t sum_j C[t, j] W[j, :]
//    A group of LPR lanes owns one row; lane l of the group owns VPL
//    consecutive columns of W and Y, so every stored entry of the row costs one
//    coalesced gather of the W row.  The gathers come from L2 (W is reused by
//    every row), and their cost is set by the number of load instructions and
//    cache lines per entry, so W rows are read as 16-byte vectors when the row
//    stride ldw allows it (ldw a multiple of the vector and >= k rounded up to
//    it): a row of k = 50 FP32 values is 13 lanes of float4, four rows per
//    wave.  Y is written with non-temporal stores (it is not read again here;
//    W should stay in L2).  Column indices and values are loaded LPR at a time,
//    one per lane, and broadcast within the group by shuffles; four W rows are
//    in flight per iteration.  The group's FP32 accumulators also feed
//    per-block column sums (fixed order) for ybar.
//
//  * FP64 passes of the second-moment operator (Section 2, Eq. 2moment;
//    Section 4.2): T1 = diag(w2) C S, then C^T T1 together with C^T w2 and
//    C^T w1, then M1^T S and the rank-one / diagonal epilogue.
//
// Malformed CSR cannot make these kernels read out of bounds: row ranges are
// clamped to [0, nnz] and entries with a column outside [0, n_cols) are skipped.
#include <cmath>
#include <mutex>

#include "otm_internal.h"

namespace otm {
namespace {

constexpr int kSpmmThreads = 256;
constexpr int kSpmmMaxBlocks = 8192;

template <class T>
__device__ __forceinline__ float to_f(T x) { return static_cast<float>(x); }

template <int VPL, class TW>
struct WVec;
template <> struct WVec<1, float> { using T = float; };
template <> struct WVec<2, float> { using T = float __attribute__((ext_vector_type(2))); };
template <> struct WVec<4, float> { using T = float __attribute__((ext_vector_type(4))); };
template <> struct WVec<1, __bf16> { using T = __bf16; };
template <> struct WVec<2, __bf16> { using T = bf16x2; };
template <> struct WVec<4, __bf16> { using T = bf16x4; };
template <> struct WVec<8, __bf16> { using T = bf16x8; };

template <int VPL, class TW>
__device__ __forceinline__ void load_w(const TW* p, float (&out)[VPL]) {
    using V = typename WVec<VPL, TW>::T;
    const V v = *reinterpret_cast<const V*>(p);
    if constexpr (VPL == 1) {
        out[0] = to_f(v);
    } else {
#pragma unroll
        for (int e = 0; e < VPL; ++e) out[e] = to_f(v[e]);
    }
}

__device__ __forceinline__ void clamp_row(const int32_t* rowptr, int64_t nnz, int row, int64_t& b, int64_t& e) {
    b = rowptr[row];
    e = rowptr[row + 1];
    b = b < 0 ? 0 : (b > nnz ? nnz : b);
    e = e < b ? b : (e > nnz ? nnz : e);
}

// Y = diag(r) C W ; per-block column sums of the FP32 rows into part[0..k)[blockIdx]
// LDSW: the whole of W (n_cols rows of ks = k rounded up to VPL entries) is
// first copied into LDS by the workgroup, and the rows are gathered from there
// (for a W of at most about 128 KB; NT threads, one workgroup per CU).
template <int VPL, int LPR, class TW, class TY, int NT = kSpmmThreads, bool LDSW = false>
__global__ __launch_bounds__(NT) void whiten_kernel(otm_csr C, int normalize, const TW* __restrict__ W,
                                                   int k, int ldw, TY* __restrict__ Y, int ldy,
                                                   float* __restrict__ part, int yfull) {
    constexpr int lpr = LPR;
    constexpr int rows_per_block = NT / LPR;
    __shared__ float s_colsum[rows_per_block * LPR * VPL];
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    TW* s_w = reinterpret_cast<TW*>(s_dyn);
    const int ks = (k + VPL - 1) / VPL * VPL;    // LDS row stride of W
    if constexpr (LDSW) {
        using V = typename WVec<VPL, TW>::T;
        const int vpr = ks / VPL;
        const int nvec = C.n_cols * vpr;
        for (int q = threadIdx.x; q < nvec; q += NT) {
            const int r = q / vpr, cv = q - r * vpr;
            *reinterpret_cast<V*>(s_w + r * ks + cv * VPL) =
                *reinterpret_cast<const V*>(W + (size_t)r * ldw + cv * VPL);
        }
        __syncthreads();
    }
    const int tid = threadIdx.x;
    const int g_lane = tid % LPR;          // lane within the row group
    const int slot = tid / LPR;
    const int col0 = g_lane * VPL;
    const bool active = col0 < k;
    float colacc[VPL];
#pragma unroll
    for (int e = 0; e < VPL; ++e) colacc[e] = 0.f;

    const int n_rows = C.n_rows;
    const int64_t nnz = C.nnz;
    for (int rb = blockIdx.x; rb * rows_per_block < n_rows; rb += gridDim.x) {
        const int row = rb * rows_per_block + slot;
        if (row < n_rows) {
            int64_t b, e;
            clamp_row(C.rowptr, nnz, row, b, e);
            float acc[VPL];
#pragma unroll
            for (int v = 0; v < VPL; ++v) acc[v] = 0.f;
            float rowsum = 0.f;
            for (int64_t base = b; base < e; base += lpr) {
                const int64_t my = base + g_lane;
                int32_t my_col = -1;
                float my_val = 0.f;
                if (my < e) {
                    my_col = C.colidx[my];
                    my_val = C.vals ? C.vals[my] : 1.0f;
                    if (my_col < 0 || my_col >= C.n_cols) { my_col = -1; my_val = 0.f; }
                }
                const int cnt = static_cast<int>(min<int64_t>(lpr, e - base));
                int jj = 0;
                for (; jj + 4 <= cnt; jj += 4) {
                    int c4[4];
                    float v4[4];
                    float w4[4][VPL];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        c4[u] = __shfl(my_col, jj + u, lpr);
                        v4[u] = __shfl(my_val, jj + u, lpr);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (active && c4[u] >= 0) {
                            if constexpr (LDSW) load_w<VPL>(s_w + c4[u] * ks + col0, w4[u]);
                            else load_w<VPL>(W + (size_t)c4[u] * ldw + col0, w4[u]);
                        } else {
#pragma unroll
                            for (int v = 0; v < VPL; ++v) w4[u][v] = 0.f;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        rowsum += v4[u];
#pragma unroll
                        for (int v = 0; v < VPL; ++v) acc[v] += v4[u] * w4[u][v];
                    }
                }
                for (; jj < cnt; ++jj) {
                    const int c = __shfl(my_col, jj, lpr);
                    const float val = __shfl(my_val, jj, lpr);
                    float w1[VPL];
                    if (active && c >= 0) {
                        if constexpr (LDSW) load_w<VPL>(s_w + c * ks + col0, w1);
                        else load_w<VPL>(W + (size_t)c * ldw + col0, w1);
                    } else {
#pragma unroll
                        for (int v = 0; v < VPL; ++v) w1[v] = 0.f;
                    }
                    rowsum += val;
#pragma unroll
                    for (int v = 0; v < VPL; ++v) acc[v] += val * w1[v];
                }
            }
            const float r = normalize ? (rowsum > 0.f ? 1.0f / rowsum : 0.f) : 1.0f;
            TY* yrow = Y + (size_t)row * ldy;
            if (yfull) {
                // whole rows in one vector store per lane, the padding
                // columns' zeros included: a wave's rows leave as whole lines
                typedef TY YVec __attribute__((ext_vector_type(VPL)));
                if (col0 < ldy) {
                    YVec y;
#pragma unroll
                    for (int v = 0; v < VPL; ++v) {
                        const bool live_c = col0 + v < k;
                        const float yv = live_c ? acc[v] * r : 0.0f;
                        if (live_c) colacc[v] += yv;
                        y[v] = static_cast<TY>(yv);
                    }
                    __builtin_nontemporal_store(y, reinterpret_cast<YVec*>(yrow + col0));
                }
            } else if (active) {
                typedef TY YVec __attribute__((ext_vector_type(VPL)));
                TY* dst = yrow + col0;
                if (col0 + VPL <= k && reinterpret_cast<uintptr_t>(dst) % sizeof(YVec) == 0) {
                    YVec y;
#pragma unroll
                    for (int v = 0; v < VPL; ++v) {
                        const float yv = acc[v] * r;
                        colacc[v] += yv;
                        y[v] = static_cast<TY>(yv);
                    }
                    __builtin_nontemporal_store(y, reinterpret_cast<YVec*>(dst));
                } else {
#pragma unroll
                    for (int v = 0; v < VPL; ++v) {
                        if (col0 + v < k) {      // the last lane's vector may reach into W's padding columns
                            const float yv = acc[v] * r;
                            colacc[v] += yv;
                            __builtin_nontemporal_store(static_cast<TY>(yv), dst + v);
                        }
                    }
                }
            }
            if (!yfull)
                for (int c = k + g_lane; c < ldy; c += lpr) __builtin_nontemporal_store(static_cast<TY>(0.0f), yrow + c);
        }
    }
    // block column sums in a fixed order: slots 0..rows_per_block-1
    const int width = lpr * VPL;
#pragma unroll
    for (int v = 0; v < VPL; ++v) s_colsum[slot * width + col0 + v] = colacc[v];
    __syncthreads();
    for (int c = tid; c < k; c += NT) {
        float s = 0.f;
        for (int sl = 0; sl < rows_per_block; ++sl) s += s_colsum[sl * width + c];
        part[(size_t)c * gridDim.x + blockIdx.x] = s;     // column-major: the finalize reads it coalesced
    }
}

// out[c] = scale * sum_b part[c][b], fixed order, FP64 accumulation
// One workgroup per column: each thread sums its strided blocks in four
// interleaved FP64 partials (independent loads in flight), then a fixed-order
// LDS tree, so the mean does not depend on scheduling.
constexpr int kFinThreads = 256;
__global__ __launch_bounds__(kFinThreads) void colsum_finalize_kernel(const float* __restrict__ part, int nblocks,
                                                                      int k, double scale, float* __restrict__ out) {
    __shared__ double red[kFinThreads];
    const int c = blockIdx.x;
    const float* col = part + (size_t)c * nblocks;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int b = threadIdx.x;
    for (; b + 3 * kFinThreads < nblocks; b += 4 * kFinThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u) s4[u] += col[b + u * kFinThreads];
    }
#pragma unroll
    for (int u = 0; u < 3; ++u)          // at most three strided blocks remain
        if (b + u * kFinThreads < nblocks) s4[u] += col[b + u * kFinThreads];
    double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kFinThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = static_cast<float>(red[0] * scale);
}

// Whole-row vector stores of Y: every lane's vector inside the row stride and
// aligned (ldy a multiple of the vector, Y aligned to it), and the row's
// lanes covering the whole stride.
template <int VPL, int LPR, class TY>
int y_full_rows(const void* Y, int ldy) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(Y);
    return (ldy % VPL == 0 && a % (VPL * sizeof(TY)) == 0 && LPR * VPL >= ldy) ? 1 : 0;
}

template <int VPL, int LPR, class TW, class TY>
int launch_whiten(const otm_csr& C, int normalize, const void* W, int k, int ldw, void* Y, int ldy, float* part,
                  int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((whiten_kernel<VPL, LPR, TW, TY>), dim3(nblocks), dim3(kSpmmThreads), 0, st, C, normalize,
                       static_cast<const TW*>(W), k, ldw, static_cast<TY*>(Y), ldy, part,
                       y_full_rows<VPL, LPR, TY>(Y, ldy));
    return check_launch("whiten_kernel");
}

template <int VPL, class TW, class TY>
int dispatch_lpr(int lpr, const otm_csr& C, int normalize, const void* W, int k, int ldw, void* Y, int ldy,
                 float* part, int nblocks, hipStream_t st) {
    switch (lpr) {
        case 2: return launch_whiten<VPL, 2, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 4: return launch_whiten<VPL, 4, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 8: return launch_whiten<VPL, 8, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 16: return launch_whiten<VPL, 16, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 32: return launch_whiten<VPL, 32, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 64: return launch_whiten<VPL, 64, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        default: return fail(OTM_EINVAL, "bad lanes per row");
    }
}

constexpr int kLdsWThreads = 1024;
constexpr int kLdsWMinRow = 64;     // mean stored entries per row below which W stays in global memory

template <int VPL, int LPR, class TW, class TY>
int launch_whiten_lds(const otm_csr& C, int normalize, const void* W, int k, int ldw, void* Y, int ldy, float* part,
                      int nblocks, hipStream_t st) {
    const int ks = (k + VPL - 1) / VPL * VPL;
    const size_t shm = sizeof(TW) * (size_t)C.n_cols * ks;
    hipLaunchKernelGGL((whiten_kernel<VPL, LPR, TW, TY, kLdsWThreads, true>), dim3(nblocks), dim3(kLdsWThreads), shm,
                       st, C, normalize, static_cast<const TW*>(W), k, ldw, static_cast<TY*>(Y), ldy, part,
                       y_full_rows<VPL, LPR, TY>(Y, ldy));
    return check_launch("whiten_kernel (W in LDS)");
}

template <class TW, class TY>
int dispatch_whiten_lds(int lpr, const otm_csr& C, int normalize, const void* W, int k, int ldw, void* Y, int ldy,
                        float* part, int nblocks, hipStream_t st) {
    constexpr int V = 16 / static_cast<int>(sizeof(TW));
    switch (lpr) {
        case 8: return launch_whiten_lds<V, 8, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 16: return launch_whiten_lds<V, 16, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 32: return launch_whiten_lds<V, 32, TW, TY>(C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        default: return fail(OTM_EINVAL, "bad lanes per row");
    }
}

template <class TW, class TY>
int dispatch_whiten(int vpl, const otm_csr& C, int normalize, const void* W, int k, int ldw, void* Y, int ldy,
                    float* part, int nblocks, int lpr, hipStream_t st) {
    switch (vpl) {
        case 1: return dispatch_lpr<1, TW, TY>(lpr, C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 2: return dispatch_lpr<2, TW, TY>(lpr, C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        case 4: return dispatch_lpr<4, TW, TY>(lpr, C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
        default:
            if constexpr (sizeof(TW) == 2) return dispatch_lpr<8, TW, TY>(lpr, C, normalize, W, k, ldw, Y, ldy, part, nblocks, st);
            return fail(OTM_EINVAL, "bad vector width");
    }
}

struct WhitenPlan {
    int vpl, lpr, nblocks;
    bool lds;          // W staged in LDS (whiten_kernel<..., LDSW = true>)
};

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            return 256;
    }
    return cus;
}

// Widest vector (at most 16 bytes) that the row stride, the base alignment and
// the row length allow: ldw % vpl == 0, W aligned to the vector, and the last
// lane's vector (up to k rounded up to vpl) inside the row.
WhitenPlan plan_whiten(int32_t n_rows, int k, int ldw, int w_dtype, uintptr_t w_addr) {
    WhitenPlan p{};
    const int esize = (w_dtype == OTM_BF16) ? 2 : 4;
    p.vpl = 1;
    for (int v = 16 / esize; v > 1; v >>= 1) {
        const int span = (k + v - 1) / v * v;
        if (ldw % v == 0 && span <= ldw && w_addr % (uintptr_t)(v * esize) == 0) { p.vpl = v; break; }
    }
    const int lanes = (k + p.vpl - 1) / p.vpl;
    p.lpr = 1;
    while (p.lpr < lanes) p.lpr <<= 1;
    if (p.lpr < 2) p.lpr = 2;
    const int rpb = kSpmmThreads / (p.lpr > 64 ? 64 : p.lpr);
    int64_t blocks = (n_rows + rpb - 1) / rpb;
    if (blocks > kSpmmMaxBlocks) blocks = kSpmmMaxBlocks;
    if (blocks < 1) blocks = 1;
    p.nblocks = static_cast<int>(blocks);
    p.lds = false;
    return p;
}

// W in LDS pays when it fits beside the column-sum buffer, every column is
// gathered many times per workgroup (each of one or two workgroups per CU
// copies all of W once: at least 512 stored entries per column of W), and the
// rows are long (at least 64 entries on average): with short rows the row
// pointers, values and Y stores dominate and the L2 gathers cost the same.
void plan_whiten_lds(WhitenPlan& p, const otm_csr& C, int k, int w_dtype) {
    const int esize = (w_dtype == OTM_BF16) ? 2 : 4;
    if (p.vpl != 16 / esize || (p.lpr != 8 && p.lpr != 16 && p.lpr != 32)) return;
    const size_t ks = (size_t)(k + p.vpl - 1) / p.vpl * p.vpl;
    const size_t w_bytes = ks * esize * (size_t)C.n_cols;
    const size_t colsum_bytes = sizeof(float) * kLdsWThreads * p.vpl;
    const size_t need = w_bytes + colsum_bytes + 1024;
    if (C.n_cols < 1 || need > 160 * 1024) return;
    if (C.nnz < (int64_t)512 * C.n_cols) return;            // each W row gathered often enough to pay its copy
    if (C.nnz < (int64_t)kLdsWMinRow * C.n_rows) return;    // short rows: no gain over the L2 gathers
    // two workgroups per CU (8 waves per SIMD) where W fits twice and the
    // kernel's registers allow it (the FP32 variant stays under 64 VGPRs)
    const int per_cu = (esize == 4 && 2 * need <= 160 * 1024) ? 2 : 1;
    const int rpb = kLdsWThreads / p.lpr;
    int64_t blocks = (C.n_rows + rpb - 1) / rpb;
    const int64_t cap = (int64_t)device_cus() * per_cu;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    p.nblocks = static_cast<int>(blocks);
    p.lds = true;
}

// ---------------------------------------------------------------------------
// FP64 passes of the M2 operator.  One wave per row, lane owns up to 4 of the
// m <= 256 columns (lane, lane+64, ...).
// ---------------------------------------------------------------------------
constexpr int kM2Threads = 256;
constexpr int kM2Unroll = 4;

// Lane columns of a row of m <= 256 doubles: four per lane.  V2: pairs
// (2 lane, 2 lane + 1) and (128 + 2 lane, 129 + 2 lane), one 16-byte load
// each (m even, rows 16-byte aligned); otherwise lane + 64 u.  Each column
// is summed over the entries in the same order either way.
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <bool V2>
__device__ __forceinline__ int m2_col(int lane, int u) {
    return V2 ? 128 * (u >> 1) + 2 * lane + (u & 1) : lane + 64 * u;
}
template <bool V2>
__device__ __forceinline__ void m2_load(const double* __restrict__ row, int lane, int m, bool ok, double (&v)[4]) {
    if constexpr (V2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 128 * h + 2 * lane;
            if (ok && c < m) {
                const f64x2 t = *reinterpret_cast<const f64x2*>(row + c);
                v[2 * h] = t[0];
                v[2 * h + 1] = t[1];
            } else {
                v[2 * h] = 0.0;
                v[2 * h + 1] = 0.0;
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = lane + 64 * u;
            v[u] = (ok && c < m) ? row[c] : 0.0;
        }
    }
}

// T1[t,:] = w2_t sum_j C[t,j] S[j,:]; w1[t], w2[t] from the row sum when normalize
template <bool V2>
__global__ __launch_bounds__(kM2Threads) void m2_pass1_kernel(otm_csr C, int normalize, const double* __restrict__ S,
                                                              int m, double* __restrict__ T1, double* __restrict__ w1,
                                                              double* __restrict__ w2, int32_t* info) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * kM2Threads + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * kM2Threads) >> 6;
    for (int row = wave; row < C.n_rows; row += nwaves) {
        int64_t b, e;
        clamp_row(C.rowptr, C.nnz, row, b, e);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        double rs = 0.0;
        int64_t p = b;
        // kM2Unroll entries at a time: their indices, then their S rows, are
        // loaded together (the loads of one entry no longer wait on the
        // previous one); the sums still take the entries in order
        for (; p + kM2Unroll <= e; p += kM2Unroll) {
            int32_t cc[kM2Unroll];
            double vv[kM2Unroll], sv[kM2Unroll][4];
#pragma unroll
            for (int x = 0; x < kM2Unroll; ++x) {
                cc[x] = C.colidx[p + x];
                vv[x] = C.vals ? static_cast<double>(C.vals[p + x]) : 1.0;
            }
#pragma unroll
            for (int x = 0; x < kM2Unroll; ++x) {
                const bool ok = cc[x] >= 0 && cc[x] < C.n_cols;
                m2_load<V2>(S + (size_t)(ok ? cc[x] : 0) * m, lane, m, ok, sv[x]);
            }
#pragma unroll
            for (int x = 0; x < kM2Unroll; ++x) {
                if (cc[x] < 0 || cc[x] >= C.n_cols) continue;
                rs += vv[x];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (m2_col<V2>(lane, u) < m) acc[u] += vv[x] * sv[x][u];
            }
        }
        for (; p < e; ++p) {
            const int32_t c = C.colidx[p];
            if (c < 0 || c >= C.n_cols) continue;
            const double v = C.vals ? static_cast<double>(C.vals[p]) : 1.0;
            rs += v;
            double sv[4];
            m2_load<V2>(S + (size_t)c * m, lane, m, true, sv);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (m2_col<V2>(lane, u) < m) acc[u] += v * sv[u];
        }
        double a1 = 1.0, a2 = 1.0;
        if (normalize) {
            if (rs < 2.0) {
                if (lane == 0) *info = 1;
                a1 = 0.0;
                a2 = 0.0;
            } else {
                a1 = 1.0 / rs;
                a2 = 1.0 / (rs * (rs - 1.0));
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int col = m2_col<V2>(lane, u);
            if (col < m) T1[(size_t)row * m + col] = a2 * acc[u];
        }
        if (lane == 0) {
            w1[row] = a1;
            w2[row] = a2;
        }
    }
}

// O[a,:] = sum_x CT[a,x] T1[x,:];  u[a] = sum_x CT[a,x] w2[x];  M1[a] = (1/n) sum_x CT[a,x] w1[x]
template <bool V2>
__global__ __launch_bounds__(kM2Threads) void m2_pass2_kernel(otm_csr CT, const double* __restrict__ T1, int m,
                                                              const double* __restrict__ w1, const double* __restrict__ w2,
                                                              double inv_n, double* __restrict__ O, double* __restrict__ u,
                                                              double* __restrict__ M1) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * kM2Threads + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * kM2Threads) >> 6;
    for (int row = wave; row < CT.n_rows; row += nwaves) {
        int64_t b, e;
        clamp_row(CT.rowptr, CT.nnz, row, b, e);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        double su = 0.0, sm = 0.0;
        int64_t p = b;
        for (; p + kM2Unroll <= e; p += kM2Unroll) {   // as in the first pass
            int32_t xx[kM2Unroll];
            double vv[kM2Unroll], tv[kM2Unroll][4], ww2[kM2Unroll], ww1[kM2Unroll];
#pragma unroll
            for (int y = 0; y < kM2Unroll; ++y) {
                xx[y] = CT.colidx[p + y];
                vv[y] = CT.vals ? static_cast<double>(CT.vals[p + y]) : 1.0;
            }
#pragma unroll
            for (int y = 0; y < kM2Unroll; ++y) {
                const bool ok = xx[y] >= 0 && xx[y] < CT.n_cols;
                const int x = ok ? xx[y] : 0;
                ww2[y] = w2[x];
                ww1[y] = w1[x];
                m2_load<V2>(T1 + (size_t)x * m, lane, m, ok, tv[y]);
            }
#pragma unroll
            for (int y = 0; y < kM2Unroll; ++y) {
                if (xx[y] < 0 || xx[y] >= CT.n_cols) continue;
                su += vv[y] * ww2[y];
                sm += vv[y] * ww1[y];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (m2_col<V2>(lane, q) < m) acc[q] += vv[y] * tv[y][q];
            }
        }
        for (; p < e; ++p) {
            const int32_t x = CT.colidx[p];
            if (x < 0 || x >= CT.n_cols) continue;
            const double v = CT.vals ? static_cast<double>(CT.vals[p]) : 1.0;
            su += v * w2[x];
            sm += v * w1[x];
            double tv[4];
            m2_load<V2>(T1 + (size_t)x * m, lane, m, true, tv);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (m2_col<V2>(lane, q) < m) acc[q] += v * tv[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int col = m2_col<V2>(lane, q);
            if (col < m) O[(size_t)row * m + col] = acc[q];
        }
        if (lane == 0) {
            u[row] = su;
            M1[row] = sm * inv_n;
        }
    }
}

// part[b][c] = sum over this block's rows r of w[r] X[r][c]   (fixed order)
constexpr int kWcsThreads = 256;
constexpr int kWcsBlocks = 256;
__global__ __launch_bounds__(kWcsThreads) void weighted_colsum_partial_kernel(const double* __restrict__ w,
                                                                              const double* __restrict__ X, int rows,
                                                                              int m, double* __restrict__ part) {
    const int per = (rows + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * per;
    const int r1 = min(rows, r0 + per);
    for (int c = threadIdx.x; c < m; c += kWcsThreads) {
        double s = 0.0;
        for (int r = r0; r < r1; ++r) s += w[r] * X[(size_t)r * m + c];
        part[(size_t)blockIdx.x * m + c] = s;
    }
}

__global__ void sum_partials64_kernel(const double* __restrict__ part, int nparts, int m, double* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[(size_t)b * m + c];
    out[c] = s;
}

// O = (alpha0+1)/n (O - u * S) - alpha0 M1 v^T
__global__ void m2_epilogue_kernel(double* __restrict__ O, const double* __restrict__ S, const double* __restrict__ u,
                                   const double* __restrict__ M1, const double* __restrict__ v, int d, int m,
                                   double scale, double alpha0) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)d * m) return;
    const int a = static_cast<int>(idx / m), c = static_cast<int>(idx % m);
    O[idx] = scale * (O[idx] - u[a] * S[idx]) - alpha0 * M1[a] * v[c];
}

// out[i] = v for i < n (a kernel, not a memset node, so the call can be captured)
__global__ void fill_f32_kernel(float* __restrict__ out, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

__global__ void set_i32_kernel(int32_t* __restrict__ out, int32_t v) { *out = v; }

// ---------------------------------------------------------------------------
// M2 applied to a column selection with random signs (Section 4.2, sparse
// M2): O[:, j] = s_j M2[:, r_j]
//   = s_j [(alpha0+1)/n (sum_t w2_t c_t[r_j] c_t - u[r_j] e_(r_j)) - alpha0 M1 M1[r_j]],
// u = C^T w2, M1 = (1/n) C^T w1.  A column of M2 needs only the samples t
// with c_t[r_j] != 0 (row r_j of C^T) and their rows.
// ---------------------------------------------------------------------------
// w1, w2 of every row (one wave per row); info = 1 for a document under 2 tokens
__global__ __launch_bounds__(kM2Threads) void row_weights_kernel(otm_csr C, int normalize, double* __restrict__ w1,
                                                                 double* __restrict__ w2, int32_t* info) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * kM2Threads + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * kM2Threads) >> 6;
    for (int row = wave; row < C.n_rows; row += nwaves) {
        int64_t b, e;
        clamp_row(C.rowptr, C.nnz, row, b, e);
        double rs = 0.0;
        for (int64_t p = b + lane; p < e; p += 64) {
            const int32_t c = C.colidx[p];
            if (c >= 0 && c < C.n_cols) rs += C.vals ? static_cast<double>(C.vals[p]) : 1.0;
        }
        for (int o = 32; o > 0; o >>= 1) rs += __shfl_xor(rs, o);
        if (lane == 0) {
            double a1 = 1.0, a2 = 1.0;
            if (normalize) {
                if (rs < 2.0) {
                    *info = 1;
                    a1 = a2 = 0.0;
                } else {
                    a1 = 1.0 / rs;
                    a2 = 1.0 / (rs * (rs - 1.0));
                }
            }
            w1[row] = a1;
            w2[row] = a2;
        }
    }
}

// u[a] = sum_x CT[a, x] w2[x], M1[a] = inv_n sum_x CT[a, x] w1[x] (one wave per row of CT)
__global__ __launch_bounds__(kM2Threads) void col_weights_kernel(otm_csr CT, const double* __restrict__ w1,
                                                                 const double* __restrict__ w2, double inv_n,
                                                                 double* __restrict__ u, double* __restrict__ M1) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * kM2Threads + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * kM2Threads) >> 6;
    for (int row = wave; row < CT.n_rows; row += nwaves) {
        int64_t b, e;
        clamp_row(CT.rowptr, CT.nnz, row, b, e);
        double su = 0.0, sm = 0.0;
        for (int64_t p = b + lane; p < e; p += 64) {
            const int32_t x = CT.colidx[p];
            if (x < 0 || x >= CT.n_cols) continue;
            const double v = CT.vals ? static_cast<double>(CT.vals[p]) : 1.0;
            su += v * w2[x];
            sm += v * w1[x];
        }
        for (int o = 32; o > 0; o >>= 1) {
            su += __shfl_xor(su, o);
            sm += __shfl_xor(sm, o);
        }
        if (lane == 0) {
            u[row] = su;
            M1[row] = sm * inv_n;
        }
    }
}

__global__ void fill_f64_kernel(double* __restrict__ out, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// One workgroup per selected column j: O[:, j] += scale w2_t c_t[r_j] s_j c_t
// over the samples t of row r_j of C^T, in their stored order; the entries of
// one sample's row are distinct columns, so its threads never collide, and a
// barrier separates consecutive samples.  info = 2 for a row outside [0, d).
__global__ __launch_bounds__(kM2Threads) void select_scatter_kernel(otm_csr C, otm_csr CT,
                                                                    const int32_t* __restrict__ sel,
                                                                    const double* __restrict__ sgn,
                                                                    const double* __restrict__ w2, double scale, int kt,
                                                                    double* __restrict__ O, int32_t* info) {
    const int j = blockIdx.x;
    const int r = sel[j];
    if (r < 0 || r >= CT.n_rows) {
        if (threadIdx.x == 0) *info = 2;
        return;
    }
    const double sj = sgn[j];
    int64_t b, e;
    clamp_row(CT.rowptr, CT.nnz, r, b, e);
    for (int64_t p = b; p < e; ++p) {
        const int32_t t = CT.colidx[p];
        if (t < 0 || t >= C.n_rows) continue;
        const double coef = scale * w2[t] * (CT.vals ? static_cast<double>(CT.vals[p]) : 1.0) * sj;
        int64_t tb, te;
        clamp_row(C.rowptr, C.nnz, t, tb, te);
        for (int64_t q = tb + threadIdx.x; q < te; q += kM2Threads) {
            const int32_t a = C.colidx[q];
            if (a < 0 || a >= C.n_cols) continue;
            O[(size_t)a * kt + j] += coef * (C.vals ? static_cast<double>(C.vals[q]) : 1.0);
        }
        __syncthreads();
    }
}

// O[a, j] -= alpha0 M1[a] M1[r_j] s_j, and at a = r_j also scale u[r_j] s_j
__global__ void select_epilogue_kernel(double* __restrict__ O, const int32_t* __restrict__ sel,
                                       const double* __restrict__ sgn, const double* __restrict__ u,
                                       const double* __restrict__ M1, int d, int kt, double scale, double alpha0) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)d * kt) return;
    const int a = static_cast<int>(idx / kt), j = static_cast<int>(idx % kt);
    const int r = sel[j];
    if (r < 0 || r >= d) return;
    double v = O[idx] - alpha0 * M1[a] * M1[r] * sgn[j];
    if (a == r) v -= scale * u[r] * sgn[j];
    O[idx] = v;
}

__global__ void selection_dense_kernel(const int32_t* __restrict__ sel, const double* __restrict__ sgn, int d, int kt,
                                       double* __restrict__ S) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)d * kt) return;
    const int a = static_cast<int>(idx / kt), j = static_cast<int>(idx % kt);
    S[idx] = (sel[j] == a) ? sgn[j] : 0.0;
}

// Scratch of the entry point that allocates nothing: the per-block column sums
// of the whitening kernel (nblocks x k floats, at most 8192 x 128).  One copy
// per device, resolved through hipGetSymbolAddress on the first call there.
constexpr size_t kWhitenScratchFloats = size_t(1) << 20;   // 4 MiB
static __device__ __align__(256) float scratch[kWhitenScratchFloats];

// Y[row, :] = scale sum_j C[row, j] X[j, :]: the first M2 pass without its
// weights (one wave per row, kM2Unroll entries loaded together, entries
// summed in order).
template <bool V2>
__global__ __launch_bounds__(kM2Threads) void spmm64_kernel(otm_csr C, const double* __restrict__ X, int m,
                                                            double scale, double* __restrict__ Y) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * kM2Threads + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * kM2Threads) >> 6;
    for (int row = wave; row < C.n_rows; row += nwaves) {
        int64_t b, e;
        clamp_row(C.rowptr, C.nnz, row, b, e);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int64_t p = b;
        for (; p + kM2Unroll <= e; p += kM2Unroll) {
            int32_t cc[kM2Unroll];
            double vv[kM2Unroll], xv[kM2Unroll][4];
#pragma unroll
            for (int x = 0; x < kM2Unroll; ++x) {
                cc[x] = C.colidx[p + x];
                vv[x] = C.vals ? static_cast<double>(C.vals[p + x]) : 1.0;
            }
#pragma unroll
            for (int x = 0; x < kM2Unroll; ++x) {
                const bool ok = cc[x] >= 0 && cc[x] < C.n_cols;
                m2_load<V2>(X + (size_t)(ok ? cc[x] : 0) * m, lane, m, ok, xv[x]);
            }
#pragma unroll
            for (int x = 0; x < kM2Unroll; ++x) {
                if (cc[x] < 0 || cc[x] >= C.n_cols) continue;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (m2_col<V2>(lane, u) < m) acc[u] += vv[x] * xv[x][u];
            }
        }
        for (; p < e; ++p) {
            const int32_t c = C.colidx[p];
            if (c < 0 || c >= C.n_cols) continue;
            const double v = C.vals ? static_cast<double>(C.vals[p]) : 1.0;
            double xv[4];
            m2_load<V2>(X + (size_t)c * m, lane, m, true, xv);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (m2_col<V2>(lane, u) < m) acc[u] += v * xv[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int col = m2_col<V2>(lane, u);
            if (col < m) Y[(size_t)row * m + col] = scale * acc[u];
        }
    }
}

}  // namespace

int spmm64(const otm_csr& C, const double* X, int m, double scale, double* Y, hipStream_t s) {
    if (m < 1 || m > 256) return fail(OTM_ECAPACITY, "FP64 SpMM needs 1 <= m <= 256 columns");
    if (C.n_rows == 0) return OTM_OK;
    const int waves_per_block = kM2Threads / 64;
    int64_t nb = (C.n_rows + waves_per_block - 1) / waves_per_block;
    const int blocks = static_cast<int>(nb < 1 ? 1 : (nb > 4096 ? 4096 : nb));
    const bool v2 = m % 2 == 0 && (reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) % 16 == 0;
    if (v2)
        hipLaunchKernelGGL(spmm64_kernel<true>, dim3(blocks), dim3(kM2Threads), 0, s, C, X, m, scale, Y);
    else
        hipLaunchKernelGGL(spmm64_kernel<false>, dim3(blocks), dim3(kM2Threads), 0, s, C, X, m, scale, Y);
    return check_launch("spmm64_kernel");
}

}  // namespace otm

using namespace otm;

extern "C" size_t otm_whiten_workspace(int32_t n_rows, int32_t k) {
    if (n_rows < 0 || k < 1) return 0;
    // every plan has at least kSpmmThreads / 64 rows per block
    int64_t nb = ((int64_t)n_rows + 3) / 4;
    if (nb > kSpmmMaxBlocks) nb = kSpmmMaxBlocks;
    if (nb < 1) nb = 1;
    return ws_round(sizeof(float) * (size_t)nb * k);
}

namespace otm {
namespace {

// The whitening call on a given partial-sum buffer of part_floats floats.
int whiten_impl(const otm_csr* C, int normalize, const void* W, int w_dtype, int32_t k, int32_t ldw, void* Y,
                int y_dtype, int32_t ldy, float* ybar, float* part, size_t part_floats, hipStream_t s) {
    int st = validate_csr_header(C, "C");
    if (st != OTM_OK) return st;
    OTM_REQUIRE(W != nullptr && (Y != nullptr || C->n_rows == 0), OTM_EINVAL, "W and Y must not be NULL");
    OTM_REQUIRE(k >= 1 && ldy >= k && ldw >= k, OTM_ESHAPE, "need k >= 1, ldw >= k and ldy >= k");
    OTM_REQUIRE(w_dtype == OTM_F32 || w_dtype == OTM_BF16, OTM_EDTYPE, "W must be F32 or BF16");
    OTM_REQUIRE(y_dtype == OTM_F32 || y_dtype == OTM_BF16, OTM_EDTYPE, "Y must be F32 or BF16");
    OTM_REQUIRE(y_dtype != OTM_BF16 || ldy % 8 == 0, OTM_ESHAPE, "BF16 Y needs ldy % 8 == 0");
    OTM_REQUIRE(y_dtype != OTM_F32 || ldy % 4 == 0, OTM_ESHAPE, "F32 Y needs ldy % 4 == 0");
    WhitenPlan p = plan_whiten(C->n_rows, k, ldw, w_dtype, reinterpret_cast<uintptr_t>(W));
    OTM_REQUIRE(p.lpr <= 64, OTM_ECAPACITY, "k too large for the whitening kernel (k <= 64 * vector width)");
    if (C->n_rows == 0) {
        if (ybar) {
            hipLaunchKernelGGL(fill_f32_kernel, dim3((k + 255) / 256), dim3(256), 0, s, ybar, k, 0.0f);
            return check_launch("fill_f32_kernel");
        }
        return OTM_OK;
    }
    plan_whiten_lds(p, *C, k, w_dtype);
    OTM_REQUIRE(part != nullptr && (size_t)p.nblocks * k <= part_floats, OTM_EWORKSPACE,
                "whitening partial sums need more space than given");
    if (p.lds) {
        if (w_dtype == OTM_F32)
            st = (y_dtype == OTM_F32)
                     ? dispatch_whiten_lds<float, float>(p.lpr, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, s)
                     : dispatch_whiten_lds<float, __bf16>(p.lpr, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, s);
        else
            st = (y_dtype == OTM_F32)
                     ? dispatch_whiten_lds<__bf16, float>(p.lpr, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, s)
                     : dispatch_whiten_lds<__bf16, __bf16>(p.lpr, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, s);
    } else if (w_dtype == OTM_F32) {
        st = (y_dtype == OTM_F32)
                 ? dispatch_whiten<float, float>(p.vpl, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, p.lpr, s)
                 : dispatch_whiten<float, __bf16>(p.vpl, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, p.lpr, s);
    } else {
        st = (y_dtype == OTM_F32)
                 ? dispatch_whiten<__bf16, float>(p.vpl, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, p.lpr, s)
                 : dispatch_whiten<__bf16, __bf16>(p.vpl, *C, normalize, W, k, ldw, Y, ldy, part, p.nblocks, p.lpr, s);
    }
    if (st != OTM_OK) return st;
    if (ybar) {
        hipLaunchKernelGGL(colsum_finalize_kernel, dim3(k), dim3(kFinThreads), 0, s, part, p.nblocks, k,
                           1.0 / C->n_rows, ybar);
        return check_launch("colsum_finalize_kernel");
    }
    return OTM_OK;
}

// Device address of this device's copy of `scratch`, resolved once per device
// (with that device current) and kept; the array's host-side name is not a
// device address and is never passed to a kernel.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};

int scratch_for_current_device(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    OTM_REQUIRE(dev >= 0 && dev < kMaxDevices, OTM_ECAPACITY, "device index beyond the scratch table (64)");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch[dev];
    return OTM_OK;
}

}  // namespace
}  // namespace otm

extern "C" int otm_whiten(const otm_csr* C, int normalize, const void* W, int w_dtype, int32_t k, int32_t ldw,
                          void* Y, int y_dtype, int32_t ldy, float* ybar, void* ws, size_t ws_bytes,
                          otm_stream stream) {
    const int32_t rows = C ? C->n_rows : 0;
    OTM_REQUIRE(C == nullptr || rows == 0 || (ws != nullptr && ws_bytes >= otm_whiten_workspace(rows, k)),
                OTM_EWORKSPACE, "whiten workspace too small");
    return whiten_impl(C, normalize, W, w_dtype, k, ldw, Y, y_dtype, ldy, ybar, static_cast<float*>(ws),
                       ws_bytes / sizeof(float), as_stream(stream));
}

extern "C" size_t otm_whiten_noalloc_capacity(void) { return kWhitenScratchFloats; }

extern "C" int otm_whiten_noalloc(const otm_csr* C, int normalize, const void* W, int w_dtype, int32_t k, int32_t ldw,
                                  void* Y, int y_dtype, int32_t ldy, float* ybar, otm_stream stream) {
    float* part = nullptr;
    int st = scratch_for_current_device(&part);
    if (st != OTM_OK) return st;
    return whiten_impl(C, normalize, W, w_dtype, k, ldw, Y, y_dtype, ldy, ybar, part, kWhitenScratchFloats,
                       as_stream(stream));
}

extern "C" size_t otm_m2_apply_workspace(int32_t n, int32_t d, int32_t k_tilde) {
    if (n < 0 || d < 0 || k_tilde < 1) return 0;
    size_t b = 0;
    b += ws_round(sizeof(double) * (size_t)n * k_tilde);  // T1
    b += 2 * ws_round(sizeof(double) * (size_t)n);        // w1, w2
    b += 2 * ws_round(sizeof(double) * (size_t)d);        // u, M1
    b += ws_round(sizeof(double) * (size_t)kWcsBlocks * k_tilde);
    b += ws_round(sizeof(double) * (size_t)k_tilde);      // v
    return b;
}

extern "C" int otm_m2_apply(const otm_csr* C, const otm_csr* CT, int normalize, double alpha0, const double* S,
                            int32_t k_tilde, double* O, int32_t* info, void* ws, size_t ws_bytes, otm_stream stream) {
    int st = validate_csr_header(C, "C");
    if (st != OTM_OK) return st;
    st = validate_csr_header(CT, "CT");
    if (st != OTM_OK) return st;
    OTM_REQUIRE(S != nullptr && O != nullptr && info != nullptr, OTM_EINVAL, "S, O, info must not be NULL");
    OTM_REQUIRE(CT->n_rows == C->n_cols && CT->n_cols == C->n_rows && CT->nnz == C->nnz, OTM_ESHAPE,
                "CT must be the transpose of C");
    OTM_REQUIRE(k_tilde >= 1 && k_tilde <= 256, OTM_ECAPACITY, "need 1 <= k_tilde <= 256");
    OTM_REQUIRE(C->n_rows >= 1, OTM_ESHAPE, "need at least one sample");
    OTM_REQUIRE(std::isfinite(alpha0) && alpha0 >= 0.0, OTM_EINVAL, "alpha0 must be finite and >= 0");
    const int n = C->n_rows, d = C->n_cols;
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_m2_apply_workspace(n, d, k_tilde), OTM_EWORKSPACE,
                "m2_apply workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    double* T1 = wc.take<double>((size_t)n * k_tilde);
    double* w1 = wc.take<double>(n);
    double* w2 = wc.take<double>(n);
    double* u = wc.take<double>(d);
    double* M1 = wc.take<double>(d);
    double* part = wc.take<double>((size_t)kWcsBlocks * k_tilde);
    double* v = wc.take<double>(k_tilde);
    hipLaunchKernelGGL(set_i32_kernel, dim3(1), dim3(1), 0, s, info, 0);
    if ((st = check_launch("set_i32_kernel")) != OTM_OK) return st;
    const int waves_per_block = kM2Threads / 64;
    auto blocks_for = [&](int rows) {
        int64_t b = (rows + waves_per_block - 1) / waves_per_block;
        return static_cast<int>(b < 1 ? 1 : (b > 4096 ? 4096 : b));
    };
    // 16-byte row pieces when every row starts 16-byte aligned
    const bool v2 = k_tilde % 2 == 0 && (reinterpret_cast<uintptr_t>(S) | reinterpret_cast<uintptr_t>(T1)) % 16 == 0;
    if (v2)
        hipLaunchKernelGGL(m2_pass1_kernel<true>, dim3(blocks_for(n)), dim3(kM2Threads), 0, s, *C, normalize, S, k_tilde,
                           T1, w1, w2, info);
    else
        hipLaunchKernelGGL(m2_pass1_kernel<false>, dim3(blocks_for(n)), dim3(kM2Threads), 0, s, *C, normalize, S,
                           k_tilde, T1, w1, w2, info);
    if ((st = check_launch("m2_pass1_kernel")) != OTM_OK) return st;
    if (v2)
        hipLaunchKernelGGL(m2_pass2_kernel<true>, dim3(blocks_for(d)), dim3(kM2Threads), 0, s, *CT, T1, k_tilde, w1, w2,
                           1.0 / n, O, u, M1);
    else
        hipLaunchKernelGGL(m2_pass2_kernel<false>, dim3(blocks_for(d)), dim3(kM2Threads), 0, s, *CT, T1, k_tilde, w1,
                           w2, 1.0 / n, O, u, M1);
    if ((st = check_launch("m2_pass2_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(weighted_colsum_partial_kernel, dim3(kWcsBlocks), dim3(kWcsThreads), 0, s, M1, S, d, k_tilde,
                       part);
    if ((st = check_launch("weighted_colsum_partial_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(sum_partials64_kernel, dim3((k_tilde + 255) / 256), dim3(256), 0, s, part, kWcsBlocks, k_tilde, v);
    if ((st = check_launch("sum_partials64_kernel")) != OTM_OK) return st;
    const int64_t total = (int64_t)d * k_tilde;
    hipLaunchKernelGGL(m2_epilogue_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, O, S, u, M1, v, d,
                       k_tilde, (alpha0 + 1.0) / n, alpha0);
    return check_launch("m2_epilogue_kernel");
}

extern "C" size_t otm_m2_apply_select_workspace(int32_t n, int32_t d) {
    if (n < 0 || d < 0) return 0;
    return 2 * ws_round(sizeof(double) * (size_t)n) + 2 * ws_round(sizeof(double) * (size_t)d);
}

extern "C" int otm_m2_apply_select(const otm_csr* C, const otm_csr* CT, int normalize, double alpha0,
                                   const int32_t* sel_rows, const double* sel_signs, int32_t k_tilde, double* O,
                                   int32_t* info, void* ws, size_t ws_bytes, otm_stream stream) {
    int st = validate_csr_header(C, "C");
    if (st != OTM_OK) return st;
    if ((st = validate_csr_header(CT, "CT")) != OTM_OK) return st;
    OTM_REQUIRE(sel_rows && sel_signs && O && info, OTM_EINVAL, "sel_rows, sel_signs, O, info must not be NULL");
    OTM_REQUIRE(CT->n_rows == C->n_cols && CT->n_cols == C->n_rows && CT->nnz == C->nnz, OTM_ESHAPE,
                "CT must be the transpose of C");
    OTM_REQUIRE(k_tilde >= 1 && k_tilde <= 256, OTM_ECAPACITY, "need 1 <= k_tilde <= 256");
    OTM_REQUIRE(C->n_rows >= 1, OTM_ESHAPE, "need at least one sample");
    OTM_REQUIRE(std::isfinite(alpha0) && alpha0 >= 0.0, OTM_EINVAL, "alpha0 must be finite and >= 0");
    const int n = C->n_rows, d = C->n_cols;
    OTM_REQUIRE(ws && ws_bytes >= otm_m2_apply_select_workspace(n, d), OTM_EWORKSPACE,
                "m2_apply_select workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    double* w1 = wc.take<double>(n);
    double* w2 = wc.take<double>(n);
    double* u = wc.take<double>(d);
    double* M1 = wc.take<double>(d);
    auto blocks_for = [&](int rows) {
        int64_t b = (rows + kM2Threads / 64 - 1) / (kM2Threads / 64);
        return static_cast<int>(b < 1 ? 1 : (b > 4096 ? 4096 : b));
    };
    const double scale = (alpha0 + 1.0) / n;
    const int64_t total = (int64_t)d * k_tilde;
    hipLaunchKernelGGL(set_i32_kernel, dim3(1), dim3(1), 0, s, info, 0);
    if ((st = check_launch("set_i32_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(row_weights_kernel, dim3(blocks_for(n)), dim3(kM2Threads), 0, s, *C, normalize, w1, w2, info);
    if ((st = check_launch("row_weights_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(col_weights_kernel, dim3(blocks_for(d)), dim3(kM2Threads), 0, s, *CT, w1, w2, 1.0 / n, u, M1);
    if ((st = check_launch("col_weights_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, O, total, 0.0);
    if ((st = check_launch("fill_f64_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(select_scatter_kernel, dim3(k_tilde), dim3(kM2Threads), 0, s, *C, *CT, sel_rows, sel_signs, w2,
                       scale, k_tilde, O, info);
    if ((st = check_launch("select_scatter_kernel")) != OTM_OK) return st;
    hipLaunchKernelGGL(select_epilogue_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, O, sel_rows,
                       sel_signs, u, M1, d, k_tilde, scale, alpha0);
    return check_launch("select_epilogue_kernel");
}

extern "C" int otm_selection_dense(const int32_t* sel_rows, const double* sel_signs, int32_t d, int32_t k_tilde,
                                   double* S, otm_stream stream) {
    OTM_REQUIRE(sel_rows && sel_signs && S, OTM_EINVAL, "sel_rows, sel_signs, S must not be NULL");
    OTM_REQUIRE(d >= 1 && k_tilde >= 1, OTM_ESHAPE, "need d, k_tilde >= 1");
    const int64_t total = (int64_t)d * k_tilde;
    hipLaunchKernelGGL(selection_dense_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, as_stream(stream),
                       sel_rows, sel_signs, d, k_tilde, S);
    return check_launch("selection_dense_kernel");
}
