// Stochastic tensor gradient descent on the implicit whitened third moment
// (Section 3.2, Lemma "update"), in the stacked matrix form of Section 4.3:
//
//   PA = YA Phi, PB = YB Phi                       (batch x k, matrix cores)
//   mA = Phi^T ybarA, mB = Phi^T ybarB             (k, vector ALU)
//   H  = PA * PB,  s = column sums of H            (cross-lane swaps)
//   Q  = a H - b PA diag(mB) - b diag(mA) PB
//   D  = YC^T Q / B + ybarC (c mA*mB - b s / B)^T  (matrix cores)
//   G  = Phi^T Phi,  O = Phi (G * G)               (matrix cores)
//   Phi <- Phi + beta (D - kappa O)                 (compensated FP32)
//
// One workgroup of 8 waves runs one whole online run (all steps), keeping the
// FP32 master copy of Phi (and its Kahan compensation) in registers.  The
// tensor is never formed.  The waves form a WR x WC grid (WR * WC = 8; 4 x 2
// by default): wave (wr, wc) owns the 16x16 output tiles (mt, nt) with
// mt = wr mod WR and nt = wc mod WC of every product, so the update of a Phi
// tile needs only the O and D tiles the same wave computed.  The -beta kappa O
// part of the update enters the register master copy right after O is formed
// (so O does not stay live), the direction part at the end of the step; the
// LDS operand copies keep the old Phi for every product of the step.  LDS
// holds the operand copy of Phi (phi_i-major; BF16 products that need it the
// other way round use transposing LDS reads), a buffer that carries G*G and
// then Q from the accumulator layout to the operand layout, the mini-batch of
// whitened rows, and small vectors.  In BF16 the rows of the Phi copy and of
// the buffer are stored with a column permutation that keeps both the
// fragment reads and the tile stores free of most bank conflicts.
//
// Batch staging (NSTAGE = 1 for one shared view, 3 for three views): the rows
// of step t+1 are fetched into registers while step t computes (their indices
// were fetched during step t-1) and written to LDS row-major at the start of
// step t+1, so the products never wait on global memory; no load is waited on
// right after it is issued (checks and masks happen where the values are
// used).  NSTAGE = 0 (shapes whose batch does not fit in LDS) reads the rows
// from global memory inside the products, after pulling the next step's rows
// into L2 at the end of each step.
//
// FP32 operands (one k per lane and MFMA): lane group q takes a contiguous k
// range, so four consecutive k are one 16-byte LDS read; the k sum is the same
// set of products in another order.
//
// Four workgroup barriers per step: after G*G, after O (the buffer then
// takes Q), after Q, after the update.  The batch is padded to 128 rows, so
// every tile loop has a compile-time trip count (the FP32 D product over rows
// read from global memory stops at the batch size instead).
//
// Optional scoring pass (score != NULL): after the last update, one more pass
// over the rows in natural order evaluates, without updating,
//   score = sum_ij (phi_i^T phi_j)^3 - 2 sum_i T(phi_i, phi_i, phi_i),
// which is ||sum_i phi_i^(x3) - T||_F^2 - ||T||_F^2: the residual up to a
// constant of the data, used to rank restarts.  T(phi_i, phi_i, phi_i) is
// phi_i^T D_i with D the step's direction term on a batch, weighted by the
// batch's share of the rows.
#pragma once

#include <cmath>
#include <type_traits>

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
    using Chunk = f32x4;                      // 16-byte row piece of the batch
    static constexpr int KI = 4;
    static constexpr int EPL = 1;
    static constexpr int SPAD = 4;            // LDS row padding (elements)
    static constexpr int CH = 4;              // elements per chunk
    __device__ static f32x4 mma(Frag a, Frag b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static Frag lds(const Op* p) { return *p; }
    __device__ static Op to_op(float x) { return x; }
    __device__ static float op_to_f(Op x) { return x; }
    __device__ static Frag zero_frag() { return 0.0f; }
    // fragment of EPL consecutive row elements a0.. (masked at k)
    __device__ static Frag yrow(const Y* row, int a0, int k) {
        return (row != nullptr && a0 < k) ? row[a0] : 0.0f;
    }
    // elements e >= valid of a row piece set to 0 (the padding past k)
    __device__ static Chunk mask_chunk(Chunk v, int valid) {
#pragma unroll
        for (int e = 0; e < CH; ++e)
            if (e >= valid) v[e] = 0.0f;
        return v;
    }
    __device__ static Chunk zero_chunk() { return Chunk{0.f, 0.f, 0.f, 0.f}; }
    // bit mask of the first `valid` elements of a chunk, and a chunk ANDed with it
    __device__ static u32x4 chunk_mask(int valid) {
        u32x4 m;
#pragma unroll
        for (int d = 0; d < 4; ++d) m[d] = (d < valid) ? 0xffffffffu : 0u;
        return m;
    }
    __device__ static Chunk and_chunk(Chunk x, u32x4 m) {
        return __builtin_bit_cast(Chunk, __builtin_bit_cast(u32x4, x) & m);
    }
    __device__ static void store4(Op* p, f32x4 v) { *reinterpret_cast<f32x4*>(p) = v; }
    __device__ static f32x4 load4(const Op* p) { return *reinterpret_cast<const f32x4*>(p); }
    // column permutation of row r of the Phi copy and the exchange buffer (none in FP32)
    __device__ static constexpr int sw(int) { return 0; }
};

struct MmaBF16 {
    using Y = __bf16;
    using Op = __bf16;
    using Frag = bf16x8;
    using Chunk = bf16x8;
    static constexpr int KI = 32;
    static constexpr int EPL = 8;
    // LDS row padding: rows 288 bytes apart.  Of the pitches 256 to 336
    // bytes this is the only one at which a fragment read (lane l: row l % 16,
    // 16-byte chunk l / 16) runs without bank conflicts on gfx950 (4 cycles
    // per wave against 8 to 32); 272 and 304 were about 4% slower per step
    static constexpr int SPAD = 16;
    static constexpr int CH = 8;
    __device__ static f32x4 mma(Frag a, Frag b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static Frag lds(const Op* p) { return *reinterpret_cast<const bf16x8*>(p); }
    // Column permutation of row r of the Phi copy and the exchange buffer: rows
    // with bit 2 set swap their 16-byte chunks in pairs.  At the 288-byte
    // pitch the 8-byte stores of a product's output tile (lane l: row l % 16,
    // piece l / 16) hit each bank twice as often as they need to (16 cycles
    // per wave); with the permutation they take 8 (a contiguous 8-byte store
    // takes 6.6), while the fragment reads stay conflict-free (measured on
    // gfx950; BF16 k = 100 step 5.02 -> 4.85 us).
    __device__ static constexpr int sw(int r) { return ((r >> 2) & 1) << 3; }
    // Fragment of a matrix stored the other way round: lane l receives
    // X[8 (l/16) + e][l % 16], e < 8, where X[r][c] = x[r * stride + c] in
    // LDS.  Two transposing 8-byte reads (rows 0-3 and 4-7 of the lane's
    // group): lane s addresses columns 4 (s % 4) .. + 3 of row
    // 8 (s/16) + (s % 16)/4, and element i of lane l comes from element l % 4
    // of lane 16 (l/16) + (l % 16)/4 + 4 i.  x and stride keep every address
    // 8-byte aligned.
    __device__ static Frag lds_t(const Op* x, int stride, int lane) {
        typedef short s16x4 __attribute__((ext_vector_type(4)));
        typedef short s16x8 __attribute__((ext_vector_type(8)));
        typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
        const Op* p = x + (8 * (lane >> 4) + ((lane >> 2) & 3)) * stride + 4 * (lane & 3);
        const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p));
        const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + 4 * stride));
        const s16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_bit_cast(Frag, v);
    }
    // lds_t on a permuted array (sw above), x at a row that is a multiple of 8
    // and a column that is a multiple of 16: the first read's rows keep their
    // order, the second read's rows (bit 2 set) have their chunks swapped
    __device__ static Frag lds_t_sw(const Op* x, int stride, int lane) {
        typedef short s16x4 __attribute__((ext_vector_type(4)));
        typedef short s16x8 __attribute__((ext_vector_type(8)));
        typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
        const Op* p = x + (8 * (lane >> 4) + ((lane >> 2) & 3)) * stride;
        const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + 4 * (lane & 3)));
        const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + 4 * stride + ((4 * (lane & 3)) ^ 8)));
        const s16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_bit_cast(Frag, v);
    }
    __device__ static Op to_op(float x) { return f32_to_bf16(x); }
    __device__ static float op_to_f(Op x) { return bf16_to_f32(x); }
    __device__ static Frag zero_frag() {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = f32_to_bf16(0.0f);
        return v;
    }
    __device__ static Frag yrow(const Y* row, int a0, int k) {
        if (row != nullptr && a0 < k) {
            // ldy % 8 == 0 and a0 % 8 == 0: the 16-byte load stays inside the row
            bf16x8 v = *reinterpret_cast<const bf16x8*>(row + a0);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (a0 + e >= k) v[e] = f32_to_bf16(0.0f);
            return v;
        }
        return zero_frag();
    }
    __device__ static Chunk mask_chunk(Chunk v, int valid) {
#pragma unroll
        for (int e = 0; e < CH; ++e)
            if (e >= valid) v[e] = f32_to_bf16(0.0f);
        return v;
    }
    __device__ static Chunk zero_chunk() { return zero_frag(); }
    // bit mask of the first `valid` elements of a chunk (two per dword), and a
    // chunk ANDed with it
    __device__ static u32x4 chunk_mask(int valid) {
        u32x4 m;
#pragma unroll
        for (int d = 0; d < 4; ++d)
            m[d] = ((2 * d < valid) ? 0x0000ffffu : 0u) | ((2 * d + 1 < valid) ? 0xffff0000u : 0u);
        return m;
    }
    __device__ static Chunk and_chunk(Chunk x, u32x4 m) {
        return __builtin_bit_cast(Chunk, __builtin_bit_cast(u32x4, x) & m);
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
    const float* Phi0;      // initial factors (may equal Phi)
    float* Phi;
    float* Phi_comp;
    float* snapshots;
    int32_t* nonfinite;
    double* score;          // NULL: no scoring pass
    int32_t n, k, batch, passes, ldy, compensated;
    int32_t start_step, end_step, spp;
    float a, b, c, kappa;
    float beta0, inv_tau;
};

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int MB = kMaxBatch;           // batch rows padded to 128 in every product
constexpr int NTM = MB / 16;            // batch tiles

// Four consecutive FP32 row entries a0..a0+3 (0 past k or without a row);
// a0 is a multiple of 4 and rows are 16-byte aligned (ldy % 4 == 0)
__device__ __forceinline__ f32x4 yrow4(const float* row, int a0, int k) {
    if (row == nullptr || a0 >= k) return f32x4{0.f, 0.f, 0.f, 0.f};
    if (a0 + 4 <= k) return *reinterpret_cast<const f32x4*>(row + a0);
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (a0 + e < k) v[e] = row[a0 + e];
    return v;
}
__device__ __forceinline__ f32x4 yrow4(const __bf16*, int, int) { return f32x4{0.f, 0.f, 0.f, 0.f}; }

template <class M, int KP, int NSTAGE, int WR = 4>
struct SgdSmem {
    using Op = typename M::Op;
    using Y = typename M::Y;
    static constexpr int SP = KP + M::SPAD;        // Phi rows
    static constexpr int SB = MB + M::SPAD;        // exchange buffer rows (t or j)
    static constexpr int SY = KP + M::SPAD;        // staged batch rows
    static constexpr bool kStageCT = (NSTAGE == 0) && M::EPL == 8;   // BF16 fallback: YC batch a-major
    alignas(16) Op phi[KP * SP];
    alignas(16) Op yfold[2 * SP];                  // ybarA, ybarB rows of the Phi^T Phi fold
    alignas(16) Op buf[KP * SB];
    alignas(16) Y ybatch[NSTAGE > 0 ? NSTAGE * MB * SY : 1];
    alignas(16) Op yct[kStageCT ? KP * SB : 1];
    alignas(16) int32_t idx[MB];
    // NSTAGE == 0: landing area of the L2 prefetch of the next step's rows
    // (written by direct-to-LDS loads, never read)
    alignas(16) uint32_t pf[NSTAGE == 0 ? kWaves * 64 : 1];
    alignas(16) float ybar[3 * KP];
    alignas(16) float m[2 * KP];
    alignas(16) float s[WR * KP];
    double red[kWaves];
};

template <class M, int KP, int NSTAGE, int WR = 4>
constexpr size_t smem_bytes() { return sizeof(SgdSmem<M, KP, NSTAGE, WR>); }

constexpr size_t kLdsLimit = 160 * 1024;

// The largest batch staging that fits in LDS (one view when the three views
// alias, else three), 0 when none fits.
template <class M, int KP, int WR = 4>
constexpr int staging_for(bool aliased) {
    if (aliased) return smem_bytes<M, KP, 1, WR>() <= kLdsLimit ? 1 : 0;
    return smem_bytes<M, KP, 3, WR>() <= kLdsLimit ? 3 : 0;
}

// x + (x of lane l ^ 1, l ^ 16 or l ^ 32) in every lane l, without a round
// trip through the LDS crossbar: a quad-permutation DPP move for l ^ 1, and
// gfx950's row swap (16 lanes) and half swap (32 lanes) for the others.  Both
// lanes of a pair get the same sum, since addition commutes, so the result
// equals that of a shuffle-based butterfly bit for bit.
__device__ __forceinline__ float add_xor1(float x) {
    const int p = __builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false);   // [1, 0, 3, 2]
    return x + __int_as_float(p);
}
__device__ __forceinline__ float add_xor16(float x) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float add_xor32(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Symmetric G = Phi^T Phi with ntk = 7 or 8 tile rows on a 4 x 2 wave grid:
// wave row wr takes tile rows wr and ntk - 1 - wr (tile row ti = 0, 1; the
// second only where it differs from the first) and, of the tile columns
// wc + 2 tj, only those on or above the diagonal and inside the ntl live
// tiles.  A wave row then carries at most 7 (ntl = 7, ntk = 8), 8 (ntk = 7)
// or 9 (ntl = 8) tiles.
__host__ __device__ constexpr int tri_row(int wr, int ti, int ntk) { return ti == 0 ? wr : ntk - 1 - wr; }
__host__ __device__ constexpr bool tri_tile(int wr, int wc, int ti, int tj, int ntl, int ntk) {
    return (ti == 0 || ntk - 1 - wr > wr) && tri_row(wr, ti, ntk) <= wc + 2 * tj && wc + 2 * tj < ntl;
}

template <int N>
using IntC = std::integral_constant<int, N>;

template <int WR>
__device__ __forceinline__ void wave_grid(int w, int& wr, int& wc) {
    constexpr int WC = kWaves / WR;
    // Waves w and w + 4 run on the same SIMD (the CU deals a workgroup's waves
    // out to its four SIMDs in turn).  With WR >= 4 the two waves of a SIMD
    // take the same wave row and both wave columns, so when the tile count
    // leaves the last wave row or column short (k = 100: 7 tiles) the four
    // SIMDs still carry near-equal shares of the MFMA work (FP32 k = 100:
    // 44.6 -> 42.2 us per step; every tile keeps its summation order, so the
    // results are unchanged).  The masks give the compiler the ranges of wr
    // and wc.
    if constexpr (WR >= 4) {
        wr = ((w & 3) + 4 * ((w >> 2) & (WR / 4 - 1))) & (WR - 1);
        wc = ((w >> 2) / (WR / 4)) & (WC - 1);
    } else {
        wr = (w / WC) & (WR - 1);
        wc = w & (WC - 1);
    }
}

// One whole run of restart r_id, by one wave of the calling workgroup whose
// last tile row (DR = 1) and column (DC = 1) it skips or not: they lie
// outside KP, or past the NTL tiles that hold components, coordinates and
// the two folded means (the rest is padding, zero in every product).  OV:
// the three views alias and the rows are read from global memory.
template <class M, int KP, int NSTAGE, int WR, bool SCORE, bool COMP, int NTL, int DR, int DC, bool OV>
__device__ __forceinline__ void sgd_body_t(const SgdArgs& g, const int r_id, SgdSmem<M, KP, NSTAGE, WR>& sm) {
    using Op = typename M::Op;
    using Y = typename M::Y;
    constexpr int WC = kWaves / WR;
    static_assert(WR * WC == kWaves, "wave grid must cover the workgroup");
    using SM = SgdSmem<M, KP, NSTAGE, WR>;
    constexpr int NTK = KP / 16;
    constexpr int TC = (NTK + WC - 1) / WC;        // tile columns per wave
    constexpr int TRK = (NTK + WR - 1) / WR;       // tile rows per wave in the k x k products
    constexpr int kTR = NTM / WR;                  // batch tile rows per wave
    constexpr int SP = SM::SP, SB = SM::SB, SY = SM::SY;
    constexpr int cpr = KP / M::CH;                // 16-byte chunks per batch row
    constexpr int KQ = KP / 4;                     // FP32: k range of one lane group
    constexpr int NCH = (MB * cpr + kThreads - 1) / kThreads;   // chunks per thread when staging
    constexpr int UNR = (M::KI >= 32) ? 4 : 2;     // unroll of the k x k and D contraction loops
    // and of the batch products: fully unrolled for staged BF16 rows (the first
    // MFMA then starts from zero without clearing registers); FP32 and
    // unstaged rows spill registers beyond 2
    constexpr int UNR_P = (M::EPL == 8 && NSTAGE > 0) ? 4 : 2;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // wave index in a scalar register
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6) & (kWaves - 1);
    int wr, wc;
    wave_grid<WR>(w, wr, wc);
    // this wave's tile rows and columns that it computes (the last of each can
    // fall outside KP when the tile count is not a multiple of the grid, or
    // hold only padding): compile-time counts, so no tile guard is left in
    // the product loops
    constexpr int TRL = TRK - DR, TCL = TC - DC;
    const int l16 = lane & 15, q = lane >> 4;
    // column permutation of every row 16 m + l16 of the Phi copy and the
    // exchange buffer, folded into the lane's fragment column (cq) and output
    // column (sq): k0 + cq and 16 mt + sq keep the tile offsets additive
    // (not for three staged views at KP = 96, where the extra per-lane offsets
    // cost registers: no gain on the plain step, 6.4 -> 6.8 us per step on the
    // compensated one)
    constexpr bool kPerm = M::EPL != 1 && !(NSTAGE == 3 && KP >= 96);
    auto swz = [](int r) { return kPerm ? M::sw(r) : 0; };
    // BF16 at KP = 128: the G product computes only the tiles of tri_tile and
    // writes the others from them (G is symmetric on the components, and the
    // matrix cores sum Phi_i^T Phi_j and Phi_j^T Phi_i in the same order, so
    // the results are unchanged).  BF16: only in the plain kernels with 7 live
    // tiles and at most one staged view (k = 100, one view: 4.28-4.37 -> 4.14
    // us per step; three views read from global memory: 16.7-16.9 -> 16.4);
    // with 8 live tiles or with compensation terms the extra registers spill
    // and the step is slower, so those keep the full product.  FP32: the
    // single-run kernels whose rows are read from global memory (k = 100, one
    // view: 31.3-31.6 -> 28.8-29.0 us; k = 128: 39.0 -> 35.8 us); the batched
    // kernels, which also score restarts from G, keep the full product (their
    // three-view variants would spill, and one of them bounds a batched run).
    constexpr bool kTri = (M::EPL == 8 && WR == 4 && KP == 128 && NSTAGE <= 1 && !COMP && NTL == 7 && !SCORE) ||
                          (M::EPL == 1 && WR == 4 && (KP == 112 || KP == 128) && NSTAGE == 0 && !SCORE);
    const int swl = swz(l16);
    const int cq = (q * M::EPL) ^ swl, sq = (4 * q) ^ swl;

    const int k = g.k;
    const int n = g.n, ldy = g.ldy, B = g.batch;
    const float* Phi0 = g.Phi0 + (size_t)r_id * k * k;
    float* Phi = g.Phi + (size_t)r_id * k * k;
    float* Comp = g.Phi_comp ? g.Phi_comp + (size_t)r_id * k * k : nullptr;
    float* Snap = g.snapshots ? g.snapshots + (size_t)r_id * g.passes * k * k : nullptr;
    const int32_t* perms = g.perms ? g.perms + (size_t)r_id * g.perm_stride : nullptr;
    const Y* Yv[3] = {static_cast<const Y*>(g.YA), static_cast<const Y*>(g.YB), static_cast<const Y*>(g.YC)};
    bool bad = false;
    const float cmask = g.compensated ? 1.0f : 0.0f;
    // mA = Phi^T ybarA and mB = Phi^T ybarB ride along in Phi^T Phi when two
    // padding rows are free: the second operand of that product takes ybarA,
    // ybarB (the yfold rows) as "components" k and k+1, so G[i][k] = mA[i] and
    // G[i][k+1] = mB[i].  Every other product reads the zero rows k, k+1 of
    // the Phi copy, so G[k][.] and G[k+1][.] are zero as well.
    const bool mfold = (k + 2 <= KP);

    // ---- master copy of Phi: tile (mt, nt) holds a = row, i = column.  In
    // BF16 it lives in registers; in FP32 the LDS operand copy is exact, so it
    // is the master copy itself and the registers go to the products.  The
    // compensation terms stay in registers.  COMP = false (BF16 only, for runs
    // without compensation) drops them: -beta kappa O then goes straight into
    // the register master copy, which frees TRK * TC * 4 registers.
    constexpr bool kPhiReg = M::EPL != 1;
    constexpr bool kComp = COMP || !kPhiReg;
    f32x4 phi_r[kPhiReg ? TRK : 1][kPhiReg ? TC : 1], comp[kComp ? TRK : 1][kComp ? TC : 1];
    auto phi_get = [&](int ti, int tj) -> f32x4 {
        if constexpr (kPhiReg) {
            return phi_r[ti][tj];
        } else {
            const int mt = wr + WR * ti, nt = wc + WC * tj;
            return M::load4(&sm.phi[(nt * 16 + l16) * SP + mt * 16 + 4 * q]);
        }
    };
#pragma unroll
    for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
        for (int tj = 0; tj < TC; ++tj) {
            const int mt = wr + WR * ti, nt = wc + WC * tj;
            f32x4 v = {0.f, 0.f, 0.f, 0.f}, cv = {0.f, 0.f, 0.f, 0.f};
            if (mt < NTK && nt < NTK) {   // every tile inside KP, the skipped padding tiles as zeros
                const int i = nt * 16 + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = mt * 16 + 4 * q + r;
                    if (a < k && i < k) {
                        v[r] = Phi0[(size_t)i * k + a];
                        if (Comp && g.compensated) cv[r] = Comp[(size_t)i * k + a];
                    }
                }
                M::store4(&sm.phi[i * SP + (mt * 16 + sq)], v);
            }
            if constexpr (kPhiReg) phi_r[ti][tj] = v;
            if constexpr (kComp) comp[ti][tj] = cv;
        }
    if constexpr (NTL < NTK) {   // regions of skipped tiles are never written: zero once
        for (int e = tid; e < KP * SB; e += kThreads) sm.buf[e] = M::to_op(0.0f);
    }
    for (int e = tid; e < 3 * KP; e += kThreads) {
        const int v = e / KP, a = e % KP;
        sm.ybar[e] = (a < k) ? g.ybar[v * k + a] : 0.0f;
    }
    for (int e = tid; e < 2 * SP; e += kThreads) {
        const int v = e / SP, a = e % SP;
        sm.yfold[v * SP + (a ^ swz(k + v))] = M::to_op((a < k) ? g.ybar[v * k + a] : 0.0f);
    }
    // rows of the second operand of Phi^T Phi: component i, or a mean at k, k+1
    const Op* grow[TC];
#pragma unroll
    for (int tj = 0; tj < TC; ++tj) {
        const int i = (tj < TCL) ? (wc + WC * tj) * 16 + l16 : 0;
        grow[tj] = (mfold && (i == k || i == k + 1)) ? &sm.yfold[(i - k) * SP] : &sm.phi[i * SP];
    }
    // per-column factor of the update: 1 for a live component, 0 for padding
    float live[TC];
#pragma unroll
    for (int tj = 0; tj < TC; ++tj) live[tj] = ((wc + WC * tj) * 16 + l16 < k) ? 1.0f : 0.0f;

    // ---- batch prefetch state (NSTAGE > 0).  Row indices run two steps ahead
    // of the rows (their load has a whole step to arrive) and are checked only
    // where the rows are loaded, so no load waits right after it is issued.
    int32_t pidx[NCH];
    uint32_t plive = 0;                 // bit j: chunk j belongs to a row of the batch
    bool pperm = false;                 // the rows come from the permutation (else row0 + tr)
    int prow0 = 0;
    // (a loaded index is only ever read where the rows are loaded: selecting
    // between it and anything else right after the load would wait for it)
    typename M::Chunk pbuf[NSTAGE > 0 ? NSTAGE : 1][NCH];
    // when the thread count is a multiple of the chunks per row, all chunks of
    // a thread start at the same column a0t
    constexpr bool kA0Const = (kThreads % cpr) == 0;
    const int a0t = (tid % cpr) * M::CH;
    const u32x4 a0mask = M::chunk_mask(k - a0t);
    if constexpr (NSTAGE > 0 && kA0Const) {   // the parts of the staging area that are never written stay zero
        for (int e = tid; e < NSTAGE * MB * SY; e += kThreads) sm.ybatch[e] = M::to_op(0.0f);
    }
    // steps t >= end_step (up to t_end) are the scoring pass: rows in natural order
    const int t_end = g.end_step + ((SCORE && g.score != nullptr) ? g.spp : 0);
    auto issue_index = [&](int t) {
        if constexpr (NSTAGE > 0) {
            const bool train = !SCORE || t < g.end_step;   // without scoring every live step trains
            const bool live_step = t < t_end;
            const int pass = train ? t / g.spp : 0;
            const int row0 = train ? (t - pass * g.spp) * B : (live_step ? (t - g.end_step) * B : 0);
            const int nb = live_step ? min(B, n - row0) : 0;
            const int32_t* pp = (train && perms) ? perms + (size_t)pass * n + row0 : nullptr;
            plive = 0;
            pperm = pp != nullptr;
            prow0 = row0;
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int c = tid + j * kThreads;
                const int tr = c / cpr;
                if (c < MB * cpr && tr < nb) {
                    if (pp) pidx[j] = pp[tr];
                    plive |= 1u << j;
                }
            }
        }
    };
    auto issue_data = [&]() {
        // The rows of every chunk are chosen first and loaded after: a row
        // chosen after an earlier chunk's load was issued would make that
        // choice wait for the load (the wait counter drains in issue order).
        if constexpr (NSTAGE > 0 && kA0Const) {
            // every chunk of this thread starts at column a0t: threads past k
            // load nothing (their LDS columns stay zero), rows past the batch
            // size are never staged, and a row outside the batch loads row 0
            // (cleared at commit)
            int32_t rsel[NCH];
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int c = tid + j * kThreads;
                const bool live_c = (plive >> j) & 1u;
                const int32_t r = pperm ? pidx[j] : prow0 + c / cpr;
                const bool in_range = r >= 0 && r < n;
                if (live_c && !in_range) bad = true;   // out-of-range permutation entry: reads row 0, reported
                rsel[j] = (live_c && in_range) ? r : 0;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int c = tid + j * kThreads;
                if (c < MB * cpr && c / cpr < B && a0t < k && n > 0) {
#pragma unroll
                    for (int v = 0; v < NSTAGE; ++v)
                        pbuf[v][j] = *reinterpret_cast<const typename M::Chunk*>(Yv[v] + (size_t)rsel[j] * ldy + a0t);
                }
            }
        } else if constexpr (NSTAGE > 0) {
            int32_t rsel[NCH];
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int c = tid + j * kThreads;
                const bool live_c = (plive >> j) & 1u;
                int32_t r = pperm ? pidx[j] : prow0 + c / cpr;
                if (live_c && (r < 0 || r >= n)) {   // out-of-range permutation entry: reads row 0, reported
                    r = 0;
                    bad = true;
                }
                rsel[j] = r;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int c = tid + j * kThreads;
                const int a0 = (c % cpr) * M::CH;
                const bool live_c = (plive >> j) & 1u;
                // the columns past k of a row's last chunk are cleared at commit,
                // so nothing here waits for the load
#pragma unroll
                for (int v = 0; v < NSTAGE; ++v)
                    pbuf[v][j] = (live_c && a0 < k) ? *reinterpret_cast<const typename M::Chunk*>(
                                                          Yv[v] + (size_t)rsel[j] * ldy + a0)
                                                    : M::zero_chunk();
            }
        }
    };
    auto commit = [&](int nb) {
        if constexpr (NSTAGE > 0 && kA0Const) {
            // columns past k cleared with the thread's constant mask; rows past
            // nb of a short batch cleared as well
            auto store = [&](bool partial) {
#pragma unroll
                for (int j = 0; j < NCH; ++j) {
                    const int c = tid + j * kThreads;
                    const int tr = c / cpr;
                    if (c < MB * cpr && tr < B && a0t < k) {
#pragma unroll
                        for (int v = 0; v < NSTAGE; ++v) {
                            typename M::Chunk x = M::and_chunk(pbuf[v][j], a0mask);
                            if (partial && tr >= nb) x = M::zero_chunk();
                            *reinterpret_cast<typename M::Chunk*>(&sm.ybatch[(v * MB + tr) * SY + a0t]) = x;
                        }
                    }
                }
            };
            if (nb == B) store(false);   // a scalar branch: full batches skip the row test
            else store(true);
        } else if constexpr (NSTAGE > 0) {
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                const int c = tid + j * kThreads;
                if (c < MB * cpr) {
                    const int tr = c / cpr, a0 = (c % cpr) * M::CH;
#pragma unroll
                    for (int v = 0; v < NSTAGE; ++v)
                        *reinterpret_cast<typename M::Chunk*>(&sm.ybatch[(v * MB + tr) * SY + a0]) =
                            M::mask_chunk(pbuf[v][j], k - a0);
                }
            }
        }
    };
    issue_index(g.start_step);
    issue_data();
    issue_index(g.start_step + 1);
    // NSTAGE == 0: this thread's row index of the next step (thread tr < MB holds
    // row tr), loaded a step ahead: nperm says whether nrow holds it (else the
    // step's rows are in natural order)
    int32_t nrow = 0;
    bool nperm = false;
    auto next_row = [&](int tn) {
        const bool tr_train = !SCORE || tn < g.end_step;
        const int tpass = tr_train ? tn / g.spp : 0;
        const int ts = tr_train ? tn - tpass * g.spp : tn - g.end_step;
        const int trow0 = ts * B;
        nperm = tr_train && perms != nullptr;
        if (nperm && tn < t_end && tid < min(B, n - trow0)) nrow = perms[(size_t)tpass * n + trow0 + tid];
    };
    if constexpr (NSTAGE == 0) next_row(g.start_step);
    __syncthreads();

    double score_g = 0.0, score_t = 0.0;   // scoring pass: sum G^3 and sum T(phi, phi, phi), per lane
    // step size of the coming step; the next one is computed during the O
    // product, whose matrix cores leave the vector ALU idle
    float beta_t = g.beta0 / (1.0f + static_cast<float>(g.start_step) * g.inv_tau);
    for (int t = g.start_step; t < t_end; ++t) {
        const bool train = !SCORE || t < g.end_step;
        const int pass = train ? t / g.spp : 0;
        const int s = train ? t - pass * g.spp : t - g.end_step;
        const int row0 = s * B;
        const int nb = min(B, n - row0);
        const float beta = beta_t;

        // ================= phase 1: batch rows, G = Phi^T Phi -> G*G (and mA, mB)
        // (the plain BF16 variant writes the batch rows after the G product,
        // whose LDS reads then do not queue behind them: 2% off the step; the
        // others, with fuller registers, spill that way and write them first)
        if constexpr (kComp) commit(nb);
        if constexpr (NSTAGE == 0) {
            if (tid < nb) {
                int32_t r = nperm ? nrow : row0 + tid;
                if (r < 0 || r >= n) {   // out-of-range permutation entry: reads row 0, reported
                    r = 0;
                    bad = true;
                }
                sm.idx[tid] = r;
            }
        }
        if (!mfold) {
            // mA, mB on the vector ALU: thread (view v, column i, half h) sums half a dot product
            const int v = tid >> 8, rem = tid & 255, i = rem >> 1, h = rem & 1;
            float acc = 0.f;
            if (i < KP) {
                constexpr int half = KP >> 1;
                const Op* prow = &sm.phi[i * SP];
                const int psw = swz(i);
                const float* yb = &sm.ybar[v * KP + h * half];
#pragma unroll
                for (int a = 0; a < half; a += 8) {
                    float x[8];
                    if constexpr (M::EPL == 8) {
                        const bf16x8 pv = *reinterpret_cast<const bf16x8*>(prow + ((h * half + a) ^ psw));
#pragma unroll
                        for (int e = 0; e < 8; ++e) x[e] = M::op_to_f(pv[e]);
                    } else {
                        const f32x4 p0 = M::load4(prow + h * half + a), p1 = M::load4(prow + h * half + a + 4);
#pragma unroll
                        for (int e = 0; e < 4; ++e) { x[e] = p0[e]; x[e + 4] = p1[e]; }
                    }
                    const f32x4 y0 = *reinterpret_cast<const f32x4*>(yb + a);
                    const f32x4 y1 = *reinterpret_cast<const f32x4*>(yb + a + 4);
                    acc += x[0] * y0[0] + x[1] * y0[1] + x[2] * y0[2] + x[3] * y0[3] +
                           x[4] * y1[0] + x[5] * y1[1] + x[6] * y1[2] + x[7] * y1[3];
                }
            }
            acc = add_xor1(acc);
            if (h == 0 && i < KP) sm.m[v * KP + i] = acc;
        }
        if constexpr (kTri) {
            // one straight-line body per wave position: the tiles, the fragment
            // loads and the stores are all fixed at compile time
            auto gtri = [&](auto wrc, auto wcc) {
                constexpr int A = decltype(wrc)::value, C = decltype(wcc)::value;
                f32x4 acc[2][TC];
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
if constexpr (M::EPL == 1) {
#pragma unroll 1
                for (int s0 = 0; s0 < KQ; s0 += 4) {
                    f32x4 fa4[2], fb4[TC];
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti) {
                        bool need = false;
#pragma unroll
                        for (int tj = 0; tj < TC; ++tj) need = need || tri_tile(A, C, ti, tj, NTL, NTK);
                        fa4[ti] = need ? M::load4(&sm.phi[(tri_row(A, ti, NTK) * 16 + l16) * SP + q * KQ + s0])
                                       : f32x4{0.f, 0.f, 0.f, 0.f};
                    }
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj)
                        fb4[tj] = (tri_tile(A, C, 0, tj, NTL, NTK) || tri_tile(A, C, 1, tj, NTL, NTK))
                                      ? M::load4(grow[tj] + q * KQ + s0) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                            for (int tj = 0; tj < TC; ++tj)
                                if (tri_tile(A, C, ti, tj, NTL, NTK))
                                    acc[ti][tj] = M::mma(fa4[ti][e], fb4[tj][e], acc[ti][tj]);
                }
                } else {
#pragma unroll
                for (int k0 = 0; k0 < KP; k0 += M::KI) {
                    typename M::Frag fa[2], fb[TC];
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti) {
                        bool need = false;
#pragma unroll
                        for (int tj = 0; tj < TC; ++tj) need = need || tri_tile(A, C, ti, tj, NTL, NTK);
                        fa[ti] = need ? M::lds(&sm.phi[(tri_row(A, ti, NTK) * 16 + l16) * SP + (k0 + cq)])
                                      : M::zero_frag();
                    }
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj)
                        fb[tj] = (tri_tile(A, C, 0, tj, NTL, NTK) || tri_tile(A, C, 1, tj, NTL, NTK))
                                     ? M::lds(grow[tj] + (k0 + cq)) : M::zero_frag();
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                        for (int tj = 0; tj < TC; ++tj)
                            if (tri_tile(A, C, ti, tj, NTL, NTK)) acc[ti][tj] = M::mma(fa[ti], fb[tj], acc[ti][tj]);
                }
                }
                if constexpr (!kComp) commit(nb);
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) {
                        if (!tri_tile(A, C, ti, tj, NTL, NTK)) continue;
                        const int mt = tri_row(A, ti, NTK), nt = C + 2 * tj;
                        const int i = nt * 16 + l16;
                        const f32x4 gv = acc[ti][tj];
                        const f32x4 g2 = gv * gv;
                        M::store4(&sm.buf[i * SB + (mt * 16 + sq)], g2);
                        if (mfold && (i == k || i == k + 1))
                            *reinterpret_cast<f32x4*>(&sm.m[(i - k) * KP + mt * 16 + 4 * q]) = gv;
                        if (mt < nt) {
                            // the transposed tile: lanes 2m and 2m + 1 (columns 2m, 2m + 1)
                            // swap halves so that the even lane holds rows 4q, 4q + 1 and
                            // the odd one rows 4q + 2, 4q + 3 of both columns, each row
                            // pair one 4-byte store.  Its entries in the padding columns
                            // k, k + 1 (mA^2, mB^2, where the other tile has zeros) meet
                            // the zero rows k, k + 1 of Phi in O.
                            const bool odd = l16 & 1;
                            const float x0 = odd ? g2[0] : g2[2], x1 = odd ? g2[1] : g2[3];
                            const float y0 =
                                __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x0), 0xB1, 0xF, 0xF, false));
                            const float y1 =
                                __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x1), 0xB1, 0xF, 0xF, false));
                            const int j0 = mt * 16 + 4 * q + (odd ? 2 : 0);
                            const int c = (nt * 16 + (l16 & ~1)) ^ swz(j0);   // row j0 + 1: same permutation
                            if constexpr (M::EPL == 1) {
                                const float2 r0 = {odd ? y0 : g2[0], odd ? g2[2] : y0};
                                const float2 r1 = {odd ? y1 : g2[1], odd ? g2[3] : y1};
                                *reinterpret_cast<float2*>(&sm.buf[j0 * SB + c]) = r0;
                                *reinterpret_cast<float2*>(&sm.buf[(j0 + 1) * SB + c]) = r1;
                            } else {
                                bf16x2 r0, r1;
                                r0[0] = M::to_op(odd ? y0 : g2[0]);
                                r0[1] = M::to_op(odd ? g2[2] : y0);
                                r1[0] = M::to_op(odd ? y1 : g2[1]);
                                r1[1] = M::to_op(odd ? g2[3] : y1);
                                *reinterpret_cast<bf16x2*>(&sm.buf[j0 * SB + c]) = r0;
                                *reinterpret_cast<bf16x2*>(&sm.buf[(j0 + 1) * SB + c]) = r1;
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
            };
            // only the wave positions that reach this body (DR, DC) are instantiated
            const int pos = wr * 2 + wc;
            auto at = [&](auto wrc, auto wcc) {
                constexpr int A = decltype(wrc)::value, C = decltype(wcc)::value;
                if constexpr (((A + WR * (TRK - 1) >= NTL) == (DR == 1)) && ((C + WC * (TC - 1) >= NTL) == (DC == 1)))
                    if (pos == A * 2 + C) gtri(wrc, wcc);
            };
            at(IntC<0>{}, IntC<0>{});
            at(IntC<0>{}, IntC<1>{});
            at(IntC<1>{}, IntC<0>{});
            at(IntC<1>{}, IntC<1>{});
            at(IntC<2>{}, IntC<0>{});
            at(IntC<2>{}, IntC<1>{});
            at(IntC<3>{}, IntC<0>{});
            at(IntC<3>{}, IntC<1>{});
        } else {
            f32x4 acc[TRK][TC];
#pragma unroll
            for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
            if constexpr (M::EPL == 1) {
                // FP32 (one k per lane and instruction): lane group q takes the
                // k range [q KQ, (q + 1) KQ), so four consecutive k of a row are
                // one 16-byte LDS read (the order of the k sum is permuted)
#pragma unroll 1
                for (int s0 = 0; s0 < KQ; s0 += 4) {
                    f32x4 fa4[TRK], fb4[TC];
#pragma unroll
                    for (int ti = 0; ti < TRK; ++ti) {
                        const int mt = wr + WR * ti;
                        fa4[ti] = (ti < TRL) ? M::load4(&sm.phi[(mt * 16 + l16) * SP + q * KQ + s0])
                                             : f32x4{0.f, 0.f, 0.f, 0.f};
                    }
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj)
                        fb4[tj] = (tj < TCL) ? M::load4(grow[tj] + q * KQ + s0) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                            for (int tj = 0; tj < TC; ++tj)
                                if (ti < TRL && tj < TCL)
                                    acc[ti][tj] = M::mma(fa4[ti][e], fb4[tj][e], acc[ti][tj]);
                }
            } else {
#pragma unroll UNR
            for (int k0 = 0; k0 < KP; k0 += M::KI) {
                typename M::Frag fa[TRK], fb[TC];
#pragma unroll
                for (int ti = 0; ti < TRK; ++ti) {
                    const int mt = wr + WR * ti;
                    fa[ti] = (ti < TRL) ? M::lds(&sm.phi[(mt * 16 + l16) * SP + (k0 + cq)]) : M::zero_frag();
                }
#pragma unroll
                for (int tj = 0; tj < TC; ++tj)
                    fb[tj] = (tj < TCL) ? M::lds(grow[tj] + (k0 + cq)) : M::zero_frag();
#pragma unroll
                for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj)
                        if (ti < TRL && tj < TCL)
                            acc[ti][tj] = M::mma(fa[ti], fb[tj], acc[ti][tj]);
            }
            }
            if constexpr (!kComp) commit(nb);
            if (SCORE && t == g.end_step) {   // first scoring step: sum of G^3 over live entries
#pragma unroll
                for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) {
                        const int mt = wr + WR * ti, nt = wc + WC * tj;
                        if (ti >= TRL || tj >= TCL) continue;
                        const int i = nt * 16 + l16;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int j = mt * 16 + 4 * q + r;
                            const double gv = acc[ti][tj][r];
                            if (i < k && j < k) score_g += gv * gv * gv;
                        }
                    }
            }
            // G*G into the exchange buffer, column-major: buf[i*SB + j] = G[j][i]^2;
            // the columns k, k+1 of G give mA, mB when folded
#pragma unroll
            for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int mt = wr + WR * ti, nt = wc + WC * tj;
                    if (ti < TRL && tj < TCL) {
                        const int i = nt * 16 + l16;
                        const f32x4 gv = acc[ti][tj];
                        M::store4(&sm.buf[i * SB + (mt * 16 + sq)], gv * gv);
                        if (mfold && (i == k || i == k + 1))
                            *reinterpret_cast<f32x4*>(&sm.m[(i - k) * KP + mt * 16 + 4 * q]) = gv;
                    }
                }
        }
        __syncthreads();

        // ================= phase 2: O = Phi (G*G), applied to the master copy at once
        beta_t = g.beta0 / (1.0f + static_cast<float>(t + 1) * g.inv_tau);   // the next step's
        f32x4 oacc[TRK][TC];
#pragma unroll
        for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) oacc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (M::EPL == 1) {
            // FP32: permuted k as in G; G*G rows give 16-byte reads, the Phi
            // operand (a-major view of live components) stays one read per k
#pragma unroll 1
            for (int s0 = 0; s0 < KQ; s0 += 4) {
                const int kk = q * KQ + s0;
                f32x4 fb4[TC];
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int nt = wc + WC * tj;
                    fb4[tj] = (tj < TCL) ? M::load4(&sm.buf[(nt * 16 + l16) * SB + kk]) : f32x4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float fa1[TRK];
#pragma unroll
                    for (int ti = 0; ti < TRK; ++ti) {
                        const int mt = wr + WR * ti;
                        fa1[ti] = (ti < TRL && kk + e < k) ? sm.phi[(kk + e) * SP + mt * 16 + l16] : 0.0f;
                    }
#pragma unroll
                    for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                        for (int tj = 0; tj < TC; ++tj)
                            if (ti < TRL && tj < TCL)
                                oacc[ti][tj] = M::mma(fa1[ti], fb4[tj][e], oacc[ti][tj]);
                }
            }
        } else {
#pragma unroll UNR
        for (int k0 = 0; k0 < KP; k0 += M::KI) {
            typename M::Frag fa[TRK], fb[TC];
#pragma unroll
            for (int ti = 0; ti < TRK; ++ti) {
                const int mt = wr + WR * ti;
                if (ti < TRL) {
                    // Phi[a][i], a = 16 mt + lane % 16, i = k0 + EPL q + e, from the
                    // component-major copy
                    fa[ti] = kPerm ? M::lds_t_sw(&sm.phi[k0 * SP + mt * 16], SP, lane)
                                   : M::lds_t(&sm.phi[k0 * SP + mt * 16], SP, lane);
                } else {
                    fa[ti] = M::zero_frag();
                }
            }
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                const int nt = wc + WC * tj;
                fb[tj] = (tj < TCL) ? M::lds(&sm.buf[(nt * 16 + l16) * SB + (k0 + cq)]) : M::zero_frag();
            }
#pragma unroll
            for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj)
                    if (ti < TRL && tj < TCL)
                        oacc[ti][tj] = M::mma(fa[ti], fb[tj], oacc[ti][tj]);
        }
        }
        // -beta kappa O goes into the compensation term now (c <- c + beta
        // kappa O), so O is not live through the batch products; the single
        // compensated addition at the end of the step then adds the whole
        // increment beta (D - kappa O) to the master copy.  The LDS operand
        // copies keep the old Phi, which every product of this step reads.
        if (!SCORE || train) {
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                const float f3 = beta * live[tj] * g.kappa;
#pragma unroll
                for (int ti = 0; ti < TRK; ++ti) {
                    if (ti >= TRL || tj >= TCL) continue;
                    if constexpr (kComp) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) comp[ti][tj][r] = fmaf(f3, oacc[ti][tj][r], comp[ti][tj][r]);
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) phi_r[ti][tj][r] = fmaf(-f3, oacc[ti][tj][r], phi_r[ti][tj][r]);
                    }
                }
            }
        }
        __syncthreads();   // every read of G*G is done: the buffer takes Q next

        // rows of step t+1 start their trip from global memory now, then the
        // row indices of step t+2 (the plain BF16 one-view variant issues them
        // after its batch product instead, so that product's operand reads
        // are the first thing after the barrier: 1-2% off the step)
        constexpr bool kLateIssue = M::EPL != 1 && NSTAGE == 1 && !kComp;
        if constexpr (!kLateIssue) {
            issue_data();
            issue_index(t + 2);
        }
        if constexpr (NSTAGE == 0) next_row(t + 1);

        // ================= phase 3: PA, PB one tile row at a time -> Q into the
        // exchange buffer (buf[i*SB + t] = Q[t][i]) and column sums of H
        {
            // per column: Q = al*xa*xb - bmB*xa - bmA*xb with the padding mask folded in
            float colsum[TC];
            float al[TC], bmA[TC], bmB[TC];
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                colsum[tj] = 0.f;
                const int i = (wc + WC * tj) * 16 + l16;
                const float mA = (tj < TCL) ? sm.m[i] : 0.f;
                const float mB = (tj < TCL) ? sm.m[KP + i] : 0.f;
                al[tj] = g.a * live[tj];
                bmA[tj] = g.b * live[tj] * mA;
                bmB[tj] = g.b * live[tj] * mB;
            }
            if constexpr (M::EPL != 1 && NSTAGE == 1 && !kComp) {
                // BF16, one staged view, plain update: both batch tile rows of
                // the wave at once, so each Phi fragment is read from LDS once
                // per k step instead of once per tile row (measured 1.5% off
                // the k = 100 step; the compensated variant, with 32 more live
                // registers, was 2% slower this way and keeps the loop below)
                f32x4 pt[kTR][TC];
#pragma unroll
                for (int ti = 0; ti < kTR; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) pt[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll UNR_P
                for (int k0 = 0; k0 < KP; k0 += M::KI) {
                    typename M::Frag fphi[TC];
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) {
                        const int nt = wc + WC * tj;
                        fphi[tj] = (tj < TCL) ? M::lds(&sm.phi[(nt * 16 + l16) * SP + (k0 + cq)])
                                              : M::zero_frag();
                    }
#pragma unroll
                    for (int ti = 0; ti < kTR; ++ti) {
                        const int tr = (wr + WR * ti) * 16 + l16;
                        const typename M::Frag fa = M::lds(&sm.ybatch[tr * SY + k0 + q * M::EPL]);
#pragma unroll
                        for (int tj = 0; tj < TC; ++tj)
                            if (tj < TCL) pt[ti][tj] = M::mma(fa, fphi[tj], pt[ti][tj]);
                    }
                }
                issue_data();
                issue_index(t + 2);
#pragma unroll
                for (int ti = 0; ti < kTR; ++ti) {
                    const int mt = wr + WR * ti;
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) {
                        const int nt = wc + WC * tj;
                        if (tj >= TCL) continue;
                        const int i = nt * 16 + l16;
                        f32x4 qv;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {   // one view: xb = xa
                            const float xa = pt[ti][tj][r];
                            colsum[tj] = fmaf(xa, xa, colsum[tj]);
                            qv[r] = xa * fmaf(al[tj], xa, -(bmA[tj] + bmB[tj]));
                        }
                        M::store4(&sm.buf[i * SB + (mt * 16 + sq)], qv);
                    }
                }
            } else {
#pragma unroll
            for (int ti = 0; ti < kTR; ++ti) {
                const int mt = wr + WR * ti;
                const int tr = mt * 16 + l16;
                const Y* rowA = nullptr;
                const Y* rowB = nullptr;
                if constexpr (NSTAGE == 0) {
                    const bool ok = tr < nb;
                    rowA = ok ? Yv[0] + (size_t)sm.idx[tr] * ldy : nullptr;
                    rowB = ok ? Yv[1] + (size_t)sm.idx[tr] * ldy : nullptr;
                }
                const Y* sA = &sm.ybatch[tr * SY];
                const Y* sB = &sm.ybatch[((NSTAGE == 3 ? 1 : 0) * MB + tr) * SY];
                f32x4 pa[TC], pb[TC];
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    pa[tj] = f32x4{0.f, 0.f, 0.f, 0.f};
                    pb[tj] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
                if constexpr (M::EPL == 1) {
                    // FP32: lane group q takes the k range [q KQ, (q + 1) KQ), so
                    // four consecutive k of a row are one 16-byte read (as in G)
#pragma unroll 1
                    for (int s0 = 0; s0 < KQ; s0 += 4) {
                        const int kk = q * KQ + s0;
                        f32x4 fa4, fb4 = {0.f, 0.f, 0.f, 0.f};
                        if constexpr (NSTAGE == 0) {
                            fa4 = yrow4(rowA, kk, k);
                            if constexpr (!OV) fb4 = yrow4(rowB, kk, k);
                        } else {
                            fa4 = M::load4(sA + kk);
                            if constexpr (NSTAGE == 3) fb4 = M::load4(sB + kk);
                        }
                        f32x4 fp4[TC];
#pragma unroll
                        for (int tj = 0; tj < TC; ++tj) {
                            const int nt = wc + WC * tj;
                            fp4[tj] = (tj < TCL) ? M::load4(&sm.phi[(nt * 16 + l16) * SP + kk])
                                                 : f32x4{0.f, 0.f, 0.f, 0.f};
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e)
#pragma unroll
                            for (int tj = 0; tj < TC; ++tj) {
                                if (tj >= TCL) continue;
                                pa[tj] = M::mma(fa4[e], fp4[tj][e], pa[tj]);
                                if constexpr (NSTAGE != 1 && !OV) pb[tj] = M::mma(fb4[e], fp4[tj][e], pb[tj]);
                            }
                    }
                } else {
#pragma unroll UNR_P
                for (int k0 = 0; k0 < KP; k0 += M::KI) {
                    typename M::Frag fa, fbv;
                    if constexpr (NSTAGE == 0) {
                        fa = M::yrow(rowA, k0 + q * M::EPL, k);
                        fbv = M::yrow(rowB, k0 + q * M::EPL, k);
                    } else {
                        fa = M::lds(sA + k0 + q * M::EPL);
                        if constexpr (NSTAGE == 3) fbv = M::lds(sB + k0 + q * M::EPL);
                    }
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) {
                        const int nt = wc + WC * tj;
                        if (tj < TCL) {
                            const typename M::Frag fphi = M::lds(&sm.phi[(nt * 16 + l16) * SP + (k0 + cq)]);
                            pa[tj] = M::mma(fa, fphi, pa[tj]);
                            if constexpr (NSTAGE != 1) pb[tj] = M::mma(fbv, fphi, pb[tj]);
                        }
                    }
                }
                }
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int nt = wc + WC * tj;
                    if (tj >= TCL) continue;
                    const int i = nt * 16 + l16;
                    f32x4 qv;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float xa = pa[tj][r];
                        if constexpr (NSTAGE == 1) {   // one view: xb = xa
                            colsum[tj] = fmaf(xa, xa, colsum[tj]);
                            qv[r] = xa * fmaf(al[tj], xa, -(bmA[tj] + bmB[tj]));
                        } else {
                            const float xb = OV ? xa : pb[tj][r];   // one view: P_B = P_A
                            colsum[tj] = fmaf(xa, xb, colsum[tj]);
                            qv[r] = fmaf(xa, fmaf(al[tj], xb, -bmB[tj]), -bmA[tj] * xb);
                        }
                    }
                    M::store4(&sm.buf[i * SB + (mt * 16 + sq)], qv);
                }
            }
            }
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                const int nt = wc + WC * tj;
                if (tj >= TCL) continue;
                colsum[tj] = add_xor16(colsum[tj]);
                colsum[tj] = add_xor32(colsum[tj]);
                if (q == 0) sm.s[wr * KP + nt * 16 + l16] = colsum[tj];
            }
        }
        if constexpr (SM::kStageCT) {
            // YC batch into LDS, a-major: yct[a*SB + t] (zero outside the batch and k)
            for (int e = tid; e < MB * KP; e += kThreads) {
                const int tr = e / KP, a = e % KP;
                const Y v = (tr < nb && a < k) ? Yv[2][(size_t)sm.idx[tr] * ldy + a] : M::to_op(0.0f);
                sm.yct[a * SB + tr] = v;
            }
        }
        __syncthreads();

        // ================= phase 4: D = YC^T Q (+ rank one), update Phi
        {
            constexpr int vc = (NSTAGE == 3) ? 2 : 0;
            f32x4 dacc[TRK][TC];
#pragma unroll
            for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) dacc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
if constexpr (M::EPL == 1 && NSTAGE > 0) {
                // FP32 with staged rows: lane group q takes the batch rows
                // [q MB/4, (q + 1) MB/4), so Q's rows give 16-byte reads; the YC
                // operand stays one read per row (rows read from L2 instead keep
                // the loop below, whose iterations overlap their latency)
                constexpr int KQB = MB / 4;
#pragma unroll 1
                for (int s0 = 0; s0 < KQB; s0 += 4) {
                    const int tt = q * KQB + s0;
                    f32x4 fb4[TC];
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj) {
                        const int nt = wc + WC * tj;
                        fb4[tj] = (tj < TCL) ? M::load4(&sm.buf[(nt * 16 + l16) * SB + tt]) : f32x4{0.f, 0.f, 0.f, 0.f};
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int tr = tt + e;
                        float fa1[TRK];
#pragma unroll
                        for (int ti = 0; ti < TRK; ++ti) {
                            const int mt = wr + WR * ti;
                            const int a = mt * 16 + l16;
                            if (ti >= TRL) {
                                fa1[ti] = 0.0f;
                            } else if constexpr (NSTAGE > 0) {
                                fa1[ti] = sm.ybatch[(vc * MB + tr) * SY + a];
                            } else {
                                fa1[ti] = (a < k && tr < nb) ? Yv[2][(size_t)sm.idx[tr] * ldy + a] : 0.0f;
                            }
                        }
#pragma unroll
                        for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                            for (int tj = 0; tj < TC; ++tj)
                                if (ti < TRL && tj < TCL)
                                    dacc[ti][tj] = M::mma(fa1[ti], fb4[tj][e], dacc[ti][tj]);
                    }
                }
            } else {
            auto dstep = [&](const int k0) {
                typename M::Frag fa[TRK], fb[TC];
#pragma unroll
                for (int ti = 0; ti < TRK; ++ti) {
                    const int mt = wr + WR * ti;
                    const int a = mt * 16 + l16;
                    if (ti >= TRL) {
                        fa[ti] = M::zero_frag();
                    } else if constexpr (NSTAGE > 0) {
                        // EPL rows t = k0 + EPL*q + e of column a of the staged batch
                        if constexpr (M::EPL == 1) {
                            fa[ti] = sm.ybatch[(vc * MB + k0 + q) * SY + a];
                        } else {
                            fa[ti] = M::lds_t(&sm.ybatch[(vc * MB + k0) * SY + mt * 16], SY, lane);
                        }
                    } else if constexpr (SM::kStageCT) {
                        fa[ti] = M::lds(&sm.yct[a * SB + k0 + q * M::EPL]);
                    } else {
                        const int tr = k0 + q;
                        fa[ti] = (a < k && tr < nb) ? Yv[2][(size_t)sm.idx[tr] * ldy + a] : 0.0f;
                    }
                }
#pragma unroll
                for (int tj = 0; tj < TC; ++tj) {
                    const int nt = wc + WC * tj;
                    fb[tj] = (tj < TCL) ? M::lds(&sm.buf[(nt * 16 + l16) * SB + (k0 + cq)]) : M::zero_frag();
                }
#pragma unroll
                for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TC; ++tj)
                        if (ti < TRL && tj < TCL)
                            dacc[ti][tj] = M::mma(fa[ti], fb[tj], dacc[ti][tj]);
            };
            if constexpr (M::EPL == 1 && NSTAGE == 0) {
                // FP32 rows read from global memory: the batch rows past the batch
                // size are zero, so the contraction stops at the first multiple of
                // KI past them (the products it skips add exact zeros; FP32 k = 100
                // 32.9 -> 31.7 us per step)
                const int dlim = (nb + M::KI - 1) / M::KI * M::KI;
                for (int k0 = 0; k0 < dlim; k0 += M::KI) dstep(k0);
            } else {
#pragma unroll UNR
                for (int k0 = 0; k0 < MB; k0 += M::KI) dstep(k0);
            }
            }
            const float invB = 1.0f / static_cast<float>(nb);
#pragma unroll
            for (int tj = 0; tj < TC; ++tj) {
                const int nt = wc + WC * tj;
                if (tj >= TCL) continue;
                const int i = nt * 16 + l16;
                float ssum = 0.f;
#pragma unroll
                for (int u = 0; u < WR; ++u) ssum += sm.s[u * KP + i];
                const float rv = g.c * sm.m[i] * sm.m[KP + i] - g.b * ssum * invB;
                if (SCORE && !train) {   // scoring: phi_i . D_i, weighted by the batch's share of rows
                    float part = 0.f;
#pragma unroll
                    for (int ti = 0; ti < TRK; ++ti) {
                        const int mt = wr + WR * ti;
                        if (ti >= TRL) continue;
                        const f32x4 ybc = *reinterpret_cast<const f32x4*>(&sm.ybar[2 * KP + mt * 16 + 4 * q]);
                        const f32x4 pv = phi_get(ti, tj);
#pragma unroll
                        for (int r = 0; r < 4; ++r) part = fmaf(pv[r], fmaf(dacc[ti][tj][r], invB, ybc[r] * rv), part);
                    }
                    score_t += static_cast<double>(nb) / static_cast<double>(n) * static_cast<double>(part * live[tj]);
                    continue;
                }
                // delta = beta*live*(dacc/B + ybarC*rv), folded per column; the
                // compensation term already holds +beta*kappa*O
                const float bl = beta * live[tj];
                const float f1 = bl * invB, f2 = bl * rv;
#pragma unroll
                for (int ti = 0; ti < TRK; ++ti) {
                    const int mt = wr + WR * ti;
                    if (ti >= TRL) continue;
                    const f32x4 ybc = *reinterpret_cast<const f32x4*>(&sm.ybar[2 * KP + mt * 16 + 4 * q]);
                    f32x4 v = phi_get(ti, tj);
                    if constexpr (kComp) {
                        f32x4 cv = comp[ti][tj];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            // Kahan step; cmask = 0 turns it into the plain update
                            const float y = fmaf(f1, dacc[ti][tj][r], fmaf(f2, ybc[r], -cv[r]));
                            const float tt = v[r] + y;
                            cv[r] = ((tt - v[r]) - y) * cmask;
                            v[r] = tt;
                        }
                        comp[ti][tj] = cv;
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) v[r] += fmaf(f1, dacc[ti][tj][r], f2 * ybc[r]);
                    }
                    if constexpr (kPhiReg) phi_r[ti][tj] = v;
                    M::store4(&sm.phi[i * SP + (mt * 16 + sq)], v);
                }
            }
            if (train && (s == g.spp - 1 || t + 1 == g.end_step)) {
                // non-finite values propagate through every later step, so one
                // check per pass (and at the end of the run) sees any of them
#pragma unroll
                for (int tj = 0; tj < TC; ++tj)
#pragma unroll
                    for (int ti = 0; ti < TRK; ++ti) {
                        if (ti >= TRL || tj >= TCL) continue;
                        const f32x4 pv = phi_get(ti, tj);
#pragma unroll
                        for (int r = 0; r < 4; ++r) bad |= !isfinite(pv[r]);
                    }
            }
            if (Snap != nullptr && train && s == g.spp - 1) {   // end of a pass: Phi to the snapshot of this pass
#pragma unroll
                for (int tj = 0; tj < TC; ++tj)
#pragma unroll
                    for (int ti = 0; ti < TRK; ++ti) {
                        const int mt = wr + WR * ti, nt = wc + WC * tj;
                        if (ti >= TRL || tj >= TCL) continue;
                        const int i = nt * 16 + l16;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int a = mt * 16 + 4 * q + r;
                            if (a < k && i < k) Snap[(size_t)pass * k * k + (size_t)i * k + a] = phi_get(ti, tj)[r];
                        }
                    }
            }
        }
        if constexpr (NSTAGE == 0) {
            // the rows of step t+1 (indices loaded in phase 3) start their trip
            // into L2 now: one 4-byte direct-to-LDS load per 128-byte line of
            // each row, whose data lands in a scratch area nobody reads; the
            // products of the next step then read them from L2, not HBM
            const int tn = t + 1;
            const bool tr_train = !SCORE || tn < g.end_step;
            const int tpass = tr_train ? tn / g.spp : 0;
            const int trow0 = (tr_train ? tn - tpass * g.spp : tn - g.end_step) * B;
            if (tn < t_end && tid < min(B, n - trow0)) {
                const int r = nperm ? nrow : trow0 + tid;
                if (r >= 0 && r < n) {
                    constexpr int kLineElems = 128 / static_cast<int>(sizeof(Y));
                    const int nv = (Yv[1] == Yv[0] && Yv[2] == Yv[0]) ? 1 : 3;
                    for (int v = 0; v < nv; ++v)
                        for (int c = 0; c < k; c += kLineElems)
                            __builtin_amdgcn_global_load_lds(
                                (__attribute__((address_space(1))) void*)(Yv[v] + (size_t)r * ldy + c),
                                (__attribute__((address_space(3))) void*)(&sm.pf[w * 64]), 4, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    if constexpr (NSTAGE == 0) __builtin_amdgcn_s_waitcnt(0);   // the prefetches land before the wave ends

    if constexpr (SCORE) {
        if (g.score != nullptr) {
            double v = score_g - 2.0 * score_t;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) sm.red[w] = v;
            __syncthreads();
            if (tid == 0) {
                double tot = 0.0;
                for (int u = 0; u < kWaves; ++u) tot += sm.red[u];
                g.score[r_id] = tot;
            }
        }
    }
    // ---- write back the master copy (and compensation)
#pragma unroll
    for (int ti = 0; ti < TRK; ++ti)
#pragma unroll
        for (int tj = 0; tj < TC; ++tj) {
            const int mt = wr + WR * ti, nt = wc + WC * tj;
            if (ti >= TRL || tj >= TCL) continue;
            const int i = nt * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = mt * 16 + 4 * q + r;
                if (a < k && i < k) {
                    Phi[(size_t)i * k + a] = phi_get(ti, tj)[r];
                    if constexpr (kComp) {
                        if (Comp) Comp[(size_t)i * k + a] = g.compensated ? comp[ti][tj][r] : 0.0f;
                    } else {
                        if (Comp) Comp[(size_t)i * k + a] = 0.0f;
                    }
                }
            }
        }
    if (bad && g.nonfinite) *g.nonfinite = 1;
}


// One whole run of restart r_id of the problem in g, by the calling workgroup:
// each wave runs the body specialised for how many of its tile rows and
// columns it computes, so no tile guard is left inside the product loops
// (with the guards as run-time branches, FP32 KP = 112 spilled 64 bytes per
// lane and took 41.5 us per k = 100 step against 39.3; BF16 KP = 96 with
// three views 5.54 against 4.97 us).  NTL < KP / 16 (BF16, when k + 2 fits
// in fewer tiles than KP holds) also drops the tiles that hold only padding:
// BF16 k = 100 at KP = 128 computes 7 x 7 output tiles per product instead
// of 8 x 8 (4.80 -> 4.23 us per step).  OV (one view, rows read from global
// memory) computes the batch product once, since P_B = P_A (FP32 k = 100:
// 39.1 -> 32.9 us per step; k = 128: 48.8 -> 40.5).  Every result is the
// same bit for bit.
template <class M, int KP, int NSTAGE, int WR, bool SCORE, bool COMP = true, int NTL = KP / 16, bool OV = false>
__device__ __forceinline__ void sgd_body(const SgdArgs& g, const int r_id, SgdSmem<M, KP, NSTAGE, WR>& sm) {
    constexpr int WC = kWaves / WR, NTK = KP / 16;
    constexpr int TC = (NTK + WC - 1) / WC, TRK = (NTK + WR - 1) / WR;
    static_assert(NTL >= 1 && NTL <= NTK, "live tiles within KP");
    constexpr bool kCanDR = WR * (TRK - 1) + (WR - 1) >= NTL;   // some wave's last tile row lies outside
    constexpr bool kCanDC = WC * (TC - 1) + (WC - 1) >= NTL;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) & (kWaves - 1);
    int wr, wc;
    wave_grid<WR>(w, wr, wc);
    const bool dr = kCanDR && wr + WR * (TRK - 1) >= NTL;
    const bool dc = kCanDC && wc + WC * (TC - 1) >= NTL;
    if constexpr (kCanDR && kCanDC) {
        if (dr && dc) sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 1, 1, OV>(g, r_id, sm);
        else if (dr) sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 1, 0, OV>(g, r_id, sm);
        else if (dc) sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 0, 1, OV>(g, r_id, sm);
        else sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 0, 0, OV>(g, r_id, sm);
    } else if constexpr (kCanDR) {
        if (dr) sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 1, 0, OV>(g, r_id, sm);
        else sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 0, 0, OV>(g, r_id, sm);
    } else if constexpr (kCanDC) {
        if (dc) sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 0, 1, OV>(g, r_id, sm);
        else sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 0, 0, OV>(g, r_id, sm);
    } else {
        sgd_body_t<M, KP, NSTAGE, WR, SCORE, COMP, NTL, 0, 0, OV>(g, r_id, sm);
    }
}

// Host: the scalar part of the arguments shared by every entry point.  The
// pointers are set by the caller.  Returns OTM_OK or a status with a message.
inline int fill_scalars(int32_t n, int32_t k, int32_t ldy, double alpha0, const otm_sgd_params* p,
                        int64_t start_step, int64_t end_step, SgdArgs& a) {
    OTM_REQUIRE(k >= 1 && p->batch >= 1 && n >= 1 && p->passes >= 1, OTM_ESHAPE,
                "k, batch, n and passes must be positive");
    OTM_REQUIRE(k <= kMaxK, OTM_ECAPACITY, "k exceeds the compiled capacity (128)");
    OTM_REQUIRE(p->batch <= kMaxBatch, OTM_ECAPACITY, "batch exceeds the compiled capacity (128)");
    OTM_REQUIRE(ldy >= k, OTM_ESHAPE, "ldy < k");
    OTM_REQUIRE(p->y_dtype == OTM_F32 || p->y_dtype == OTM_BF16, OTM_EDTYPE, "y_dtype must be F32 or BF16");
    OTM_REQUIRE(p->y_dtype != OTM_BF16 || ldy % 8 == 0, OTM_ESHAPE, "BF16 rows need ldy % 8 == 0");
    OTM_REQUIRE(p->y_dtype != OTM_F32 || ldy % 4 == 0, OTM_ESHAPE, "F32 rows need ldy % 4 == 0");
    OTM_REQUIRE(p->beta_tau > 0.0, OTM_EINVAL, "beta_tau must be positive");
    OTM_REQUIRE(std::isfinite(p->beta0) && std::isfinite(alpha0) && std::isfinite(p->theta) && alpha0 >= 0.0,
                OTM_EINVAL, "alpha0, beta0, theta must be finite, alpha0 >= 0");
    a.n = n; a.k = k; a.batch = p->batch; a.passes = p->passes; a.ldy = ldy;
    a.compensated = p->compensated ? 1 : 0;
    const int64_t spp = (n + p->batch - 1) / p->batch;
    const int64_t total = spp * p->passes;
    OTM_REQUIRE(total + spp < (int64_t(1) << 31), OTM_ECAPACITY, "(passes + 1) * ceil(n / batch) must be < 2^31");
    const int64_t end = end_step < 0 ? total : end_step;
    OTM_REQUIRE(start_step >= 0 && start_step <= end && end <= total, OTM_ESHAPE,
                "need 0 <= start_step <= end_step <= passes * ceil(n / batch)");
    a.spp = static_cast<int32_t>(spp);
    a.start_step = static_cast<int32_t>(start_step);
    a.end_step = static_cast<int32_t>(end);
    a.a = static_cast<float>((alpha0 + 1.0) * (alpha0 + 2.0) / 2.0);
    a.b = static_cast<float>(alpha0 * (alpha0 + 1.0) / 2.0);
    a.c = static_cast<float>(alpha0 * alpha0);
    a.kappa = static_cast<float>(0.5 * (1.0 + p->theta));
    a.beta0 = static_cast<float>(p->beta0);
    a.inv_tau = static_cast<float>(1.0 / p->beta_tau);
    return OTM_OK;
}

}  // namespace
}  // namespace otm
