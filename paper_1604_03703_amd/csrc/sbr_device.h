// sbr_device.h -- device-side building blocks shared by the SBR kernels
// (gfx950 / CDNA4, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

typedef double sbr_d4 __attribute__((ext_vector_type(4)));
typedef float sbr_f4 __attribute__((ext_vector_type(4)));

// Compute-type traits: FP64 tiles use v_mfma_f64_16x16x4_f64, the FP32 form
// uses v_mfma_f32_16x16x4_f32 (operands rounded to FP32 when staged, FP32
// accumulation, the result added into FP64 storage by the caller).
//
// Operand / result lane layout of the 16x16x4 single-block instructions
// (measured on gfx950):
//   A operand (16 x 4): lane l holds A[l % 16][l / 16]
//   B operand (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16):        lane l, element r holds D[out_row(l, r)][l % 16] with
//                       out_row = 4 r + l / 16 for f64, 4 (l / 16) + r for f32.
template <typename CT> struct Mfma;
template <> struct Mfma<double> {
    typedef sbr_d4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
    typedef sbr_f4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int SBR_BK = 16;   // K extent of one LDS-staged chunk

// Which of (row, k) is the fastest-varying index when a thread block copies an
// (ROWS x SBR_BK) operand tile from global memory: pick the one that is
// contiguous in memory so the loads coalesce.
template <int ROWS, int NT, bool KFAST>
struct TileMap {
    static constexpr int E = ROWS * SBR_BK / NT;   // elements per thread
    static_assert(E >= 1 && E * NT == ROWS * SBR_BK, "tile / thread mismatch");
    static __device__ __forceinline__ void coords(int t, int e, int& row, int& k) {
        const int idx = t + e * NT;
        if (KFAST) { k = idx % SBR_BK; row = idx / SBR_BK; }
        else       { row = idx % ROWS; k = idx / ROWS; }
    }
};

// Block-level MFMA tile engine: C tile (BM x BN) += op(A) tile (BM x K) *
// op(B) tile (K x BN), K streamed through LDS in SBR_BK chunks.
//   LDS operand layouts: As[k * LDA + i] = op(A)(i, k), Bs[k * LDB + j] = op(B)(k, j).
// The MFMA "A" operand is taken from op(B) and the "B" operand from op(A), so
// the instruction computes C^T tiles: a lane's accumulator elements then lie
// along one column of C with consecutive lanes on consecutive rows, which
// makes column-major stores of C coalesce.
// Waves are arranged WM x WN; wave (wm, wn) owns C rows [wm*WTM, +WTM) and
// columns [wn*WTN, +WTN).  Accumulator acc[tn][tm][r] holds
//   C(wm*WTM + tm*16 + (lane & 15), wn*WTN + tn*16 + Mfma<CT>::out_row(lane, r)).
template <typename CT, int BM, int BN, int WM, int WN, int PAD = 2, bool PF = true>
struct TileEngine {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int WTM = BM / WM, WTN = BN / WN;
    static constexpr int TM = WTM / 16, TN = WTN / 16;
    static constexpr int LDA = BM + PAD, LDB = BN + PAD;   // LDS row strides (elements)
    static_assert(TM >= 1 && TN >= 1 && TM * 16 * WM == BM && TN * 16 * WN == BN, "bad tile shape");
    typedef typename Mfma<CT>::acc_t acc_t;
    acc_t acc[TN][TM];

    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int a = 0; a < TN; ++a)
#pragma unroll
            for (int b = 0; b < TM; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    }

    // One LDS chunk (SBR_BK deep, four k-steps).  PF: the operands of step
    // s + 1 are read before the products of step s are issued (a scheduling
    // barrier keeps the compiler from sinking the reads back below them), so
    // the LDS latency of a step hides behind the matrix instructions of the
    // previous one, for 2 (TM + TN) more registers.
    __device__ __forceinline__ void chunk(const CT* As, const CT* Bs, int wm, int wn, int lane) {
        const int kr = lane >> 4, c = lane & 15;
        constexpr int KS = SBR_BK / 4;
        CT p[2][TN], q[2][TM];
        auto read = [&](int s, int slot) {
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) p[slot][tn] = Bs[(4 * s + kr) * LDB + wn * WTN + tn * 16 + c];
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) q[slot][tm] = As[(4 * s + kr) * LDA + wm * WTM + tm * 16 + c];
        };
        if constexpr (PF) {
            read(0, 0);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s + 1 < KS) read(s + 1, (s + 1) & 1);
                __builtin_amdgcn_sched_barrier(0);
                products(p[s & 1], q[s & 1]);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                read(s, 0);
                products(p[0], q[0]);
            }
        }
    }

    // The chunk with the scheduler fenced between k-steps: the operand reads
    // of a step are not hoisted above the products of the previous one (no
    // more registers live than one step's operands).
    __device__ __forceinline__ void chunk_fenced(const CT* As, const CT* Bs, int wm, int wn, int lane) {
        const int kr = lane >> 4, c = lane & 15;
        constexpr int KS = SBR_BK / 4;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            CT p[TN], q[TM];
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) p[tn] = Bs[(4 * s + kr) * LDB + wn * WTN + tn * 16 + c];
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) q[tm] = As[(4 * s + kr) * LDA + wm * WTM + tm * 16 + c];
            products(p, q);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    __device__ __forceinline__ void products(const CT (&p)[TN], const CT (&q)[TM]) {
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) acc[tn][tm] = Mfma<CT>::mma(p[tn], q[tm], acc[tn][tm]);
    }

    static __device__ __forceinline__ int row_of(int wm, int tm, int lane) { return wm * WTM + tm * 16 + (lane & 15); }
    static __device__ __forceinline__ int col_of(int wn, int tn, int lane, int r) {
        return wn * WTN + tn * 16 + Mfma<CT>::out_row(lane, r);
    }
};

// Raw buffer loads for operand staging.  A buffer resource covers
// num_records bytes from its base; a load whose (per-lane) offset is at or
// beyond that range returns zero instead of touching memory, so a lane whose
// element lies outside the matrix gets the offset SBR_BUF_OOB and needs no
// branch.  Offsets are 32-bit byte offsets from a base that the caller moves
// per chunk (uniform across the block).
constexpr uint32_t SBR_BUF_OOB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t sbr_buffer(const void* base, uint32_t bytes) {
    // dword 3 of the descriptor: 32-bit data format, no swizzle (gfx9 family)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double sbr_buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float sbr_buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// 1 / q for a normal q: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - q r) (each roughly squares the
// relative error), which leaves an error of about one ulp at a third of the
// cost of a correctly rounded division.
__device__ __forceinline__ double sbr_recip(double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(fma(-q, r, 1.0), r, r);
    r = fma(fma(-q, r, 1.0), r, r);
    return r;
}

// 1/sqrt(a) for a normal a > 0: the hardware estimate refined by two Newton
// steps y <- y + y (1 - a y^2) / 2 (each roughly doubles the correct bits),
// about one ulp like sbr_recip.
__device__ __forceinline__ double sbr_rsqrt(double a) {
    double y = __builtin_amdgcn_rsq(a);
    y = fma(0.5 * y, fma(-a, y * y, 1.0), y);
    y = fma(0.5 * y, fma(-a, y * y, 1.0), y);
    return y;
}

// Sturm count of T - x I by the three-term recurrence of the leading
// principal minors, p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2} (p_0 = 1,
// e_0 = 0): the number of eigenvalues below x is the number of sign changes
// along p_0, ..., p_n (an exact zero counts by its sign bit, which gives the
// same total over two steps as Kahan's guard).  The data are scaled by a power
// of two so that |d_i - x| <= 1 and e^2 <= 1/4, so the larger of two
// consecutive minors grows by at most 1.25 a step; every U steps both are
// rescaled by a power of two (no rounding), so nothing overflows.  If the
// pair falls below 2^-600 at a block end (a split with x on an eigenvalue of
// the leading block, or couplings near underflow), some step of the block may
// have lost accuracy to underflow: `low` is set and the caller recounts with
// the guarded ratio recurrence.  Otherwise the count is exact for T with each
// d_i - x and e^2 perturbed by a few ulps, the same backward error as the
// ratio form (Barth, Martin and Wilkinson's scaled form of the recurrence).
// A step is three FP64 operations and one bit append, against a division or
// a refined reciprocal, a guard and a compare in the ratio form.
struct SturmChain {
    double pm, pc;   // p_{i-2}, p_{i-1}
    unsigned bits;   // sign bits of the current block, newest in bit 0, the last sign before it above them
    int cnt;
    bool low;

    __device__ __forceinline__ void start() {
        pm = 0.0;
        pc = 1.0;
        bits = 0u;
        cnt = 0;
        low = false;
    }
    // one step inside a block: dx = d_i - x, e2 = e_{i-1}^2 (scaled)
    __device__ __forceinline__ void step(double dx, double e2) {
        const double pn = fma(dx, pc, -(e2 * pm));
        pm = pc;
        pc = pn;
        bits = __builtin_amdgcn_alignbit(bits, (unsigned)__double2hiint(pn), 31u);   // (bits << 1) | sign
    }
    // end of a block of U steps: count its sign changes, rescale the pair
    template <int U>
    __device__ __forceinline__ void close_block() {
        static_assert(U >= 1 && U <= 31, "block length");
        cnt += __builtin_popcount((bits ^ (bits >> 1)) & ((1u << U) - 1u));
        bits &= 1u;
        const double m = fmax(fabs(pm), fabs(pc));
        low |= !(m >= 0x1p-600);
        const int ex = __builtin_amdgcn_frexp_exp(m);
        pm = __builtin_amdgcn_ldexp(pm, -ex);
        pc = __builtin_amdgcn_ldexp(pc, -ex);
    }
    // a step after the last full block (bits holds the last sign in bit 0)
    __device__ __forceinline__ void step_tail(double dx, double e2) {
        const double pn = fma(dx, pc, -(e2 * pm));
        pm = pc;
        pc = pn;
        const unsigned sg = (unsigned)__double2hiint(pn) >> 31;
        cnt += (int)(sg ^ bits);
        bits = sg;
    }
    __device__ __forceinline__ void finish() { low |= !(fmax(fabs(pm), fabs(pc)) >= 0x1p-600); }
};

// The ratio form q_i = (d_i - x) - e_{i-1}^2 / q_{i-1} with a correctly
// rounded division and Kahan's guard (|q| < pivmin -> -pivmin), counting the
// negative pivots: the recount for a chain whose scaled minors came near
// underflow.  On the scaled data pivmin = DBL_MIN keeps e^2 / q finite.
struct SturmRatio {
    double q;
    int cnt;
    __device__ __forceinline__ void start() {
        q = 1.0;
        cnt = 0;
    }
    __device__ __forceinline__ void step(double dx, double e2) {
        double v = dx - e2 / q;
        if (fabs(v) < DBL_MIN) v = -DBL_MIN;
        q = v;
        cnt += (v < 0.0);
    }
};

// Power of two 2^-E with w 2^-E in [1/2, 1): the scale of the Sturm data for
// a Gershgorin interval of width w > 0.
__device__ __forceinline__ double sturm_scale(double w) {
    return __builtin_amdgcn_ldexp(1.0, -__builtin_amdgcn_frexp_exp(w));
}

// Sum of N values by pairs (a tree of depth log2 N instead of a chain of N).
template <int N>
__device__ __forceinline__ double tree_sum(const double* v) {
    if constexpr (N == 1) {
        return v[0];
    } else {
        return tree_sum<N / 2>(v) + tree_sum<N - N / 2>(v + N / 2);
    }
}

// Agent-scope flag helpers for the pipelined chase schedule.
__device__ __forceinline__ int sbr_load_acquire(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void sbr_store_release(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Move a double across lanes with a DPP control (two 32-bit halves).  Only
// full permutations are used (quad_perm, row_half_mirror, row_mirror), so no
// lane reads an invalid source and no fallback value is needed.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Sum over the TPC lanes of an aligned group (TPC in {2, 4, 8, 16}):
// quad_perm(1,0,3,2) = lane ^ 1, quad_perm(2,3,0,1) = lane ^ 2,
// row_half_mirror = lane i <-> 7 - i inside each 8-lane half row,
// row_mirror = lane i <-> 15 - i inside each 16-lane row.
template <int TPC>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(TPC == 2 || TPC == 4 || TPC == 8 || TPC == 16, "group size");
    v += dpp_d<0xB1>(v);
    if constexpr (TPC >= 4) v += dpp_d<0x4E>(v);
    if constexpr (TPC >= 8) v += dpp_d<0x141>(v);
    if constexpr (TPC >= 16) v += dpp_d<0x140>(v);
    return v;
}

// Small dense product done cooperatively by NT threads: every output
// (i, j) in [0, M) x [0, N) gets sum_{k < K} A(i, k) B(k, j), handed to
// store(i, j, value).  Each thread computes RM x RN register blocks, so an
// operand element read from memory feeds RN (or RM) fused multiply-adds.
template <int M, int N, int K, int RM, int RN, int NT, class FA, class FB, class FS>
__device__ __forceinline__ void block_gemm(int t, const FA& A, const FB& B, const FS& store) {
    static_assert(M % RM == 0 && N % RN == 0, "register block must divide the product");
    constexpr int BM = M / RM, NB = BM * (N / RN);
    for (int blk = t; blk < NB; blk += NT) {
        const int i0 = (blk % BM) * RM, j0 = (blk / BM) * RN;
        double acc[RM][RN];
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int c = 0; c < RN; ++c) acc[r][c] = 0.0;
#pragma unroll 4
        for (int k = 0; k < K; ++k) {
            double av[RM], bv[RN];
#pragma unroll
            for (int r = 0; r < RM; ++r) av[r] = A(i0 + r, k);
#pragma unroll
            for (int c = 0; c < RN; ++c) bv[c] = B(k, j0 + c);
#pragma unroll
            for (int r = 0; r < RM; ++r)
#pragma unroll
                for (int c = 0; c < RN; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
        }
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int c = 0; c < RN; ++c) store(i0 + r, j0 + c, acc[r][c]);
    }
}
