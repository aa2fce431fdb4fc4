// sbr_gemm.hip -- MFMA tile kernels for the dense contractions of the
// full-to-band stage (Algorithm 4.1 with the update of Eq. (4.1)):
//   * symm_lower : W = A22 * Y, A22 symmetric with only its lower triangle
//                  stored (the X U T product of Eq. (4.1));
//   * syr2k_lower: A22 += U V^T + V U^T on lower-triangle tiles only
//                  (the rank-2b trailing update of Eq. (4.1));
//   * gemm       : C = alpha op(A) op(B) + beta C for the skinny products
//                  (U T, Q2 W1^{-1}, T^T (U^T W), 1/2 U M - W) and a split-K
//                  form for the tall reductions U^T W.
// CT = double uses v_mfma_f64_16x16x4_f64; CT = float is the precision form
// (operands rounded to FP32 in LDS, FP32 accumulation, FP64 result).
#include <type_traits>

#include "sbr_device.h"
#include "sbr_internal.h"

namespace {

template <typename CT, bool TA, bool TB, int BM, int BN, int WM, int WN, bool FAST = true>
__global__ __launch_bounds__(64 * WM * WN) void gemm_kernel(
    int64_t M, int64_t N, int64_t K, int64_t kchunk, double alpha,
    const double* __restrict__ A, int64_t lda, const double* __restrict__ B, int64_t ldb,
    double beta, const double* Cin, int64_t ldci, double* Cout, int64_t ldco, int64_t slice_stride) {
    typedef TileEngine<CT, BM, BN, WM, WN> E;
    typedef TileMap<BM, E::NT, TA> MA;      // op(A)(i,k): k contiguous iff TA
    typedef TileMap<BN, E::NT, !TB> MB;     // op(B)(k,j): k contiguous iff !TB
    __shared__ CT As[SBR_BK * E::LDA];
    __shared__ CT Bs[SBR_BK * E::LDB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t i0 = (int64_t)blockIdx.x * BM, j0 = (int64_t)blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
    E eng;
    eng.zero();
    CT ra[MA::E], rb[MB::E];
    // FAST (every offset below fits 31 bits; the launcher checks): raw buffer
    // loads, 32-bit offsets from the chunk's corner, elements past M, N or
    // kend read zero through an out-of-range offset.  Otherwise element-wise
    // loads with bounds checks.
    const uint32_t lda32 = (uint32_t)lda, ldb32 = (uint32_t)ldb;
    const int mi = (int)(M - i0 < BM ? M - i0 : BM), nj = (int)(N - j0 < BN ? N - j0 : BN);
    auto load = [&](int64_t k0) {
        if constexpr (FAST) {
            const int kv = (int)(kend - k0 < SBR_BK ? kend - k0 : SBR_BK);
            const __amdgpu_buffer_rsrc_t rsa = sbr_buffer(TA ? A + k0 + i0 * lda : A + i0 + k0 * lda, SBR_BUF_OOB - 1);
            const __amdgpu_buffer_rsrc_t rsb = sbr_buffer(TB ? B + j0 + k0 * ldb : B + k0 + j0 * ldb, SBR_BUF_OOB - 1);
#pragma unroll
            for (int e = 0; e < MA::E; ++e) {
                int i, k;
                MA::coords(t, e, i, k);
                const uint32_t off = TA ? (uint32_t)k + (uint32_t)i * lda32 : (uint32_t)i + (uint32_t)k * lda32;
                ra[e] = (CT)sbr_buffer_load(rsa, (i < mi && k < kv) ? off * 8u : SBR_BUF_OOB, 0.0);
            }
#pragma unroll
            for (int e = 0; e < MB::E; ++e) {
                int j, k;
                MB::coords(t, e, j, k);
                const uint32_t off = TB ? (uint32_t)j + (uint32_t)k * ldb32 : (uint32_t)k + (uint32_t)j * ldb32;
                rb[e] = (CT)sbr_buffer_load(rsb, (j < nj && k < kv) ? off * 8u : SBR_BUF_OOB, 0.0);
            }
            return;
        }
#pragma unroll
        for (int e = 0; e < MA::E; ++e) {
            int i, k;
            MA::coords(t, e, i, k);
            const int64_t gi = i0 + i, gk = k0 + k;
            double v = 0.0;
            if (gi < M && gk < kend) v = TA ? A[gk + gi * lda] : A[gi + gk * lda];
            ra[e] = (CT)v;
        }
#pragma unroll
        for (int e = 0; e < MB::E; ++e) {
            int j, k;
            MB::coords(t, e, j, k);
            const int64_t gj = j0 + j, gk = k0 + k;
            double v = 0.0;
            if (gj < N && gk < kend) v = TB ? B[gj + gk * ldb] : B[gk + gj * ldb];
            rb[e] = (CT)v;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < MA::E; ++e) {
            int i, k;
            MA::coords(t, e, i, k);
            As[k * E::LDA + i] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < MB::E; ++e) {
            int j, k;
            MB::coords(t, e, j, k);
            Bs[k * E::LDB + j] = rb[e];
        }
    };
    if (kbeg < kend) {
        load(kbeg);
        store();
        __syncthreads();
        for (int64_t k0 = kbeg; k0 < kend; k0 += SBR_BK) {
            const bool more = k0 + SBR_BK < kend;
            if (more) load(k0 + SBR_BK);
            eng.chunk(As, Bs, wm, wn, lane);
            __syncthreads();
            if (more) {
                store();
                __syncthreads();
            }
        }
    }
    double* Co = Cout + (int64_t)blockIdx.z * slice_stride;
#pragma unroll
    for (int tn = 0; tn < E::TN; ++tn)
#pragma unroll
        for (int tm = 0; tm < E::TM; ++tm)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + E::row_of(wm, tm, lane);
                const int64_t j = j0 + E::col_of(wn, tn, lane, r);
                if (i < M && j < N) {
                    double v = alpha * (double)eng.acc[tn][tm][r];
                    if (beta != 0.0) v += beta * Cin[i + j * ldci];
                    Co[i + j * ldco] = v;
                }
            }
}

// sum_{z < splits} p[z * stride], added in slice order (so the result does not
// depend on how the loads are grouped), the loads eight at a time: a loop that
// loads one slice and adds it before the next load makes every thread wait for
// `splits` round trips to memory one after another (up to 128 slices for the
// b x b products over the whole trailing matrix).
__device__ __forceinline__ double sum_slices(const double* __restrict__ p, int64_t stride, int splits) {
    constexpr int G = 8;
    double s = 0.0;
    int z = 0;
    for (; z + G <= splits; z += G) {
        double v[G];
#pragma unroll
        for (int u = 0; u < G; ++u) v[u] = p[(int64_t)(z + u) * stride];
#pragma unroll
        for (int u = 0; u < G; ++u) s += v[u];
    }
    for (; z < splits; ++z) s += p[(int64_t)z * stride];
    return s;
}

// out = alpha * sum_s part[s] + beta * Cin (part[s] is M x N with ld M).
__global__ void reduce_slices_kernel(int64_t M, int64_t N, int splits, const double* __restrict__ part,
                                     double alpha, double beta, const double* Cin, int64_t ldci,
                                     double* Cout, int64_t ldco) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * N) return;
    const int64_t i = idx % M, j = idx / M;
    const double s = sum_slices(part + idx, M * N, splits);
    double v = alpha * s;
    if (beta != 0.0) v += beta * Cin[i + j * ldci];
    Cout[i + j * ldco] = v;
}

// M = T^T Z with Z the sum of `splits` split-K partial slices (b x b each,
// ld b): one block per column j of M, thread k first sums row k of the
// slices (slice order, as reduce_slices), then thread i forms
// M[i][j] = sum_k T[k][i] Z[k][j], walking its own column of T.
__global__ __launch_bounds__(128) void tt_reduce_kernel(int b, int splits, const double* __restrict__ part,
                                                        const double* __restrict__ T, int64_t ldt,
                                                        double* __restrict__ M) {
    __shared__ double z[128];
    const int j = blockIdx.x, t = threadIdx.x;
    const int64_t bb = (int64_t)b * b;
    if (t < b) {
        z[t] = sum_slices(part + t + (int64_t)j * b, bb, splits);
    }
    __syncthreads();
    if (t < b) {
        const double* Tc = T + (int64_t)t * ldt;
        double acc = 0.0;
        for (int k = 0; k < b; ++k) acc += Tc[k] * z[k];
        M[t + (int64_t)j * b] = acc;
    }
}

// Blocks are dealt round-robin to the 8 XCDs (block x runs on XCD x mod 8).
// Renumber them so that each XCD works on a contiguous range of logical
// tiles: neighbouring tiles share operand rows, which then stay in that
// XCD's L2.
__device__ __forceinline__ int64_t xcd_logical_tile(int64_t x, int64_t ntiles) {
    const int64_t q = ntiles / 8, r = ntiles % 8, k = x % 8;
    return k * q + (k < r ? k : r) + x / 8;
}

// Lower tile x (of T x T tiles, lower triangle) in an L2-friendly order: bands
// of 8 tile rows, and inside a band the tiles column by column, so the 8 row
// operands of a band stay in L2 and each column operand serves 8 tiles in a
// row.  Bands before the last are full; the last may have fewer rows.
__device__ __forceinline__ void lower_tile_banded(int64_t x, int64_t T, int64_t& I, int64_t& J) {
    auto cum = [](int64_t P) -> int64_t { return 32 * P * P + 4 * P; };   // tiles in bands < P
    int64_t P = (int64_t)((sqrt(16.0 + 128.0 * (double)x) - 4.0) / 64.0);
    while (P > 0 && cum(P) > x) --P;
    while (cum(P + 1) <= x && 8 * (P + 1) < T) ++P;
    int64_t y = x - cum(P);
    const int64_t r = (T - 8 * P < 8) ? T - 8 * P : 8;
    if (y < r * 8 * P) {
        I = 8 * P + y % r;
        J = y / r;
        return;
    }
    y -= r * 8 * P;
    int64_t q = 0;
    while (y >= r - q) {
        y -= r - q;
        ++q;
    }
    J = 8 * P + q;
    I = J + y;
}

// Lower triangle of C (m x m) += U V^T + V U^T, restricted to the columns
// j < nc; one block per lower tile pair (I >= J).  The two products are one
// GEMM with K' = 2K: [U_I, V_I] * [V_J, U_J]^T.  jt = 0: all lower tiles,
// in the banded order above (nc = m); jt > 0: the first jt tile columns,
// enumerated row by row.  Double-buffered LDS, one barrier per K chunk.
// The result is added into C with atomic adds that return nothing: with
// K' = 256 a tile is only 16 chunks long, and a read-modify-write epilogue
// would hold the block for a full C read latency.
// ST: storage type of C (double, or float for the FP32-storage form); OT:
// type of U and V (double, or FP32 copies of them in the FP32 form, half the
// bytes per operand).
// DL (128 x 128 tiles on 8 waves, every tile inside the matrix, columns of U
// and V 16-byte aligned, CT = OT; the launcher checks): operands go from
// memory straight into LDS (16-byte buffer loads with an LDS destination,
// lane l's bytes at the window base + 16 l).  Wave w moves k-columns 2w and
// 2w + 1 of both operands: FP64, one load per 128-row k-column (LDS rows
// padded to 130); FP32, one load for both columns (lanes 0-31 and 32-63;
// LDS rows unpadded, 128 floats).  The loads of chunk c + 1 run behind the
// products of chunk c, and each wave waits for its own loads before the
// chunk's closing barrier.  The two buffers are separate LDS objects and the
// chunk loop runs in pairs, so a load into one buffer is seen not to alias
// the reads of the other.
template <typename CT, int BM, int WM, int WN, int PAD = 2, typename ST = double, bool FAST = true,
          typename OT = double, bool DL = false>
__global__ __launch_bounds__(64 * WM * WN) void syr2k_lower_kernel(
    int64_t m, int64_t nc, int64_t jt, int64_t K, const OT* __restrict__ U, int64_t ldu,
    const OT* __restrict__ V, int64_t ldv, ST* C, int64_t ldc, int64_t ntiles) {
    typedef TileEngine<CT, BM, BM, WM, WN, PAD, false> E;
    typedef TileMap<BM, E::NT, false> MA;   // row fastest (column-major U, V)
    typedef TileMap<BM, E::NT, false> MB;
    static_assert(!DL || (FAST && std::is_same<CT, OT>::value && BM == 128 && WM * WN == 8 && SBR_BK == 16 &&
                          (sizeof(CT) == 8 ? PAD == 2 : PAD == 0)),
                  "direct LDS loads: 128 x 128 tiles on 8 waves");
    const int64_t x = xcd_logical_tile(blockIdx.x, ntiles);
    int64_t I, J;
    if (jt == 0) {
        lower_tile_banded(x, (m + BM - 1) / BM, I, J);
    } else {
        I = x / jt;
        J = x % jt;
        if (J > I) return;   // whole block: above the diagonal
    }
    const int64_t i0 = I * BM, j0 = J * BM;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t K2 = 2 * K;
    E eng;
    eng.zero();
    constexpr int64_t SO = sizeof(OT);
    const uint32_t span = (uint32_t)((m + (int64_t)(SBR_BK - 1) * ldu) * SO);
    const int64_t nch = (K2 + SBR_BK - 1) / SBR_BK;
    if constexpr (DL) {
        __shared__ __align__(16) CT As0[SBR_BK * E::LDA], As1[SBR_BK * E::LDA];
        __shared__ __align__(16) CT Bs0[SBR_BK * E::LDB], Bs1[SBR_BK * E::LDB];
        constexpr bool F64 = sizeof(CT) == 8;
        constexpr int EPL = 16 / (int)sizeof(CT);   // elements a lane moves
        constexpr int NLD = F64 ? 2 : 1;            // loads per operand and wave
        const int li = F64 ? EPL * lane : EPL * (lane & 31);
        const int lk = F64 ? 0 : (lane >> 5);
        const uint32_t la = (uint32_t)(((i0 + li) + (int64_t)(2 * wave + lk) * ldu) * SO);
        const uint32_t lb = (uint32_t)(((j0 + li) + (int64_t)(2 * wave + lk) * ldu) * SO);
        const uint32_t ldub = (uint32_t)(ldu * SO);
        auto dload = [&](int64_t k0, CT* as, CT* bs) {
            const OT* pa = (k0 < K) ? U + k0 * ldu : V + (k0 - K) * ldu;
            const OT* pb = (k0 < K) ? V + k0 * ldu : U + (k0 - K) * ldu;
            const __amdgpu_buffer_rsrc_t rsa = sbr_buffer(pa, span);
            const __amdgpu_buffer_rsrc_t rsb = sbr_buffer(pb, span);
#pragma unroll
            for (int kk = 0; kk < NLD; ++kk) {
                const int k = 2 * wave + kk;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsa, (__attribute__((address_space(3))) void*)(as + k * E::LDA), 16, la + kk * ldub, 0, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsb, (__attribute__((address_space(3))) void*)(bs + k * E::LDB), 16, lb + kk * ldub, 0, 0, 0);
            }
        };
        // K is a multiple of the chunk depth, so K' = 2K holds an even
        // number of chunks
        dload(0, As0, Bs0);
        __syncthreads();
        for (int64_t c = 0; c < nch; c += 2) {
            dload((c + 1) * SBR_BK, As1, Bs1);   // last read before the previous barrier
            eng.chunk_fenced(As0, Bs0, wm, wn, lane);
            __syncthreads();
            if (c + 2 < nch) dload((c + 2) * SBR_BK, As0, Bs0);
            eng.chunk_fenced(As1, Bs1, wm, wn, lane);
            __syncthreads();
        }
    } else {
    __shared__ CT As[2][SBR_BK * E::LDA];
    __shared__ CT Bs[2][SBR_BK * E::LDB];
    CT ra[MA::E], rb[MB::E];
    // FAST (U and V share the leading dimension, K is a multiple of the chunk
    // depth, so a chunk lies wholly in the U or the V half of K', and
    // (m + (SBR_BK - 1) ldu) * 8 < 2^31; the launcher checks): raw buffer
    // loads with fixed per-thread byte offsets; a chunk only moves the
    // (block-uniform) buffer base, and rows past m read zero through an
    // out-of-range offset.  No branches and no 64-bit address arithmetic per
    // element.  Otherwise element-wise loads with bounds checks.
    uint32_t offa[MA::E], offb[MB::E];
    if constexpr (FAST) {
#pragma unroll
        for (int e = 0; e < MA::E; ++e) {
            int i, k;
            MA::coords(t, e, i, k);
            offa[e] = (i0 + i < m) ? (uint32_t)(((i0 + i) + (int64_t)k * ldu) * SO) : SBR_BUF_OOB;
        }
#pragma unroll
        for (int e = 0; e < MB::E; ++e) {
            int j, k;
            MB::coords(t, e, j, k);
            offb[e] = (j0 + j < m) ? (uint32_t)(((j0 + j) + (int64_t)k * ldu) * SO) : SBR_BUF_OOB;
        }
    }
    auto load = [&](int64_t k0) {
        if constexpr (FAST) {
            const OT* pa = (k0 < K) ? U + k0 * ldu : V + (k0 - K) * ldu;
            const OT* pb = (k0 < K) ? V + k0 * ldu : U + (k0 - K) * ldu;
            const __amdgpu_buffer_rsrc_t rsa = sbr_buffer(pa, span);
            const __amdgpu_buffer_rsrc_t rsb = sbr_buffer(pb, span);
#pragma unroll
            for (int e = 0; e < MA::E; ++e) ra[e] = (CT)sbr_buffer_load(rsa, offa[e], OT());
#pragma unroll
            for (int e = 0; e < MB::E; ++e) rb[e] = (CT)sbr_buffer_load(rsb, offb[e], OT());
            return;
        }
#pragma unroll
        for (int e = 0; e < MA::E; ++e) {
            int i, k;
            MA::coords(t, e, i, k);
            const int64_t gi = i0 + i, gk = k0 + k;
            OT v = 0;
            if (gi < m && gk < K2) v = (gk < K) ? U[gi + gk * ldu] : V[gi + (gk - K) * ldv];
            ra[e] = (CT)v;
        }
#pragma unroll
        for (int e = 0; e < MB::E; ++e) {
            int j, k;
            MB::coords(t, e, j, k);
            const int64_t gj = j0 + j, gk = k0 + k;
            OT v = 0;
            if (gj < m && gk < K2) v = (gk < K) ? V[gj + gk * ldv] : U[gj + (gk - K) * ldu];
            rb[e] = (CT)v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < MA::E; ++e) {
            int i, k;
            MA::coords(t, e, i, k);
            As[buf][k * E::LDA + i] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < MB::E; ++e) {
            int j, k;
            MB::coords(t, e, j, k);
            Bs[buf][k * E::LDB + j] = rb[e];
        }
    };
    load(0);
    store(0);
    __syncthreads();
    for (int64_t c = 0; c < nch; ++c) {
        const int cur = (int)(c & 1);
        const bool more = c + 1 < nch;
        if (more) load((c + 1) * SBR_BK);
        eng.chunk(As[cur], Bs[cur], wm, wn, lane);
        if (more) store(cur ^ 1);     // that buffer was last read before the previous barrier
        __syncthreads();
    }
    }
#pragma unroll
    for (int tn = 0; tn < E::TN; ++tn)
#pragma unroll
        for (int tm = 0; tm < E::TM; ++tm)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + E::row_of(wm, tm, lane);
                const int64_t j = j0 + E::col_of(wn, tn, lane, r);
                // fire-and-forget atomic add: each element gets exactly one
                // add per launch (deterministic), and the block does not wait
                // for a read of C before it retires
                if (i < m && j <= i && j < nc)
                    __hip_atomic_fetch_add(&C[i + j * ldc], (ST)eng.acc[tn][tm][r], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
}

// W (m x nb) = A Y with A symmetric, lower triangle stored.  The K range of
// a tile row splits into chunks below the diagonal block (A read directly
// from A[i0 + k0 lda], rows contiguous), the diagonal block itself
// (element-wise choice between the lower part and its mirror) and chunks
// above it (the mirror, read from A[k0 + i0 lda], k contiguous).  Each
// segment runs its own double-buffered LDS pipeline, so the per-thread
// offsets of one load form are live only during its segment.
//
// Operands come through raw buffer loads: 32-bit byte offsets from a
// block-uniform base that a chunk moves, rows past m, columns past nb and k
// past kend read zero through an out-of-range offset.  Every offset is below
// 2^31 (the launcher checks (m + BM lda) sizeof(ST) and BN ldy 8 against it).
// YT: type of Y (double, or an FP32 copy of it in the FP32 form).
template <typename CT, int BM, int BN, int WM, int WN, int PAD = 2, typename ST = double, typename YT = double>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(BM == 128 ? 4 : 1))) void symm_lower_kernel(
    int64_t m, int64_t nb, int64_t kchunk, const ST* __restrict__ A, int64_t lda,
    const YT* __restrict__ Y, int64_t ldy, double* W, int64_t ldw, int64_t slice_stride) {
    typedef TileEngine<CT, BM, BN, WM, WN, PAD, false> E;   // long K: no operand prefetch (registers)
    typedef TileMap<BM, E::NT, false> MAi;   // row fastest
    typedef TileMap<BM, E::NT, true> MAk;    // k fastest
    typedef TileMap<BN, E::NT, true> MB;     // Y[k + j ldy]: k contiguous
    static_assert(MAi::E == MAk::E, "maps");
    __shared__ CT As[2][SBR_BK * E::LDA];
    __shared__ CT Bs[2][SBR_BK * E::LDB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t i0 = (int64_t)blockIdx.x * BM, j0 = (int64_t)blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;   // kchunk is a multiple of SBR_BK
    const int64_t kend = (kbeg + kchunk < m) ? kbeg + kchunk : m;
    E eng;
    eng.zero();
    CT ra[MAi::E], rb[MB::E];
    constexpr uint32_t SA = sizeof(ST);
    const uint32_t lda32 = (uint32_t)lda, ldy32 = (uint32_t)ldy;
    const uint32_t spanD = (uint32_t)((BM + (int64_t)(SBR_BK - 1) * lda) * SA);
    const uint32_t spanM = (uint32_t)((SBR_BK + (int64_t)(BM - 1) * lda) * SA);
    const uint32_t spanS = (uint32_t)((m + (int64_t)BM * lda) * SA);
    constexpr uint32_t SY = sizeof(YT);
    const uint32_t spanY = (uint32_t)((SBR_BK + (int64_t)(BN - 1) * ldy) * SY);
    const uint32_t mrows = (uint32_t)(m - i0 < BM ? m - i0 : BM);      // valid rows of the tile
    const uint32_t ncols = (uint32_t)(nb - j0 < BN ? nb - j0 : BN);    // valid columns of Y

    auto load_y = [&](int64_t k0) {
        const __amdgpu_buffer_rsrc_t ry = sbr_buffer(Y + k0 + j0 * ldy, spanY);
        const int64_t kv = kend - k0;     // valid k of the chunk
#pragma unroll
        for (int e = 0; e < MB::E; ++e) {
            int j, k;
            MB::coords(t, e, j, k);
            const bool ok = (uint32_t)j < ncols && k < kv;
            rb[e] = (CT)sbr_buffer_load(ry, ok ? ((uint32_t)k + (uint32_t)j * ldy32) * SY : SBR_BUF_OOB, YT());
        }
    };
    // below the diagonal block: A[i0 + i + (k0 + k) lda]
    auto load_below = [&](int64_t k0) {
        const __amdgpu_buffer_rsrc_t rs = sbr_buffer(A + i0 + k0 * lda, spanD);
#pragma unroll
        for (int e = 0; e < MAi::E; ++e) {
            int i, k;
            MAi::coords(t, e, i, k);
            ra[e] = (CT)sbr_buffer_load(rs, (uint32_t)i < mrows ? ((uint32_t)i + (uint32_t)k * lda32) * SA : SBR_BUF_OOB,
                                        ST());
        }
        load_y(k0);
    };
    // above it: the mirror A[k0 + k + (i0 + i) lda]
    auto load_above = [&](int64_t k0) {
        const __amdgpu_buffer_rsrc_t rs = sbr_buffer(A + k0 + i0 * lda, spanM);
#pragma unroll
        for (int e = 0; e < MAk::E; ++e) {
            int i, k;
            MAk::coords(t, e, i, k);
            ra[e] = (CT)sbr_buffer_load(rs, (uint32_t)i < mrows ? ((uint32_t)k + (uint32_t)i * lda32) * SA : SBR_BUF_OOB,
                                        ST());
        }
        load_y(k0);
    };
    // the diagonal block, or a chunk ending past kend: element-wise choice
    // between the lower part and its mirror, offsets from the corner (d0, d0),
    // d0 = min(i0, k0), where both choices are non-negative and the smaller
    // index is below BM
    auto load_mixed = [&](int64_t k0) {
        const int64_t d0 = i0 < k0 ? i0 : k0;
        const __amdgpu_buffer_rsrc_t rs = sbr_buffer(A + d0 + d0 * lda, spanS);
        const int64_t kv = kend - k0;
#pragma unroll
        for (int e = 0; e < MAi::E; ++e) {
            int i, k;
            MAi::coords(t, e, i, k);
            const uint32_t r = (uint32_t)(i0 + i - d0), c = (uint32_t)(k0 + k - d0);
            const uint32_t off = (r >= c) ? r + c * lda32 : c + r * lda32;
            ra[e] = (CT)sbr_buffer_load(rs, ((uint32_t)i < mrows && k < kv) ? off * SA : SBR_BUF_OOB, ST());
        }
        load_y(k0);
    };
    auto store = [&](int buf, bool kfast) {
#pragma unroll
        for (int e = 0; e < MAi::E; ++e) {
            int i, k;
            if (kfast) MAk::coords(t, e, i, k); else MAi::coords(t, e, i, k);
            As[buf][k * E::LDA + i] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < MB::E; ++e) {
            int j, k;
            MB::coords(t, e, j, k);
            Bs[buf][k * E::LDB + j] = rb[e];
        }
    };
    // chunks [ka, kb) with one load form (kfast: the k-fastest map)
    auto segment = [&](int64_t ka, int64_t kb, bool kfast, auto&& load) {
        if (ka >= kb) return;
        const int64_t nch = (kb - ka + SBR_BK - 1) / SBR_BK;
        load(ka);
        store(0, kfast);
        __syncthreads();
        for (int64_t c = 0; c < nch; ++c) {
            const int cur = (int)(c & 1);
            const bool more = c + 1 < nch;
            if (more) load(ka + (c + 1) * SBR_BK);
            eng.chunk(As[cur], Bs[cur], wm, wn, lane);
            if (more) store(cur ^ 1, kfast);     // that buffer was last read before the previous barrier
            __syncthreads();
        }
    };
    if (kbeg < kend) {
        // whole chunks end at kfull; a last partial chunk takes the mixed form
        const int64_t kfull = kbeg + (kend - kbeg) / SBR_BK * SBR_BK;
        const int64_t dlo = i0, dhi = i0 + BM;             // the diagonal block's columns
        segment(kbeg, kfull < dlo ? kfull : dlo, false, load_below);
        segment(kbeg > dlo ? kbeg : dlo, kend < dhi ? kend : dhi, false, load_mixed);
        segment(kbeg > dhi ? kbeg : dhi, kfull, true, load_above);
        // the partial chunk, unless it lies in the diagonal block's segment
        if (kfull < kend && (kfull < dlo || kfull >= dhi)) segment(kfull, kend, false, load_mixed);
    }
    double* Wo = W + (int64_t)blockIdx.z * slice_stride;
#pragma unroll
    for (int tn = 0; tn < E::TN; ++tn)
#pragma unroll
        for (int tm = 0; tm < E::TM; ++tm)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + E::row_of(wm, tm, lane);
                const int64_t j = j0 + E::col_of(wn, tn, lane, r);
                if (i < m && j < nb) Wo[i + j * ldw] = (double)eng.acc[tn][tm][r];
            }
}

// The same product for full tiles (m a multiple of 128, nb = 128), reading Y
// transposed: Yt = Y^T (nb x m, ld ldyt = 128), so that a k-row of the Y tile
// is 128 contiguous elements.  Operands that are contiguous along the tile's
// fast index go from memory straight into LDS (16-byte buffer loads with an
// LDS destination, lane l's bytes at the window base + 16 l): Yt in every
// chunk and the A tile in the chunks below the diagonal block.  FP64 (CT = ST
// = double): one load moves one 128-element k-row, wave w moves rows 2w and
// 2w + 1 of each operand; the LDS rows keep their padding (130 doubles).
// FP32 (the FP32-MFMA form, CT = ST = float, A the FP32 copy of the trailing
// matrix): one load moves rows 2w (lanes 0-31) and 2w + 1 (lanes 32-63), so
// the LDS rows are unpadded (128 floats).  The diagonal block (element-wise
// choice of the entry or its mirror) and the chunks above it (the mirror, k
// contiguous) still pass A through registers.  The two LDS buffers are
// separate objects and each segment runs its chunks in pairs, so a load into
// one buffer is seen not to alias the other buffer's reads; the products and
// their order are those of symm_lower_kernel.
constexpr int SYMM_DL_NT = 512;

template <typename CT>
__global__ __launch_bounds__(SYMM_DL_NT) __attribute__((amdgpu_waves_per_eu(4))) void symm_lower_dl_kernel(
    int64_t m, int64_t kchunk, const CT* __restrict__ A, int64_t lda, const CT* __restrict__ Yt, int64_t ldyt,
    double* W, int64_t ldw, int64_t slice_stride) {
    constexpr int BM = 128, BN = 128;
    constexpr bool F64 = sizeof(CT) == 8;
    constexpr int PADL = F64 ? 2 : 0;
    typedef TileEngine<CT, BM, BN, 2, 4, PADL, false> E;
    typedef TileMap<BM, E::NT, false> MAi;   // row fastest
    typedef TileMap<BM, E::NT, true> MAk;    // k fastest
    static_assert(MAi::E == MAk::E && E::NT == SYMM_DL_NT && SBR_BK == 16, "tile shape");
    static_assert(F64 || E::LDA * sizeof(CT) == 512, "FP32 rows of 512 bytes, two per load");
    __shared__ __align__(16) CT As0[SBR_BK * E::LDA], As1[SBR_BK * E::LDA];
    __shared__ __align__(16) CT Bs0[SBR_BK * E::LDB], Bs1[SBR_BK * E::LDB];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave % 2, wn = wave / 2;
    const int64_t i0 = (int64_t)blockIdx.x * BM;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;   // kchunk and m are multiples of SBR_BK
    const int64_t kend = (kbeg + kchunk < m) ? kbeg + kchunk : m;
    E eng;
    eng.zero();
    constexpr uint32_t SA = sizeof(CT);
    const uint32_t lda32 = (uint32_t)lda;
    const uint32_t spanD = (uint32_t)((BM + (int64_t)(SBR_BK - 1) * lda) * SA);
    const uint32_t spanM = (uint32_t)((SBR_BK + (int64_t)(BM - 1) * lda) * SA);
    const uint32_t spanS = (uint32_t)((m + (int64_t)BM * lda) * SA);
    const uint32_t spanY = (uint32_t)((BN + (int64_t)(SBR_BK - 1) * ldyt) * SA);
    // per-lane byte offsets of the straight-to-LDS loads (k-row 2 wave first)
    constexpr int EPL = 16 / sizeof(CT);   // elements a lane moves
    const int li = F64 ? EPL * lane : EPL * (lane & 31);
    const int lk = F64 ? 0 : (lane >> 5);
    const uint32_t ly = (uint32_t)((li + (int64_t)(2 * wave + lk) * ldyt) * SA);
    const uint32_t la = (uint32_t)((li + (int64_t)(2 * wave + lk) * lda) * SA);
    const uint32_t ldyb = (uint32_t)(ldyt * SA), ldab = (uint32_t)(lda * SA);
    constexpr int NLD = F64 ? 2 : 1;   // loads per operand and wave
    typedef __attribute__((address_space(3))) void* lds_ptr;
    CT ra[MAi::E];
    // MODE 0: below the diagonal block (A straight to LDS); 1: the diagonal
    // block (element-wise, registers); 2: above it (the mirror, registers)
    auto issue = [&](auto mode, int64_t k0, CT* as, CT* bs) {
        constexpr int MODE = decltype(mode)::value;
        const __amdgpu_buffer_rsrc_t ry = sbr_buffer(Yt + k0 * ldyt, spanY);
#pragma unroll
        for (int kk = 0; kk < NLD; ++kk)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ry, (lds_ptr)(bs + (2 * wave + kk) * E::LDB), 16,
                                                     ly + kk * ldyb, 0, 0, 0);
        if constexpr (MODE == 0) {
            const __amdgpu_buffer_rsrc_t rs = sbr_buffer(A + i0 + k0 * lda, spanD);
#pragma unroll
            for (int kk = 0; kk < NLD; ++kk)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr)(as + (2 * wave + kk) * E::LDA), 16,
                                                         la + kk * ldab, 0, 0, 0);
        } else if constexpr (MODE == 1) {
            const int64_t d0 = i0 < k0 ? i0 : k0;
            const __amdgpu_buffer_rsrc_t rs = sbr_buffer(A + d0 + d0 * lda, spanS);
#pragma unroll
            for (int e = 0; e < MAi::E; ++e) {
                int i, k;
                MAi::coords(t, e, i, k);
                const uint32_t r = (uint32_t)(i0 + i - d0), c = (uint32_t)(k0 + k - d0);
                const uint32_t off = (r >= c) ? r + c * lda32 : c + r * lda32;
                ra[e] = sbr_buffer_load(rs, off * SA, CT());
            }
        } else {
            const __amdgpu_buffer_rsrc_t rs = sbr_buffer(A + k0 + i0 * lda, spanM);
#pragma unroll
            for (int e = 0; e < MAk::E; ++e) {
                int i, k;
                MAk::coords(t, e, i, k);
                ra[e] = sbr_buffer_load(rs, ((uint32_t)k + (uint32_t)i * lda32) * SA, CT());
            }
        }
    };
    auto store = [&](auto mode, CT* as) {
        constexpr int MODE = decltype(mode)::value;
        if constexpr (MODE != 0) {
#pragma unroll
            for (int e = 0; e < MAi::E; ++e) {
                int i, k;
                if constexpr (MODE == 2) MAk::coords(t, e, i, k);
                else MAi::coords(t, e, i, k);
                as[k * E::LDA + i] = ra[e];
            }
        }
    };
    auto segment = [&](auto mode, int64_t ka, int64_t kb) {
        if (ka >= kb) return;
        const int64_t nch = (kb - ka) / SBR_BK;
        issue(mode, ka, As0, Bs0);
        store(mode, As0);
        __syncthreads();
        for (int64_t c = 0; c + 1 < nch; c += 2) {
            issue(mode, ka + (c + 1) * SBR_BK, As1, Bs1);   // last read before the previous barrier
            eng.chunk_fenced(As0, Bs0, wm, wn, lane);
            store(mode, As1);
            __syncthreads();
            const bool more = c + 2 < nch;
            if (more) issue(mode, ka + (c + 2) * SBR_BK, As0, Bs0);
            eng.chunk_fenced(As1, Bs1, wm, wn, lane);
            if (more) store(mode, As0);
            __syncthreads();
        }
        if (nch & 1) {   // the last chunk is in the first buffer
            eng.chunk_fenced(As0, Bs0, wm, wn, lane);
            __syncthreads();
        }
    };
    const int64_t dlo = i0, dhi = i0 + BM;   // the diagonal block's columns
    segment(std::integral_constant<int, 0>(), kbeg, kend < dlo ? kend : dlo);
    segment(std::integral_constant<int, 1>(), kbeg > dlo ? kbeg : dlo, kend < dhi ? kend : dhi);
    segment(std::integral_constant<int, 2>(), kbeg > dhi ? kbeg : dhi, kend);
    double* Wo = W + (int64_t)blockIdx.z * slice_stride;
#pragma unroll
    for (int tn = 0; tn < E::TN; ++tn)
#pragma unroll
        for (int tm = 0; tm < E::TM; ++tm)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + E::row_of(wm, tm, lane);
                const int64_t j = E::col_of(wn, tn, lane, r);
                Wo[i + j * ldw] = (double)eng.acc[tn][tm][r];
            }
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <typename CT, bool TA, bool TB, bool FAST>
void gemm_dispatch_f(int64_t M, int64_t N, int64_t K, int64_t kchunk, int splits, double alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                     const double* Cin, int64_t ldci, double* Cout, int64_t ldco, int64_t slice_stride,
                     hipStream_t s) {
    if (N > 32) {
        dim3 g(cdiv(M, 64), cdiv(N, 64), splits);
        gemm_kernel<CT, TA, TB, 64, 64, 2, 2, FAST><<<g, 256, 0, s>>>(M, N, K, kchunk, alpha, A, lda, B, ldb, beta,
                                                                       Cin, ldci, Cout, ldco, slice_stride);
    } else if (N > 16) {
        dim3 g(cdiv(M, 64), cdiv(N, 32), splits);
        gemm_kernel<CT, TA, TB, 64, 32, 4, 1, FAST><<<g, 256, 0, s>>>(M, N, K, kchunk, alpha, A, lda, B, ldb, beta,
                                                                       Cin, ldci, Cout, ldco, slice_stride);
    } else {
        dim3 g(cdiv(M, 64), cdiv(N, 16), splits);
        gemm_kernel<CT, TA, TB, 64, 16, 4, 1, FAST><<<g, 256, 0, s>>>(M, N, K, kchunk, alpha, A, lda, B, ldb, beta,
                                                                       Cin, ldci, Cout, ldco, slice_stride);
    }
}

template <typename CT, bool TA, bool TB>
void gemm_dispatch(int64_t M, int64_t N, int64_t K, int64_t kchunk, int splits, double alpha,
                   const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                   const double* Cin, int64_t ldci, double* Cout, int64_t ldco, int64_t slice_stride,
                   hipStream_t s) {
    // the largest offset of a 64-row tile chunk: (64 + 16) (ld + 1) elements
    const int64_t ld = lda > ldb ? lda : ldb;
    if ((int64_t)(64 + SBR_BK) * (ld + 1) * 8 < (int64_t)SBR_BUF_OOB - 8)
        gemm_dispatch_f<CT, TA, TB, true>(M, N, K, kchunk, splits, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout,
                                          ldco, slice_stride, s);
    else
        gemm_dispatch_f<CT, TA, TB, false>(M, N, K, kchunk, splits, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout,
                                           ldco, slice_stride, s);
}

template <typename CT>
void gemm_dispatch_t(bool ta, bool tb, int64_t M, int64_t N, int64_t K, int64_t kchunk, int splits,
                     double alpha, const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                     const double* Cin, int64_t ldci, double* Cout, int64_t ldco, int64_t slice_stride,
                     hipStream_t s) {
    if (!ta && !tb) gemm_dispatch<CT, false, false>(M, N, K, kchunk, splits, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout, ldco, slice_stride, s);
    else if (ta && !tb) gemm_dispatch<CT, true, false>(M, N, K, kchunk, splits, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout, ldco, slice_stride, s);
    else if (!ta && tb) gemm_dispatch<CT, false, true>(M, N, K, kchunk, splits, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout, ldco, slice_stride, s);
    else gemm_dispatch<CT, true, true>(M, N, K, kchunk, splits, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout, ldco, slice_stride, s);
}

template <typename CT, typename ST, typename YT = double>
void symm_dispatch(int64_t m, int64_t nb, int64_t kchunk, int splits, const ST* A, int64_t lda,
                   const YT* Y, int64_t ldy, double* W, int64_t ldw, int64_t slice_stride, hipStream_t s) {
    if (nb > 64) {
        if (m >= 2048) {
            dim3 g(cdiv(m, 128), cdiv(nb, 128), splits);
            symm_lower_kernel<CT, 128, 128, 2, 4, 2, ST, YT><<<g, 512, 0, s>>>(m, nb, kchunk, A, lda, Y, ldy, W, ldw, slice_stride);
        } else {
            dim3 g(cdiv(m, 64), cdiv(nb, 128), splits);
            symm_lower_kernel<CT, 64, 128, 2, 2, 2, ST, YT><<<g, 256, 0, s>>>(m, nb, kchunk, A, lda, Y, ldy, W, ldw, slice_stride);
        }
    } else if (nb > 32) {
        dim3 g(cdiv(m, 64), cdiv(nb, 64), splits);
        symm_lower_kernel<CT, 64, 64, 2, 2, 2, ST, YT><<<g, 256, 0, s>>>(m, nb, kchunk, A, lda, Y, ldy, W, ldw, slice_stride);
    } else if (nb > 16) {
        dim3 g(cdiv(m, 64), cdiv(nb, 32), splits);
        symm_lower_kernel<CT, 64, 32, 4, 1, 2, ST, YT><<<g, 256, 0, s>>>(m, nb, kchunk, A, lda, Y, ldy, W, ldw, slice_stride);
    } else {
        dim3 g(cdiv(m, 64), cdiv(nb, 16), splits);
        symm_lower_kernel<CT, 64, 16, 4, 1, 2, ST, YT><<<g, 256, 0, s>>>(m, nb, kchunk, A, lda, Y, ldy, W, ldw, slice_stride);
    }
}

// Lower triangle of the m x m block of A (ld lda) into the FP32 copy As
// (ld lds), and a column block of As (rows [0, m), the first nc columns, lower
// part) back into A.
__global__ void lower_to_f32_kernel(int64_t m, const double* __restrict__ A, int64_t lda, float* As, int64_t lds) {
    const int64_t j = blockIdx.y;
    for (int64_t i = j + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        As[i + j * lds] = (float)A[i + j * lda];
}
// The m x nc block of X (ld ldx) rounded to FP32 into Xs (ld lds).
__global__ void block_to_f32_kernel(int64_t m, const double* __restrict__ X, int64_t ldx, float* Xs, int64_t lds) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        Xs[i + j * lds] = (float)X[i + j * ldx];
}
__global__ void cols_to_f64_kernel(int64_t m, const float* __restrict__ As, int64_t lds, double* A, int64_t lda) {
    const int64_t j = blockIdx.y;
    for (int64_t i = j + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        A[i + j * lda] = (double)As[i + j * lds];
}

void reduce_slices(int64_t M, int64_t N, int splits, const double* part, double alpha, double beta,
                   const double* Cin, int64_t ldci, double* Cout, int64_t ldco, hipStream_t s) {
    const int64_t tot = M * N;
    reduce_slices_kernel<<<cdiv(tot, 256), 256, 0, s>>>(M, N, splits, part, alpha, beta, Cin, ldci, Cout, ldco);
}

}  // namespace

namespace sbr {

void launch_gemm(bool f32, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 const double* Cin, int64_t ldci, double* Cout, int64_t ldco, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    const int64_t kc = K > 0 ? K : 1;
    if (f32) gemm_dispatch_t<float>(ta, tb, M, N, K, kc, 1, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout, ldco, 0, s);
    else gemm_dispatch_t<double>(ta, tb, M, N, K, kc, 1, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout, ldco, 0, s);
}

int gemm_splits(int64_t M, int64_t N, int64_t K) {
    const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int64_t splits = 1;
    while (tiles * splits < 512 && K / (splits * 2) >= 128) splits *= 2;
    return (int)splits;
}

void launch_gemm_splitk(bool f32, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                        const double* Cin, int64_t ldci, double* Cout, int64_t ldco, double* part,
                        int splits, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    if (splits <= 1) {
        launch_gemm(f32, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, Cin, ldci, Cout, ldco, s);
        return;
    }
    int64_t kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + SBR_BK - 1) / SBR_BK * SBR_BK;
    if (f32) gemm_dispatch_t<float>(ta, tb, M, N, K, kchunk, splits, 1.0, A, lda, B, ldb, 0.0, nullptr, 0, part, M, M * N, s);
    else gemm_dispatch_t<double>(ta, tb, M, N, K, kchunk, splits, 1.0, A, lda, B, ldb, 0.0, nullptr, 0, part, M, M * N, s);
    reduce_slices(M, N, splits, part, alpha, beta, Cin, ldci, Cout, ldco, s);
}

void launch_ttuw(int b, int64_t m, const double* U, int64_t ldu, const double* W, int64_t ldw, const double* T,
                 int64_t ldt, double* M, double* part, int splits, hipStream_t s) {
    if (b <= 0 || b > 128) return;
    if (splits < 1) splits = 1;
    // partials of Z = U^T W (b x b slices in part), then M = T^T Z
    int64_t kchunk = (m + splits - 1) / splits;
    kchunk = (kchunk + SBR_BK - 1) / SBR_BK * SBR_BK;
    if (kchunk < 1) kchunk = SBR_BK;
    gemm_dispatch_t<double>(true, false, b, b, m, kchunk, splits, 1.0, U, ldu, W, ldw, 0.0, nullptr, 0, part, b,
                            (int64_t)b * b, s);
    tt_reduce_kernel<<<(unsigned)b, 128, 0, s>>>(b, splits, part, T, ldt, M);
}

bool syr2k_big_tiles(int64_t m) {
    // 128 x 128 tiles on 8 waves (each wave 64 x 32) once there are enough
    // of them to fill the chip; 64 x 64 tiles on 4 waves below that
    const int64_t T128 = (m + 127) / 128;
    return T128 * (T128 + 1) / 2 >= 512;
}

// One launch of syr2k_lower_kernel over nt tiles: the buffer-load form when
// its conditions hold, the element-wise form otherwise.
template <typename CT, int BM, int WM, int WN, typename ST, typename OT = double>
void syr2k_go(int64_t nt, int64_t m, int64_t nc, int64_t jt, int64_t K, const OT* U, int64_t ldu,
              const OT* V, int64_t ldv, ST* C, int64_t ldc, hipStream_t s) {
    const bool fast = (ldu == ldv) && (K % SBR_BK == 0) &&
                      (m + (int64_t)(SBR_BK - 1) * ldu) * (int64_t)sizeof(OT) < (int64_t)SBR_BUF_OOB;
    if constexpr (std::is_same<CT, OT>::value && BM == 128 && WM * WN == 8) {
        // every tile inside the matrix (full lower tiles only) and 16-byte
        // aligned columns: operands straight into LDS
        if (fast && jt == 0 && m % BM == 0 && (ldu * (int64_t)sizeof(OT)) % 16 == 0) {
            constexpr int PADL = sizeof(CT) == 8 ? 2 : 0;
            syr2k_lower_kernel<CT, BM, WM, WN, PADL, ST, true, OT, true><<<(unsigned)nt, 64 * WM * WN, 0, s>>>(
                m, nc, jt, K, U, ldu, V, ldv, C, ldc, nt);
            return;
        }
    }
    if (fast)
        syr2k_lower_kernel<CT, BM, WM, WN, 2, ST, true, OT><<<(unsigned)nt, 64 * WM * WN, 0, s>>>(m, nc, jt, K, U, ldu,
                                                                                              V, ldv, C, ldc, nt);
    else
        syr2k_lower_kernel<CT, BM, WM, WN, 2, ST, false, OT><<<(unsigned)nt, 64 * WM * WN, 0, s>>>(m, nc, jt, K, U, ldu,
                                                                                               V, ldv, C, ldc, nt);
}

void launch_syr2k_lower(bool f32, int64_t m, int64_t K, const double* U, int64_t ldu, const double* V,
                        int64_t ldv, double* C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || K <= 0) return;
    const int64_t T128 = (m + 127) / 128;
    if (syr2k_big_tiles(m)) {
        const int64_t nt = T128 * (T128 + 1) / 2;
        if (f32) syr2k_go<float, 128, 2, 4, double>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
        else syr2k_go<double, 128, 2, 4, double>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
        return;
    }
    const int64_t T = (m + 63) / 64;
    const int64_t nt = T * (T + 1) / 2;
    if (f32) syr2k_go<float, 64, 2, 2, double>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
    else syr2k_go<double, 64, 2, 2, double>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
}

void launch_syr2k_lower_cols(bool f32, int64_t m, int64_t nc, int64_t K, const double* U, int64_t ldu,
                             const double* V, int64_t ldv, double* C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || K <= 0 || nc <= 0) return;
    if (nc > m) nc = m;
    // a tall column block: 64 x 64 tiles for more blocks in flight
    const int64_t T = (m + 63) / 64, jt = (nc + 63) / 64;
    const int64_t nt = T * jt;
    if (f32) syr2k_go<float, 64, 2, 2, double>(nt, m, nc, jt, K, U, ldu, V, ldv, C, ldc, s);
    else syr2k_go<double, 64, 2, 2, double>(nt, m, nc, jt, K, U, ldu, V, ldv, C, ldc, s);
}

bool symm_offsets_fit(int64_t m, int64_t lda, int64_t ldy, int64_t elem) {
    // the largest tile (BM = BN = 128) bounds every buffer offset of the kernel
    return (m + 128 * lda) * elem < (int64_t)SBR_BUF_OOB && (SBR_BK + 127 * ldy) * 8 < (int64_t)SBR_BUF_OOB;
}

int symm_splits(int64_t m, int64_t nb) {
    // split the reduction over A22's columns until about 1024 blocks are in
    // flight, keeping at least 256 columns per slice (a small trailing
    // matrix has few row tiles: without splits most CUs would idle)
    const int64_t bm = (nb > 64 && m >= 2048) ? 128 : 64;
    const int64_t tiles = ((m + bm - 1) / bm) * ((nb + 127) / 128);
    int64_t splits = 1;
    while (tiles * splits < 1024 && m / (splits * 2) >= 256 && splits < 16) splits *= 2;
    return (int)splits;
}

void launch_symm_lower(bool f32, int64_t m, int64_t nb, const double* A, int64_t lda, const double* Y,
                       int64_t ldy, double* W, int64_t ldw, double* part, int splits, hipStream_t s) {
    if (m <= 0 || nb <= 0) return;
    if (splits <= 1 || part == nullptr) {
        if (f32) symm_dispatch<float, double>(m, nb, m, 1, A, lda, Y, ldy, W, ldw, 0, s);
        else symm_dispatch<double, double>(m, nb, m, 1, A, lda, Y, ldy, W, ldw, 0, s);
        return;
    }
    int64_t kchunk = (m + splits - 1) / splits;
    kchunk = (kchunk + SBR_BK - 1) / SBR_BK * SBR_BK;
    if (f32) symm_dispatch<float, double>(m, nb, kchunk, splits, A, lda, Y, ldy, part, m, m * nb, s);
    else symm_dispatch<double, double>(m, nb, kchunk, splits, A, lda, Y, ldy, part, m, m * nb, s);
    reduce_slices(m, nb, splits, part, 1.0, 0.0, nullptr, 0, W, ldw, s);
}

bool symm_yt_ok(int64_t m, int64_t nb, int64_t lda, int64_t elem) {
    // 16-byte aligned columns of A (lda a multiple of 16 / elem), 32-bit offsets
    return m >= 2048 && m % 128 == 0 && nb == 128 && (lda * elem) % 16 == 0 &&
           (m + 128 * lda) * elem < (int64_t)SBR_BUF_OOB;
}

template <typename CT>
void symm_yt_go(int64_t m, int64_t nb, const CT* A, int64_t lda, const CT* Yt, int64_t ldyt, double* W,
                int64_t ldw, double* part, int splits, hipStream_t s) {
    if (m <= 0 || nb <= 0) return;
    const bool split = splits > 1 && part != nullptr;
    int64_t kchunk = m;
    if (split) {
        kchunk = (m + splits - 1) / splits;
        kchunk = (kchunk + SBR_BK - 1) / SBR_BK * SBR_BK;
    }
    dim3 g(cdiv(m, 128), 1, split ? splits : 1);
    if (split) {
        symm_lower_dl_kernel<CT><<<g, SYMM_DL_NT, 0, s>>>(m, kchunk, A, lda, Yt, ldyt, part, m, m * nb);
        reduce_slices(m, nb, splits, part, 1.0, 0.0, nullptr, 0, W, ldw, s);
    } else {
        symm_lower_dl_kernel<CT><<<g, SYMM_DL_NT, 0, s>>>(m, kchunk, A, lda, Yt, ldyt, W, ldw, 0);
    }
}

void launch_symm_lower_yt(int64_t m, int64_t nb, const double* A, int64_t lda, const double* Yt, int64_t ldyt,
                          double* W, int64_t ldw, double* part, int splits, hipStream_t s) {
    symm_yt_go<double>(m, nb, A, lda, Yt, ldyt, W, ldw, part, splits, s);
}

void launch_symm_lower_yt_f32s(int64_t m, int64_t nb, const float* A, int64_t lda, const float* Yt, int64_t ldyt,
                               double* W, int64_t ldw, double* part, int splits, hipStream_t s) {
    symm_yt_go<float>(m, nb, A, lda, Yt, ldyt, W, ldw, part, splits, s);
}

// ---- FP32-storage form: the trailing matrix lives in an FP32 copy
void launch_syr2k_lower_f32s(int64_t m, int64_t K, const double* U, int64_t ldu, const double* V, int64_t ldv,
                             float* C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || K <= 0) return;
    const int64_t T128 = (m + 127) / 128;
    if (syr2k_big_tiles(m)) {
        const int64_t nt = T128 * (T128 + 1) / 2;
        syr2k_go<float, 128, 2, 4, float>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
        return;
    }
    const int64_t T = (m + 63) / 64;
    const int64_t nt = T * (T + 1) / 2;
    syr2k_go<float, 64, 2, 2, float>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
}

void launch_syr2k_lower_cols_f32s(int64_t m, int64_t nc, int64_t K, const double* U, int64_t ldu, const double* V,
                                  int64_t ldv, float* C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || K <= 0 || nc <= 0) return;
    if (nc > m) nc = m;
    const int64_t T = (m + 63) / 64, jt = (nc + 63) / 64;
    const int64_t nt = T * jt;
    syr2k_go<float, 64, 2, 2, float>(nt, m, nc, jt, K, U, ldu, V, ldv, C, ldc, s);
}

void launch_symm_lower_f32s(int64_t m, int64_t nb, const float* A, int64_t lda, const double* Y, int64_t ldy,
                            double* W, int64_t ldw, double* part, int splits, hipStream_t s) {
    if (m <= 0 || nb <= 0) return;
    if (splits <= 1 || part == nullptr) {
        symm_dispatch<float, float>(m, nb, m, 1, A, lda, Y, ldy, W, ldw, 0, s);
        return;
    }
    int64_t kchunk = (m + splits - 1) / splits;
    kchunk = (kchunk + SBR_BK - 1) / SBR_BK * SBR_BK;
    symm_dispatch<float, float>(m, nb, kchunk, splits, A, lda, Y, ldy, part, m, m * nb, s);
    reduce_slices(m, nb, splits, part, 1.0, 0.0, nullptr, 0, W, ldw, s);
}

void launch_lower_to_f32(int64_t m, const double* A, int64_t lda, float* As, int64_t lds, hipStream_t s) {
    if (m <= 0) return;
    dim3 g((unsigned)cdiv(m, 1024) < 64 ? (unsigned)cdiv(m, 1024) : 64, (unsigned)m);
    lower_to_f32_kernel<<<g, 256, 0, s>>>(m, A, lda, As, lds);
}

void launch_block_to_f32(int64_t m, int64_t nc, const double* X, int64_t ldx, float* Xs, int64_t lds, hipStream_t s) {
    if (m <= 0 || nc <= 0) return;
    dim3 g((unsigned)cdiv(m, 1024) < 64 ? (unsigned)cdiv(m, 1024) : 64, (unsigned)nc);
    block_to_f32_kernel<<<g, 256, 0, s>>>(m, X, ldx, Xs, lds);
}

// FP32-storage form with FP32 copies of the operands (U, V; Y)
void launch_syr2k_lower_f32s(int64_t m, int64_t K, const float* U, int64_t ldu, const float* V, int64_t ldv,
                             float* C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || K <= 0) return;
    const int64_t T128 = (m + 127) / 128;
    if (syr2k_big_tiles(m)) {
        const int64_t nt = T128 * (T128 + 1) / 2;
        syr2k_go<float, 128, 2, 4, float, float>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
        return;
    }
    const int64_t T = (m + 63) / 64;
    const int64_t nt = T * (T + 1) / 2;
    syr2k_go<float, 64, 2, 2, float, float>(nt, m, m, 0, K, U, ldu, V, ldv, C, ldc, s);
}

void launch_syr2k_lower_cols_f32s(int64_t m, int64_t nc, int64_t K, const float* U, int64_t ldu, const float* V,
                                  int64_t ldv, float* C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || K <= 0 || nc <= 0) return;
    if (nc > m) nc = m;
    const int64_t T = (m + 63) / 64, jt = (nc + 63) / 64;
    const int64_t nt = T * jt;
    syr2k_go<float, 64, 2, 2, float, float>(nt, m, nc, jt, K, U, ldu, V, ldv, C, ldc, s);
}

void launch_symm_lower_f32s(int64_t m, int64_t nb, const float* A, int64_t lda, const float* Y, int64_t ldy,
                            double* W, int64_t ldw, double* part, int splits, hipStream_t s) {
    if (m <= 0 || nb <= 0) return;
    if (splits <= 1 || part == nullptr) {
        symm_dispatch<float, float, float>(m, nb, m, 1, A, lda, Y, ldy, W, ldw, 0, s);
        return;
    }
    int64_t kchunk = (m + splits - 1) / splits;
    kchunk = (kchunk + SBR_BK - 1) / SBR_BK * SBR_BK;
    symm_dispatch<float, float, float>(m, nb, kchunk, splits, A, lda, Y, ldy, part, m, m * nb, s);
    reduce_slices(m, nb, splits, part, 1.0, 0.0, nullptr, 0, W, ldw, s);
}

void launch_cols_to_f64(int64_t m, int64_t nc, const float* As, int64_t lds, double* A, int64_t lda, hipStream_t s) {
    if (m <= 0 || nc <= 0) return;
    dim3 g((unsigned)cdiv(m, 1024) < 64 ? (unsigned)cdiv(m, 1024) : 64, (unsigned)nc);
    cols_to_f64_kernel<<<g, 256, 0, s>>>(m, As, lds, A, lda);
}

}  // namespace sbr
