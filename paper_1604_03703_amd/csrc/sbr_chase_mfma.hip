// sbr_chase_mfma.hip -- one reduction b -> h of the band (Algorithm 4.2,
// h = b / k) for b in {16, 32, 64, 128} and h in {b/2, b/4, b/8, b/16} (h >= 8),
// every product of a chase on FP64 MFMA.
//
// A chase (i, j) works on the rows [o, o + n_r) of the band, o = ih + (j-1)b
// (the same offsets and extents as the small-b kernels).  One work-group runs
// the chases of a sweep in order.  Chase (i, j > 1) factors its QR block and
// updates its left block right after chase (i, j-1): both lie in the previous
// chase's below block and no unfinished chase of sweep i-1 touches them
// (h <= b/2); chase (i, 1) first waits for the QR block of (i-1, 2).  The
// diagonal and below blocks wait until chase (i-1, j+2) has finished its QR
// block (the only entries the two chases share; the left block of (i-1, j+1)
// is done by then), so a sweep overlaps the rest of the chase two ahead of it
// in the previous sweep.  This holds for every k: chases of consecutive sweeps
// three or more apart are 3b - h >= 2b rows apart and touch no common entry.
// With [U, T, R] = QR(QR block, b x h) and Q = I - U T U^T:
//   left block  X_L  (rows [o, o+n_r), cols [o-b+h, o), j > 1): X_L <- Q^T X_L
//   below block X_B  (rows [o+b, o+2b), cols [o, o+n_r)):       X_B <- X_B Q
//   diagonal    D    (rows and cols [o, o+n_r), symmetric):     D   <- Q^T D Q
// computed as
//   X_L -= (U T^T)(U^T X_L)
//   X_B -= ((X_B U) T) U^T
//   W = (D U) T,  G = U^T W,  V = 1/2 (U T^T) G - W,  D += U V^T + V U^T.
// T comes from the identity T^{-1} = diag(1/tau) + strict upper part of U^T U
// (the compact WY form of a product of reflectors), inverted column by column.
// The left block is b - h columns wide (h for a halving); the QR block of chase
// j + 1 and its left block are the first h and the last b - h columns of chase
// j's below block.
//
// Wave w of the block owns the rows [16w, 16w + 16) of every b x h quantity.
// MFMA 16x16x4 lane layout: with a = R(k0 + l/16, c0 + l%16) and
// b = L(r0 + l%16, k0 + l/16), accumulator element r of lane l is
// (L R)(r0 + l%16, c0 + 4r + l/16).  A row tile held this way ("row-in-lane"
// layout) is, element for element, the b operand of a following product
// L' R' with L' = that tile; so the chains X_B U -> (.) T -> (.) U^T and
// D U -> (.) T stay in registers.  Cross-wave quantities (U, T, U^T X_L,
// U^T W) go through LDS; W goes through LDS or, when LDS is short (b = 128
// with h >= 32), a per-block global scratch slice.  h < 16 is padded to
// 16-wide tiles with zero columns.
//
// The update of D is split in two wave-local phases separated by a barrier:
// wave w adds V_w U_X^T to its own tiles (w, X <= w), then U_X V_w^T to the
// tiles (X >= w, w) of its column; every tile is read-modified-written by at
// most one wave per phase.
#include <type_traits>

#include "sbr_device.h"
#include "sbr_internal.h"

namespace {

struct MChaseArgs {
    int64_t n;
    double* band;
    int64_t ldb;
    int nsweeps;
    int* ticket;       // one int
    int* progress;     // nsweeps + 1 ints; progress[i] = chases of sweep i done
    double* gscratch;  // per-block W slices (b = 128)
    int64_t scratch_stride;
    int* error;        // the plan's status word: nonzero stops every block
    uint64_t wait_ticks;   // a wait gives up after this many ticks of the
                           // 100 MHz clock (it only bounds the kernel's lifetime
                           // should the schedule's progress guarantee break)
};

constexpr int MSWEEP_DONE = 1 << 30;

template <int B_, int H>
struct MChase {
    static constexpr int B = B_;
    static constexpr int HP = H < 16 ? 16 : H;   // h rounded up to whole 16-wide tiles
    static constexpr int HL = B - H;             // width of the left block
    static constexpr int CL = (HL + 15) / 16;    // its 16-wide tiles
    static constexpr int NW = B / 16;          // one wave per 16-row tile
    static constexpr int NT = 64 * NW;
    static constexpr int RT = B / 16, CT = HP / 16;
    static constexpr int LDU = B + 1, LDH = HP + 1;
    // CARRY: the updated below block stays in LDS for the next chase of the
    // sweep (its QR and left blocks), the diagonal and below blocks are loaded
    // into registers right after the wait, and the diagonal update is applied
    // to those registers (V goes through LDS).  One round trip to memory per
    // chase instead of one per block.
    static constexpr bool CARRY = B <= 64;
    static constexpr int LDX = B + 1;
    // W (b x h) in LDS unless the block's LDS would run short
    static constexpr bool WR_LDS = B * HP <= 2048;
    // LDS (doubles): U (b x h), T (h x h; QR staging before T exists), one
    // exchange buffer (L = T^{-1}, then U^T X_L (h x (b - h)), then U^T W), W
    // (b x h; V after G is formed), the carried below block (b x b);
    // for h < 16 the columns h .. 15 are zero padding
    static constexpr int RW = CL * 16 > HP ? CL * 16 : HP;   // exchange buffer columns
    static constexpr int US = 0;
    static constexpr int TS = US + LDU * HP;
    static constexpr int RS = TS + LDH * HP;
    static constexpr int WS = RS + LDH * RW;
    static constexpr int XS = WS + (WR_LDS ? B * HP : 0);
    static constexpr int TOTAL = XS + (CARRY ? B * LDX : 0);
    // QR: TPCQ lanes per column (8 for a halving, at most 16), the threads
    // t < h TPCQ take part
    static constexpr int TPCQ = (NT / H) < 16 ? (NT / H) : 16, RPT = B / TPCQ;
    static constexpr int QRT = H * TPCQ;
    static_assert(QRT <= NT && QRT % 64 == 0 && RPT * TPCQ == B, "QR layout");
    static_assert(2 * B + H <= LDH * HP, "QR staging fits in the T region");
    static_assert(TOTAL * 8 <= 160 * 1024, "LDS");
    // the QR staging (2 b + h doubles from the start of the T region) spills
    // into T's padding columns, which must be zero again before T is used
    static constexpr bool TPAD_DIRTY = HP > H && 2 * B + H > LDH * H;
};

__device__ __forceinline__ sbr_d4 mma(double a, double b, sbr_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ sbr_d4 zero4() { return sbr_d4{0.0, 0.0, 0.0, 0.0}; }
// The products of the WY applications take their precision from the
// accumulator: FP64 MFMA into sbr_d4, or (the FP32-MFMA form) operands
// rounded to FP32 and FP32 MFMA with FP32 accumulation into sbr_f4.  Both
// instructions have the same lane layout.
__device__ __forceinline__ sbr_d4 mmx(double a, double b, sbr_d4 c) { return mma(a, b, c); }
__device__ __forceinline__ sbr_f4 mmx(double a, double b, sbr_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
}
template <class Acc>
__device__ __forceinline__ Acc zacc() {
    return Acc{0, 0, 0, 0};
}

// acc + the chain of N products mma(fa(i), fb(i)), i = 0 .. N-1, in that order,
// with every operand read before the first product: left to itself the
// compiler issues each product right after its operand's LDS read and a wait
// for it.  Only where the registers allow it (two operands per step).
template <int N, class Acc, class FA, class FB>
__device__ __forceinline__ Acc mma_chain(Acc acc, const FA& fa, const FB& fb) {
    double a[N], b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        a[i] = fa(i);
        b[i] = fb(i);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) acc = mmx(a[i], b[i], acc);
    return acc;
}

// The value of lane q of each aligned group of 8 lanes, in all 8: quad_perm
// (q%4 x4) fills the quads, row_half_mirror (lane i <-> 7 - i) brings the
// source quad's value to the other quad.  q must fold to a constant.
__device__ __forceinline__ double bcast8(double v, int q) {
    double a;
    switch (q & 3) {
        case 0: a = dpp_d<0x00>(v); break;
        case 1: a = dpp_d<0x55>(v); break;
        case 2: a = dpp_d<0xAA>(v); break;
        default: a = dpp_d<0xFF>(v); break;
    }
    const double b = dpp_d<0x141>(a);
    return (((threadIdx.x >> 2) & 1) == (q >> 2)) ? a : b;
}

// A product over k = 0 .. B-1 in steps of 4 whose operand for step k0 comes
// from global memory: the operands of KB steps are loaded as a batch while
// the previous batch's products run (two batches in registers).  use(k0, v)
// issues the products of step k0.
template <int B, int KB, class LoadF, class UseF>
__device__ __forceinline__ void kloop_pipelined(const LoadF& load, const UseF& use) {
    constexpr int NS = B / 4;
    static_assert(NS % KB == 0, "batch size");
    double cur[KB], nxt[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) cur[u] = load(4 * u);
#pragma unroll 1
    for (int kb = 0; kb < NS; kb += KB) {
        if (kb + KB < NS) {
#pragma unroll
            for (int u = 0; u < KB; ++u) nxt[u] = load(4 * (kb + KB + u));
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) use(4 * (kb + u), cur[u]);
#pragma unroll
        for (int u = 0; u < KB; ++u) cur[u] = nxt[u];
    }
}

// The same product with the loads issued step by step (a partial unroll
// keeps a few in flight); used where the two batches of the pipelined form
// do not fit in the registers.
template <int B, class LoadF, class UseF>
__device__ __forceinline__ void kloop_plain(const LoadF& load, const UseF& use) {
#pragma unroll 4
    for (int k0 = 0; k0 < B; k0 += 4) use(k0, load(k0));
}

template <int B_, int H, bool F32>
__global__ __launch_bounds__((MChase<B_, H>::NT)) void chase_mfma_kernel(MChaseArgs a) {
    typedef MChase<B_, H> C;
    // accumulators of the WY applications (steps 4 - 10); the QR, L = U^T U
    // and T are FP64 in both forms
    typedef typename std::conditional<F32, sbr_f4, sbr_d4>::type Acc;
    constexpr int B = C::B, HP = C::HP, NW = C::NW, RT = C::RT, CT = C::CT, LDU = C::LDU, LDH = C::LDH;
    constexpr int TPCQ = C::TPCQ, RPT = C::RPT, LDX = C::LDX, HL = C::HL, CL = C::CL;
    constexpr bool CARRY = C::CARRY;
    extern __shared__ double sm[];
    double* Us = sm + C::US;
    double* Ts = sm + C::TS;
    double* Rs = sm + C::RS;
    double* vbuf = Ts;            // two reflectors in flight during the QR ...
    double* tau = Ts + 2 * B;     // ... and the tau, until T is formed
    double* Wsc = C::WR_LDS ? sm + C::WS : a.gscratch + (int64_t)blockIdx.x * a.scratch_stride;
    double* Xs = sm + C::XS;      // carried below block (CARRY only)
    __shared__ int sweep_sh;
    __shared__ int abort_sh;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // Accumulator element r of a WY product lies in column ocol(r) of its
    // 16 x 16 tile (row li): 4 r + lk for FP64 MFMA, 4 lk + r for FP32 MFMA.
    // A register-held operand (an accumulator, or a block loaded in that
    // layout) feeds k-step q of a following product, whose other operand is
    // then read at k = kq(q): the same k in both operands of every step.
    auto ocol = [&](int r) { return F32 ? 4 * lk + r : 4 * r + lk; };
    auto kq = [&](int q) { return 16 * (q >> 2) + ocol(q & 3); };
    const int qc = t / TPCQ, qs = t % TPCQ;
    const int64_t n = a.n, ldb = a.ldb;
    double* band = a.band;
    // band element (r, c), r >= c, of the chase-local rows/cols
    auto B_at = [&](int64_t r, int64_t c) -> double& { return band[(r - c) + c * ldb]; };

    if (HP > H) {
        // padding columns (h .. 15) of U, T and the exchange blocks are read by
        // the 16-wide tiles and must be zero; nothing writes them later
        for (int idx = t; idx < C::TOTAL; idx += C::NT) sm[idx] = 0.0;
        __syncthreads();
    }
    while (true) {
        if (t == 0) {
            const bool failed = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            sweep_sh = failed ? a.nsweeps + 1 : atomicAdd(a.ticket, 1) + 1;
            abort_sh = 0;
        }
        __syncthreads();
        const int i = sweep_sh;
        __syncthreads();
        if (i > a.nsweeps) break;
        const int64_t nchase = (n - 2 - (int64_t)i * H) / B + 1;
        // Wait until sweep i - 1 has published chase `need` (its QR block, or
        // the whole sweep); true when the stage is abandoned.
        auto wait_prev = [&](int need) -> bool {
            if (t == 0) {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(&a.progress[i - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        abort_sh = 1;
                        break;
                    }
                    if (wall_clock64() - t0 > a.wait_ticks) {
                        atomicOr(a.error, sbr::STATUS_STALLED);
                        abort_sh = 1;
                        break;
                    }
                }
                // one acquire for the block: it invalidates this CU's L1 and
                // the XCD's L2, which every wave of the block reads through
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            __syncthreads();
            return abort_sh != 0;
        };
        for (int64_t j = 1; j <= nchase; ++j) {
            // Schedule (every conflict ordered as in the loop nest; checked on
            // the model for every k): the QR block of chase (i, j > 1) is the
            // first h columns of this block's own previous below block and the
            // left block the rest, which no pending chase of sweep i - 1
            // touches, so both go ahead at once; chase (i, 1) first waits for
            // the QR block of (i - 1, 2).  The diagonal and below blocks wait
            // for the QR block of (i - 1, j + 2).
            if (i > 1 && j == 1) {
                if (wait_prev(2)) return;
            }
            const int64_t o = (int64_t)i * H + (j - 1) * B;
            const int nr = (int)((n - o < B) ? (n - o) : B);
            const int64_t cq = (j == 1) ? o - H : o - B;
            int64_t nb64 = n - (o + B);
            if (nb64 > B) nb64 = B;
            const int nbr = nb64 > 0 ? (int)nb64 : 0;

            // ---- 1. Householder QR of the QR block (rows [o, o+nr), cols
            // [cq, cq+h)): 8 lanes per column, one barrier per reflector.
            // With CARRY, chase j > 1 finds the block in LDS: it is the first
            // h columns of the previous chase's below block.
            // The first chase of a sweep stages its QR block through the same
            // LDS slots (each thread writes the entries it reads back), so the
            // registers of the reflector loop are only ever filled from LDS and
            // the loop never waits on the memory counter, which would also wait
            // for the previous chase's stores.
            const bool inqr = qc < H;   // wave-uniform (h TPCQ is a multiple of 64)
            {
                double x[RPT];
                if (CARRY && j == 1 && inqr) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int row = qs + TPCQ * r;
                        Xs[row + qc * LDX] = (row < nr) ? B_at(o + row, cq + qc) : 0.0;
                    }
                }
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int row = qs + TPCQ * r;
                    if (!inqr)
                        x[r] = 0.0;
                    else if (CARRY)
                        x[r] = (row < nr) ? Xs[row + qc * LDX] : 0.0;
                    else
                        x[r] = (row < nr) ? B_at(o + row, cq + qc) : 0.0;
                }
                for (int k = 0; k < H; ++k) {
                    double* v = vbuf + (k & 1) * B;
                    if (qc == k) {
                        double sq[RPT], xk = 0.0;
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            const int row = qs + TPCQ * r;
                            sq[r] = (row > k) ? x[r] * x[r] : 0.0;
                            if (row == k) xk = x[r];
                        }
                        const double ss = group_sum<TPCQ>(tree_sum<RPT>(sq));
                        xk = group_sum<TPCQ>(xk);
                        // beta = -sign(xk) ||x||, tau = (beta - xk) / beta =
                        // 1 + |xk| / ||x||, v below the diagonal = x / (xk - beta)
                        // = sign(xk) x / (|xk| + ||x||): one reciprocal square
                        // root and one reciprocal, Newton-refined
                        double beta, tk, scal;
                        if (ss == 0.0) {
                            beta = xk; tk = 0.0; scal = 0.0;
                        } else {
                            const double s2 = fma(xk, xk, ss);
                            const double sg = (xk >= 0.0) ? 1.0 : -1.0, ax = fabs(xk);
                            if (s2 > 1e-290 && s2 < 1e290) {
                                const double rs = sbr_rsqrt(s2);
                                const double nrm = s2 * rs;
                                beta = -sg * nrm;
                                tk = fma(ax, rs, 1.0);
                                scal = sg * sbr_recip(ax + nrm);
                            } else {
                                const double nrm = sqrt(s2);
                                beta = -sg * nrm;
                                tk = (beta - xk) / beta;
                                scal = 1.0 / (xk - beta);
                            }
                        }
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            const int row = qs + TPCQ * r;
                            const double vv = (row < k) ? 0.0 : ((row == k) ? 1.0 : x[r] * scal);
                            v[row] = vv;
                            x[r] = (row == k) ? beta : ((row > k) ? vv : x[r]);   // selects, no branches
                        }
                        if (qs == 0) tau[k] = tk;
                    }
                    __syncthreads();
                    if (qc > k && inqr) {
                        // tau and v in one round trip to LDS: a zero tau (v is
                        // then finite, its tail zero) leaves x as it is
                        const double tk = tau[k];
                        double vr[RPT], dp[RPT];
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            vr[r] = v[qs + TPCQ * r];
                            dp[r] = vr[r] * x[r];
                        }
                        const double f = tk * group_sum<TPCQ>(tree_sum<RPT>(dp));
#pragma unroll
                        for (int r = 0; r < RPT; ++r) x[r] -= f * vr[r];
                    }
                }
                // U (unit lower; a zero column where no reflector was applied)
                // into LDS, [R; 0] into the band
                if (inqr) {
                    const double tq = tau[qc];
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int row = qs + TPCQ * r;
                        double u = 0.0;
                        if (tq != 0.0) u = (row == qc) ? 1.0 : ((row > qc) ? x[r] : 0.0);
                        Us[row + qc * LDU] = u;
                        if (row < nr) B_at(o + row, cq + qc) = (row <= qc) ? x[r] : 0.0;
                    }
                }
            }
            // ---- publish the QR block: it is the only part of this chase that
            // chase (i+1, j-2) shares (its below block meets this QR block; the
            // rest of this chase lies beyond its columns), so sweep i+1 may go
            // on while this chase updates its left, diagonal and below blocks.
            // Every wave's stores complete to L2, then one agent-scope release
            // (L2 write-back) by thread 0 covers the block.
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (t == 0) sbr_store_release(&a.progress[i], (int)j);

            // ---- 2. L = T^{-1}: strict upper part of U^T U, tau on the diagonal
            // (the multiplier that replaces 1/tau below; a zero tau gives a zero
            // row and column of T)
            {
                constexpr int NTL = CT * (CT + 1) / 2;
                for (int idx = w; idx < NTL; idx += NW) {
                    int I = 0, rem = idx;
                    while (rem >= CT - I) { rem -= CT - I; ++I; }
                    const int J = I + rem;
                    sbr_d4 acc = zero4();
                    if constexpr (CARRY) {
                        acc = mma_chain<B / 4>(
                            acc, [&](int i) { return Us[(4 * i + lk) + (J * 16 + li) * LDU]; },
                            [&](int i) { return Us[(4 * i + lk) + (I * 16 + li) * LDU]; });
                    } else {
#pragma unroll 8
                        for (int k0 = 0; k0 < B; k0 += 4)
                            acc = mma(Us[(k0 + lk) + (J * 16 + li) * LDU], Us[(k0 + lk) + (I * 16 + li) * LDU], acc);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int gi = I * 16 + li, gj = J * 16 + 4 * r + lk;
                        Rs[gi + gj * LDH] = (gi < gj) ? acc[r] : ((gi == gj && gi < H) ? tau[gi] : 0.0);
                    }
                }
            }
            __syncthreads();

            // ---- 3. T by columns: T[j][j] = tau_j, T[i][j] = -tau_i sum_{i<k<=j}
            // L[i][k] T[k][j] for i = j-1 .. 0; 8 lanes per column.  Lane s
            // keeps the partial sums of the rows i = s (mod 8) in registers and
            // adds L[i][k] T[k][j] once T[k][j] is known; the owner of row k-1
            // then finishes T[k-1][j] and hands it to the other seven lanes
            // (two DPP moves), so each new entry costs one FMA, one product and
            // the hand-over.  Adding L[i][k] T[k][j] for i >= k is harmless:
            // L is zero below its diagonal and a row's sum is no longer read
            // once its entry is formed.
            if (t < 8 * H) {   // wave-uniform: 8 h is a multiple of 64
                constexpr int M = H / 8;
                const int jc = t >> 3, s = t & 7;
                double p[M], tr[M];
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    p[m] = 0.0;
                    tr[m] = Rs[(s + 8 * m) + (s + 8 * m) * LDH];
                }
                double tk = Rs[jc + jc * LDH];
                if (s == 0) Ts[jc + jc * LDH] = tk;
                for (int r = jc + 1 + s; r < HP; r += 8) Ts[r + jc * LDH] = 0.0;
#pragma unroll
                for (int k = H - 1; k >= 1; --k) {
                    if (k <= jc) {
#pragma unroll
                        for (int m = 0; m < M; ++m)
                            if (8 * m < k) p[m] += Rs[(s + 8 * m) + k * LDH] * tk;
                        const int q = (k - 1) & 7, mq = (k - 1) >> 3;
                        const double tn = -tr[mq] * p[mq];
                        if (s == q) Ts[(k - 1) + jc * LDH] = tn;
                        tk = bcast8(tn, q);
                    }
                }
            }
            if constexpr (C::TPAD_DIRTY) {
                for (int idx = t; idx < (HP - H) * HP; idx += C::NT) Ts[(idx % HP) + (H + idx / HP) * LDH] = 0.0;
            }
            __syncthreads();

            // ---- 4. Z_w = U_w T^T (row-in-lane, rows of this wave)
            Acc Z[CT];
#pragma unroll
            for (int J = 0; J < CT; ++J) {
                Z[J] = zacc<Acc>();
#pragma unroll
                for (int k0 = J * 16; k0 < HP; k0 += 4)     // T^T(k, c) = 0 for k < c
                    Z[J] = mmx(Ts[(J * 16 + li) + (k0 + lk) * LDH], Us[(w * 16 + li) + (k0 + lk) * LDU], Z[J]);
            }

            // ---- 5. left block (j > 1): M_L = U^T X_L into LDS, then X_L -= Z M_L
            if (j > 1) {
                for (int idx = w; idx < CT * CL; idx += NW) {
                    const int I = idx % CT, J = idx / CT;
                    const int64_t gc = o - HL + J * 16 + li;
                    const bool colv = J * 16 + li < HL;
                    Acc acc = zacc<Acc>();
                    if constexpr (CARRY) {
                        acc = mma_chain<B / 4>(
                            acc,
                            [&](int i) {
                                const int row = 4 * i + lk;
                                return (row < nr && colv) ? Xs[row + (H + J * 16 + li) * LDX] : 0.0;
                            },
                            [&](int i) { return Us[(4 * i + lk) + (I * 16 + li) * LDU]; });
                    } else {
                        kloop_pipelined<B, 4>(
                            [&](int k0) {
                                const int row = k0 + lk;
                                return (row < nr && colv) ? B_at(o + row, gc) : 0.0;
                            },
                            [&](int k0, double av) { acc = mmx(av, Us[(k0 + lk) + (I * 16 + li) * LDU], acc); });
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) Rs[(I * 16 + li) + (J * 16 + ocol(r)) * LDH] = acc[r];
                }
                __syncthreads();
                if (w * 16 < nr) {
#pragma unroll
                    for (int J = 0; J < CL; ++J) {
                        Acc acc = zacc<Acc>();
                        if constexpr (CARRY) {
                            acc = mma_chain<CT * 4>(
                                acc, [&](int i) { return Rs[kq(i) + (J * 16 + li) * LDH]; },
                                [&](int i) { return Z[i / 4][i % 4]; });
                        } else {
#pragma unroll
                            for (int K = 0; K < CT; ++K)
#pragma unroll
                                for (int r4 = 0; r4 < 4; ++r4)
                                    acc = mmx(Rs[(K * 16 + ocol(r4)) + (J * 16 + li) * LDH], Z[K][r4], acc);
                        }
                        const int row = w * 16 + li;
                        if (row < nr) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int col = J * 16 + ocol(r);
                                if (col < HL) {
                                    if (CARRY)
                                        B_at(o + row, o - HL + col) = Xs[row + (H + col) * LDX] - acc[r];
                                    else
                                        B_at(o + row, o - HL + col) -= acc[r];
                                }
                            }
                        }
                    }
                }
            }

            // ---- the diagonal and below blocks meet the QR block of chase
            // (i-1, j+2) and the left block of (i-1, j+1)
            if (i > 1) {
                if (wait_prev((int)(j + 2))) return;
            }

            // ---- (CARRY) the chase's diagonal block (full, from the lower
            // triangle) and below block, row-in-lane: element q of lane l is
            // (16 w + l%16, 4 q + l/16), loaded together
            constexpr int NQ = CARRY ? B / 4 : 1;
            double dr[NQ], xb[NQ];
            if (CARRY) {
                const int row = w * 16 + li;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int col = kq(q);
                    double dv = 0.0, bv = 0.0;
                    if (row < nr && col < nr) dv = (row >= col) ? B_at(o + row, o + col) : B_at(o + col, o + row);
                    if (row < nbr && col < nr) bv = B_at(o + B + row, o + col);
                    dr[q] = dv;
                    xb[q] = bv;
                }
            }

            // ---- 6. below block: P = X_B U, W_B = P T, X_B -= W_B U^T
            if (w * 16 < nbr) {
                const int row = w * 16 + li;
                Acc P[CT];
#pragma unroll
                for (int J = 0; J < CT; ++J) P[J] = zacc<Acc>();
                if constexpr (CARRY) {
                    // every U operand read from LDS before the first product
                    double ua[B / 4][CT];
#pragma unroll
                    for (int q = 0; q < B / 4; ++q)
#pragma unroll
                        for (int J = 0; J < CT; ++J) ua[q][J] = Us[kq(q) + (J * 16 + li) * LDU];
#pragma unroll
                    for (int q = 0; q < B / 4; ++q)
#pragma unroll
                        for (int J = 0; J < CT; ++J) P[J] = mmx(ua[q][J], xb[q], P[J]);
                } else {
                    kloop_plain<B>(
                        [&](int k0) {
                            const int col = k0 + lk;
                            return (row < nbr && col < nr) ? B_at(o + B + row, o + col) : 0.0;
                        },
                        [&](int k0, double bv) {
#pragma unroll
                            for (int J = 0; J < CT; ++J) P[J] = mmx(Us[(k0 + lk) + (J * 16 + li) * LDU], bv, P[J]);
                        });
                }
                Acc WB[CT];
#pragma unroll
                for (int J = 0; J < CT; ++J) {
                    WB[J] = zacc<Acc>();
#pragma unroll
                    for (int K = 0; K <= J; ++K)                // T(k, c) = 0 for k > c
#pragma unroll
                        for (int r4 = 0; r4 < 4; ++r4)
                            WB[J] = mmx(Ts[(K * 16 + ocol(r4)) + (J * 16 + li) * LDH], P[K][r4], WB[J]);
                }
                for (int X = 0; X < RT; ++X) {
                    if (X * 16 >= nr) break;
                    Acc acc = zacc<Acc>();
                    if constexpr (CARRY) {
                        acc = mma_chain<CT * 4>(
                            acc, [&](int i) { return Us[(X * 16 + li) + kq(i) * LDU]; },
                            [&](int i) { return WB[i / 4][i % 4]; });
                    } else {
#pragma unroll
                        for (int K = 0; K < CT; ++K)
#pragma unroll
                            for (int r4 = 0; r4 < 4; ++r4)
                                acc = mmx(Us[(X * 16 + li) + (K * 16 + ocol(r4)) * LDU], WB[K][r4], acc);
                    }
                    if (CARRY) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) xb[4 * X + r] -= acc[r];
                    } else if (row < nbr) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int col = X * 16 + ocol(r);
                            if (col < nr) B_at(o + B + row, o + col) -= acc[r];
                        }
                    }
                }
            }

            // ---- 7. diagonal block: W_w = (D_w U) T, to the exchange buffer
            Acc WR[CT];
            {
                const int row = w * 16 + li;
                Acc P[CT];
#pragma unroll
                for (int J = 0; J < CT; ++J) P[J] = zacc<Acc>();
                if constexpr (CARRY) {
                    // every U operand read from LDS before the first product
                    double ua[B / 4][CT];
#pragma unroll
                    for (int q = 0; q < B / 4; ++q)
#pragma unroll
                        for (int J = 0; J < CT; ++J) ua[q][J] = Us[kq(q) + (J * 16 + li) * LDU];
#pragma unroll
                    for (int q = 0; q < B / 4; ++q)
#pragma unroll
                        for (int J = 0; J < CT; ++J) P[J] = mmx(ua[q][J], dr[q], P[J]);
                } else {
                    kloop_plain<B>(
                        [&](int k0) {
                            const int col = k0 + lk;
                            double dv = 0.0;
                            if (row < nr && col < nr) dv = (row >= col) ? B_at(o + row, o + col) : B_at(o + col, o + row);
                            return dv;
                        },
                        [&](int k0, double bv) {
#pragma unroll
                            for (int J = 0; J < CT; ++J) P[J] = mmx(Us[(k0 + lk) + (J * 16 + li) * LDU], bv, P[J]);
                        });
                }
#pragma unroll
                for (int J = 0; J < CT; ++J) {
                    WR[J] = zacc<Acc>();
#pragma unroll
                    for (int K = 0; K <= J; ++K)
#pragma unroll
                        for (int r4 = 0; r4 < 4; ++r4)
                            WR[J] = mmx(Ts[(K * 16 + ocol(r4)) + (J * 16 + li) * LDH], P[K][r4], WR[J]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) Wsc[row + (J * 16 + ocol(r)) * B] = WR[J][r];
                }
            }
            __syncthreads();
            // ---- (CARRY) the updated below block to LDS for the next chase,
            // whose QR and left blocks write every entry of it back; the
            // sweep's last chase stores it (every wave is past the left
            // block's reads of the previous contents)
            if (CARRY) {
                const int row = w * 16 + li;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int col = kq(q);
                    Xs[row + col * LDX] = xb[q];
                    if (j == nchase && row < nbr && col < nr) B_at(o + B + row, o + col) = xb[q];
                }
            }

            // ---- 8. G = U^T W into LDS (the left block is done with it)
            for (int idx = w; idx < CT * CT; idx += NW) {
                const int I = idx % CT, J = idx / CT;
                Acc acc = zacc<Acc>();
                if constexpr (CARRY) {
                    acc = mma_chain<B / 4>(
                        acc, [&](int i) { return Wsc[(4 * i + lk) + (J * 16 + li) * B]; },
                        [&](int i) { return Us[(4 * i + lk) + (I * 16 + li) * LDU]; });
                } else {
#pragma unroll 8
                    for (int k0 = 0; k0 < B; k0 += 4)
                        acc = mmx(Wsc[(k0 + lk) + (J * 16 + li) * B], Us[(k0 + lk) + (I * 16 + li) * LDU], acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) Rs[(I * 16 + li) + (J * 16 + ocol(r)) * LDH] = acc[r];
            }
            __syncthreads();

            // ---- 9. V_w = 1/2 Z_w G - W_w
            Acc V[CT];
#pragma unroll
            for (int J = 0; J < CT; ++J) {
                Acc acc = zacc<Acc>();
                if constexpr (CARRY) {
                    acc = mma_chain<CT * 4>(
                        acc, [&](int i) { return Rs[kq(i) + (J * 16 + li) * LDH]; },
                        [&](int i) { return Z[i / 4][i % 4]; });
                } else {
#pragma unroll
                    for (int K = 0; K < CT; ++K)
#pragma unroll
                        for (int r4 = 0; r4 < 4; ++r4)
                            acc = mmx(Rs[(K * 16 + ocol(r4)) + (J * 16 + li) * LDH], Z[K][r4], acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) V[J][r] = 0.5 * acc[r] - WR[J][r];
            }

            if (CARRY) {
                // ---- 10. D += V U^T + U V^T on the registers of the diagonal
                // block: wave w forms its tiles (w, X <= w) from V_w U_X^T and
                // U_w V_X^T, V through LDS (in place of W, which G has consumed)
                double* Vs = Wsc;
                const int row = w * 16 + li;
#pragma unroll
                for (int J = 0; J < CT; ++J)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Vs[row + (J * 16 + ocol(r)) * B] = V[J][r];
                __syncthreads();
#pragma unroll
                for (int X = 0; X < RT; ++X) {
                    if (X > w || X * 16 >= nr) break;
                    Acc acc = mma_chain<CT * 4>(
                        zacc<Acc>(), [&](int i) { return Us[(X * 16 + li) + kq(i) * LDU]; },
                        [&](int i) { return V[i / 4][i % 4]; });
                    acc = mma_chain<HP / 4>(
                        acc, [&](int i) { return Vs[(X * 16 + li) + (4 * i + lk) * B]; },
                        [&](int i) { return Us[row + (4 * i + lk) * LDU]; });
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int col = X * 16 + ocol(r);
                        if (row < nr && col <= row) B_at(o + row, o + col) = dr[4 * X + r] + acc[r];
                    }
                }
            } else {
            // ---- 10. D += V U^T + U V^T, lower triangle: tiles (w, X <= w)
            // with V_w U_X^T, then tiles (X >= w, w) with U_X V_w^T
            if (w * 16 < nr) {
                const int row = w * 16 + li;
                for (int X = 0; X <= w; ++X) {
                    Acc acc = zacc<Acc>();
#pragma unroll
                    for (int K = 0; K < CT; ++K)
#pragma unroll
                        for (int r4 = 0; r4 < 4; ++r4)
                            acc = mmx(Us[(X * 16 + li) + (K * 16 + ocol(r4)) * LDU], V[K][r4], acc);
                    if (row < nr) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int col = X * 16 + ocol(r);
                            if (col <= row) B_at(o + row, o + col) += acc[r];
                        }
                    }
                }
            }
            __syncthreads();
            for (int X = w; X < RT; ++X) {
                if (X * 16 >= nr) break;
                Acc acc = zacc<Acc>();
#pragma unroll
                for (int K = 0; K < CT; ++K)
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4)
                        acc = mmx(V[K][r4], Us[(X * 16 + li) + (K * 16 + ocol(r4)) * LDU], acc);
                const int row = X * 16 + li;
                if (row < nr) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int col = w * 16 + ocol(r);
                        if (col <= row) B_at(o + row, o + col) += acc[r];
                    }
                }
            }
            }

            // ---- the sweep's last chase: publish the whole sweep (a chase of
            // sweep i+1 without a partner two chases ahead waits for it)
            if (j == nchase) {
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (t == 0) sbr_store_release(&a.progress[i], MSWEEP_DONE);
            }
        }
    }
}

template <int H>
int mchase_grid(int64_t n) {
    const int64_t nsweeps = (n - 2) / H;
    const int64_t cap = 256;
    int64_t g = nsweeps < cap ? nsweeps : cap;
    return (int)(g < 1 ? 1 : g);
}

template <int B, int H, bool F32>
void launch_mchase(int64_t n, double* band, int64_t ldb, double* scratch, const sbr::StageCtl& ctl, hipStream_t s) {
    const int64_t nsweeps = (n - 2) / H;
    if (nsweeps < 1) return;
    typedef MChase<B, H> C;
    MChaseArgs a;
    a.n = n;
    a.band = band;
    a.ldb = ldb;
    a.nsweeps = (int)nsweeps;
    a.ticket = ctl.flags;
    a.progress = ctl.flags + 1;
    a.gscratch = scratch;
    a.scratch_stride = (int64_t)C::B * C::HP;
    a.error = ctl.status;
    a.wait_ticks = ctl.wait_ticks;
    sbr::launch_fill_int(ctl.flags, nsweeps + 2, 0, s);
    int grid = mchase_grid<H>(n);
    if (ctl.max_grid > 0 && grid > ctl.max_grid) grid = ctl.max_grid;
    chase_mfma_kernel<B, H, F32><<<grid, C::NT, (size_t)C::TOTAL * sizeof(double), s>>>(a);
}

template <int B, int H>
int set_mchase_attr() {
    const int bytes = MChase<B, H>::TOTAL * (int)sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)chase_mfma_kernel<B, H, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)chase_mfma_kernel<B, H, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e == hipSuccess ? 0 : (int)e;
}

// global W scratch (doubles) of one (b, h) kernel: its grid's slices
template <int B, int H>
int64_t mchase_scratch(int64_t n) {
    typedef MChase<B, H> C;
    return C::WR_LDS ? 0 : (int64_t)mchase_grid<H>(n) * C::B * C::HP;
}

}  // namespace

namespace sbr {

bool band_mfma_supported(int b) { return b == 16 || b == 32 || b == 64 || b == 128; }

bool band_reduce_mfma_supported(int b, int h) {
    if (!band_mfma_supported(b) || h < 8 || h >= b || b % h) return false;
    return true;
}

int64_t band_mfma_workspace_doubles(int64_t n, int b) {
    if (b < 128) return 0;
    const int64_t a = mchase_scratch<128, 64>(n), c = mchase_scratch<128, 32>(n);
    return a > c ? a : c;
}

template <bool F32>
void launch_band_reduce_mfma_t(int64_t n, double* band, int64_t ldband, int b, int h, double* scratch,
                               const StageCtl& ctl, hipStream_t s) {
    switch (b * 1000 + h) {
        case 16008: launch_mchase<16, 8, F32>(n, band, ldband, scratch, ctl, s); break;
        case 32016: launch_mchase<32, 16, F32>(n, band, ldband, scratch, ctl, s); break;
        case 32008: launch_mchase<32, 8, F32>(n, band, ldband, scratch, ctl, s); break;
        case 64032: launch_mchase<64, 32, F32>(n, band, ldband, scratch, ctl, s); break;
        case 64016: launch_mchase<64, 16, F32>(n, band, ldband, scratch, ctl, s); break;
        case 64008: launch_mchase<64, 8, F32>(n, band, ldband, scratch, ctl, s); break;
        case 128064: launch_mchase<128, 64, F32>(n, band, ldband, scratch, ctl, s); break;
        case 128032: launch_mchase<128, 32, F32>(n, band, ldband, scratch, ctl, s); break;
        case 128016: launch_mchase<128, 16, F32>(n, band, ldband, scratch, ctl, s); break;
        case 128008: launch_mchase<128, 8, F32>(n, band, ldband, scratch, ctl, s); break;
        default: break;
    }
}

void launch_band_reduce_mfma(int64_t n, double* band, int64_t ldband, int b, int h, bool f32, double* scratch,
                             const StageCtl& ctl, hipStream_t s) {
    if (f32)
        launch_band_reduce_mfma_t<true>(n, band, ldband, b, h, scratch, ctl, s);
    else
        launch_band_reduce_mfma_t<false>(n, band, ldband, b, h, scratch, ctl, s);
}

void launch_band_halve_mfma(int64_t n, double* band, int64_t ldband, int b, bool f32, double* scratch,
                            const StageCtl& ctl, hipStream_t s) {
    launch_band_reduce_mfma(n, band, ldband, b, b / 2, f32, scratch, ctl, s);
}

int init_band_mfma_attributes() {
    int rc = 0;
    rc |= set_mchase_attr<16, 8>();
    rc |= set_mchase_attr<32, 16>();
    rc |= set_mchase_attr<32, 8>();
    rc |= set_mchase_attr<64, 32>();
    rc |= set_mchase_attr<64, 16>();
    rc |= set_mchase_attr<64, 8>();
    rc |= set_mchase_attr<128, 64>();
    rc |= set_mchase_attr<128, 32>();
    rc |= set_mchase_attr<128, 16>();
    rc |= set_mchase_attr<128, 8>();
    return rc;
}

}  // namespace sbr
