// sbr_batched.hip -- the batched form: many independent symmetric matrices
// (n <= 512), each taken through the same steps as the single-matrix path
// (Algorithm 4.1 full-to-band with the Eq. (4.1) update, Algorithm 4.2
// halvings with k = 2 down to a tridiagonal, Sturm bisection), one matrix per
// work-group instead of one step per grid.
//
// Three persistent kernel kinds take matrices from a ticket counter, largest
// first (the host orders the descriptors by decreasing n):
//   * batched_f2b_kernel: 8 waves per matrix.  Per panel (width b <= 16, the
//     tiles padded to 16 columns): Householder QR of the m x b panel (the
//     single-leaf case of Algorithm 3.2, which yields U, tau and R directly,
//     so Corollary 3.7's reconstruction is not needed); T from
//     T^{-1} = diag(1/tau) + striu(U^T U); W = (A22 U) T; Z = U^T W;
//     V = 1/2 U (T^T Z) - W; A22 += U V^T + V U^T on lower tiles.  FP64
//     MFMA 16x16x4 throughout, U and T in LDS, W and V in a per-block
//     global scratch slice.
//   * batched_band_kernel<h>: one wavefront per matrix for the halving
//     b = 2h -> h, teams of 2h lanes each chasing one sweep (the team chase of
//     the small-bandwidth path) in the lag-3 order: chase (i, j) runs after
//     chase (i, j-1) and after sweep i-1 has finished chase j + 2.  The band
//     lives in a per-matrix global buffer with ld 2b + 1; the halvings
//     h = 2 and 1 move it into LDS first and chase it there.
//   * batched_bisect_kernel: one wavefront per matrix, d and e^2 in LDS, each
//     lane bisecting up to 8 eigenvalue indices in lockstep.
#include <float.h>
#include <type_traits>

#include "sbr_device.h"
#include "sbr_internal.h"
#include "sbr_team_chase.h"

namespace {

using sbr::BatchDesc;

constexpr int BF_NT = 512;                 // 8 waves
constexpr int BF_NW = BF_NT / 64;
constexpr int BF_MP = sbr::BATCH_NMAX;     // panel rows held in LDS
constexpr int BF_LDU = BF_MP + 1;          // U column-major, padded ld
constexpr int BF_LDT = 17;                 // 16 x 16 blocks, padded ld
constexpr int BF_TPC = 32;                 // QR: lanes per column (16 columns x 32 = 512)
constexpr int BF_RPT = BF_MP / BF_TPC;     // QR: rows per lane
// LDS (doubles): U | T | L | M | Z partials (4 x 256; the QR staging of two
// reflectors aliases it) | tau
constexpr int BF_US = 0;
constexpr int BF_TS = BF_US + BF_LDU * 16;
constexpr int BF_LS = BF_TS + BF_LDT * 16;
constexpr int BF_MS = BF_LS + BF_LDT * 16;
constexpr int BF_ZP = BF_MS + BF_LDT * 16;
constexpr int BF_TAU = BF_ZP + 4 * 256;
constexpr int BF_TOTAL = BF_TAU + 16;
static_assert(4 * 256 >= 2 * BF_MP, "QR staging fits in the partial-product area");

__device__ __forceinline__ sbr_d4 mma(double a, double b, sbr_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ sbr_d4 zero4() { return sbr_d4{0.0, 0.0, 0.0, 0.0}; }
// Products of the trailing update in the precision of their accumulator:
// FP64 MFMA into sbr_d4, or operands rounded to FP32 and FP32 MFMA with FP32
// accumulation into sbr_f4 (the FP32-MFMA form).
__device__ __forceinline__ sbr_d4 mmx(double a, double b, sbr_d4 c) { return mma(a, b, c); }
__device__ __forceinline__ sbr_f4 mmx(double a, double b, sbr_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
}
template <class Acc>
__device__ __forceinline__ Acc zacc() {
    return Acc{0, 0, 0, 0};
}

// All-reduce over the 32 lanes of an aligned half-wave: 16-lane DPP sums, then
// the two halves exchanged.
__device__ __forceinline__ double sum32(double v) {
    v = team_sum<16>(v);
    return v + __shfl_xor(v, 16);
}

// MFMA lane layout used below: with a = R(k0 + l/16, c0 + l%16) and
// b = L(r0 + l%16, k0 + l/16), element r of the accumulator of lane l is
// (L R)(r0 + l%16, c0 + 4r + l/16) for FP64 MFMA and (L R)(r0 + l%16,
// c0 + 4 (l/16) + r) for FP32 MFMA (ocol below).
// F32: the trailing update (W, Z, V and the A22 update) on FP32 MFMA with
// FP32 accumulation, the results added into the FP64 matrix; the panel QR,
// tau, U^T U and T stay FP64.
// Two work-groups a CU (two waves a SIMD: the register budget spills about
// 100 values to scratch; 41.4 against 42.8 ms per 4096 matrices with one
// work-group a CU and no spills).
template <bool F32>
__global__ __launch_bounds__(BF_NT) __attribute__((amdgpu_waves_per_eu(4))) void batched_f2b_kernel(const BatchDesc* __restrict__ desc, int count,
                                                            int* ticket, double* scratch) {
    typedef typename std::conditional<F32, sbr_f4, sbr_d4>::type Acc;
    extern __shared__ double sm[];
    double* Us = sm + BF_US;
    double* Ts = sm + BF_TS;
    double* Ls = sm + BF_LS;
    double* Ms = sm + BF_MS;
    double* Zp = sm + BF_ZP;
    double* vbuf = Zp;
    double* tau = sm + BF_TAU;
    __shared__ int mat_sh;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // tile column of accumulator element r (the FP32 instruction's layout
    // differs from the FP64 one)
    auto ocol = [&](int r) { return F32 ? 4 * lk + r : 4 * r + lk; };
    double* Wg = scratch + (int64_t)blockIdx.x * (2 * BF_MP * 16);   // W, column-major, ld BF_MP
    double* Vg = Wg + BF_MP * 16;                                    // V, same layout

    while (true) {
        if (t == 0) mat_sh = atomicAdd(ticket, 1);
        __syncthreads();
        const int mi = mat_sh;
        __syncthreads();
        if (mi >= count) break;
        const BatchDesc dm = desc[mi];
        const int n = dm.n, B = dm.b0;
        const int64_t lda = dm.lda;
        double* A = dm.A;
        if (B < 2) continue;
        for (int c0 = 0;; c0 += B) {
            const int r0 = c0 + B, m = n - r0;
            if (m < 2) break;
            double* P = A + r0 + (int64_t)c0 * lda;
            double* A22 = A + r0 + (int64_t)r0 * lda;

            // ---- 1. Householder QR of the m x b panel (32 lanes per column)
            {
                const int qc = t / BF_TPC, qs = t % BF_TPC;
                const bool qa = qc < B;
                double x[BF_RPT];
#pragma unroll
                for (int r = 0; r < BF_RPT; ++r) {
                    const int row = qs + BF_TPC * r;
                    x[r] = (qa && row < m) ? P[row + (int64_t)qc * lda] : 0.0;
                }
                for (int k = 0; k < B; ++k) {
                    double* v = vbuf + (k & 1) * BF_MP;
                    if (qc == k) {
                        double ss = 0.0, xk = 0.0;
#pragma unroll
                        for (int r = 0; r < BF_RPT; ++r) {
                            const int row = qs + BF_TPC * r;
                            ss += (row > k) ? x[r] * x[r] : 0.0;
                            xk += (row == k) ? x[r] : 0.0;
                        }
                        ss = sum32(ss);
                        xk = sum32(xk);
                        const bool none = (ss == 0.0);
                        const double nrm = sqrt(xk * xk + ss);
                        const double beta = none ? xk : ((xk >= 0.0) ? -nrm : nrm);
                        const double tk = none ? 0.0 : (beta - xk) / beta;
                        const double scal = none ? 0.0 : 1.0 / (xk - beta);
#pragma unroll
                        for (int r = 0; r < BF_RPT; ++r) {
                            const int row = qs + BF_TPC * r;
                            const double vv = (row < k) ? 0.0 : ((row == k) ? 1.0 : x[r] * scal);
                            v[row] = vv;
                            x[r] = (row == k) ? beta : ((row > k) ? vv : x[r]);
                        }
                        if (qs == 0) tau[k] = tk;
                    }
                    __syncthreads();
                    if (qa && qc > k) {
                        const double tk = tau[k];
                        double d = 0.0;
#pragma unroll
                        for (int r = 0; r < BF_RPT; ++r) d += v[qs + BF_TPC * r] * x[r];
                        d = sum32(d);
                        const double f = tk * d;
#pragma unroll
                        for (int r = 0; r < BF_RPT; ++r) x[r] -= f * v[qs + BF_TPC * r];
                    }
                }
                // U (a zero column where no reflector), [R; 0] back into A; the
                // padding columns b .. 15 of U are zero
                {
                    const double tq = qa ? tau[qc] : 0.0;
#pragma unroll
                    for (int r = 0; r < BF_RPT; ++r) {
                        const int row = qs + BF_TPC * r;
                        double u = 0.0;
                        if (tq != 0.0) u = (row == qc) ? 1.0 : ((row > qc) ? x[r] : 0.0);
                        Us[row + qc * BF_LDU] = u;
                        if (qa && row < m) P[row + (int64_t)qc * lda] = (row <= qc) ? x[r] : 0.0;
                    }
                }
            }
            __syncthreads();

            // ---- 2. L = striu(U^T U) + diag(tau): four waves split the rows
            if (w < 4) {
                const int kb = (m + 3) / 4;
                const int ka = w * kb, ke = (ka + kb < m) ? ka + kb : m;
                sbr_d4 acc = zero4();
                for (int k0 = ka; k0 < ke; k0 += 4) {
                    const int k = k0 + lk;
                    const double uv = (k < ke) ? Us[k + li * BF_LDU] : 0.0;
                    const double ub = (k < ke) ? Us[k + li * BF_LDU] : 0.0;
                    acc = mma(uv, ub, acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) Zp[w * 256 + li + (4 * r + lk) * 16] = acc[r];
            }
            __syncthreads();
            if (t < 256) {
                const int gi = t % 16, gj = t / 16;
                const double g = Zp[t] + Zp[256 + t] + Zp[512 + t] + Zp[768 + t];
                Ls[gi + gj * BF_LDT] = (gi < gj) ? g : ((gi == gj && gi < B) ? tau[gi] : 0.0);
            }
            __syncthreads();

            // ---- 3. T = L^{-1} by columns (8 lanes per column)
            if (t < 128) {
                const int jc = t >> 3, s = t & 7;
                const int jmax = ((t >> 6) << 3) + 7;
                if (s == 0) Ts[jc + jc * BF_LDT] = Ls[jc + jc * BF_LDT];
                for (int r = jc + 1 + s; r < 16; r += 8) Ts[r + jc * BF_LDT] = 0.0;
                for (int r = jmax - 1; r >= 0; --r) {
                    double p = 0.0;
                    if (r < jc)
                        for (int k = r + 1 + s; k <= jc; k += 8) p += Ls[r + k * BF_LDT] * Ts[k + jc * BF_LDT];
                    p = group_sum<8>(p);
                    if (r < jc && s == 0) Ts[r + jc * BF_LDT] = -Ls[r + r * BF_LDT] * p;
                }
            }
            __syncthreads();

            // ---- 4. W = (A22 U) T by row tiles; W kept in registers (at most
            // 4 row tiles per wave) and written to the scratch slice
            const int nI = (m + 15) / 16;
            Acc Wr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Wr[q] = zacc<Acc>();
                const int I = w + q * BF_NW;
                if (I < nI) {
                    const int row = I * 16 + li;
                    Acc acc = zacc<Acc>();
                    // 32 columns of A22 a batch: their loads are in flight
                    // together, then the batch's products in column order
                    for (int k0 = 0; k0 < m; k0 += 32) {
                        double bv[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int col = k0 + 4 * j + lk;
                            double v = 0.0;
                            if (row < m && col < m)
                                v = (row >= col) ? A22[row + (int64_t)col * lda] : A22[col + (int64_t)row * lda];
                            bv[j] = v;
                        }
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int col = k0 + 4 * j + lk;
                            const double av = (col < m) ? Us[col + li * BF_LDU] : 0.0;
                            acc = mmx(av, bv[j], acc);
                        }
                    }
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4)
                        Wr[q] = mmx(Ts[ocol(r4) + li * BF_LDT], acc[r4], Wr[q]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) Wg[row + ocol(r) * BF_MP] = Wr[q][r];
                }
            }
            __syncthreads();

            // ---- 5. Z = U^T W (four waves over row quarters), M = T^T Z
            if (w < 4) {
                const int kb = (m + 3) / 4;
                const int ka = w * kb, ke = (ka + kb < m) ? ka + kb : m;
                Acc acc = zacc<Acc>();
                // W rows in batches of 32, loads in flight together
                for (int k0 = ka; k0 < ke; k0 += 32) {
                    double wv[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int k = k0 + 4 * j + lk;
                        wv[j] = (k < ke) ? Wg[k + li * BF_MP] : 0.0;
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int k = k0 + 4 * j + lk;
                        const double ub = (k < ke) ? Us[k + li * BF_LDU] : 0.0;
                        acc = mmx(wv[j], ub, acc);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) Zp[w * 256 + li + ocol(r) * 16] = acc[r];
            }
            __syncthreads();
            if (t < 256) {
                const int gi = t % 16, gj = t / 16;
                double mv = 0.0;
                for (int k = 0; k <= gi; ++k) {
                    const int e = k + gj * 16;
                    mv += Ts[k + gi * BF_LDT] * (Zp[e] + Zp[256 + e] + Zp[512 + e] + Zp[768 + e]);
                }
                Ms[gi + gj * BF_LDT] = mv;
            }
            __syncthreads();

            // ---- 6. V = 1/2 U M - W by row tiles, to the scratch slice
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int I = w + q * BF_NW;
                if (I < nI) {
                    const int row = I * 16 + li;
                    Acc acc = zacc<Acc>();
#pragma unroll
                    for (int k0 = 0; k0 < 16; k0 += 4)
                        acc = mmx(Ms[(k0 + lk) + li * BF_LDT], Us[row + (k0 + lk) * BF_LDU], acc);
#pragma unroll
                    for (int r = 0; r < 4; ++r) Vg[row + ocol(r) * BF_MP] = 0.5 * acc[r] - Wr[q][r];
                }
            }
            __syncthreads();

            // ---- 7. A22 += U V^T + V U^T, lower tiles: [U_I, V_I] [V_J, U_J]^T.
            // Two tiles at a time (x and x + 8 of the wave's share): the old
            // entries and the V operands of both are loaded before the first
            // product, so their round trips overlap.
            const int ntl = nI * (nI + 1) / 2;
            for (int x0 = w; x0 < ntl; x0 += 2 * BF_NW) {
                int ri[2], rj[2], Jt[2];
                bool ok[2];
                double old[2][4], vj[2][4], vi[2][4];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const int x = x0 + p * BF_NW;
                    ok[p] = x < ntl;
                    int I = 0, J = 0;
                    if (ok[p]) {
                        I = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
                        while (I * (I + 1) / 2 > x) --I;
                        while ((I + 1) * (I + 2) / 2 <= x) ++I;
                        J = x - I * (I + 1) / 2;
                    }
                    ri[p] = I * 16 + li;
                    rj[p] = J * 16 + li;
                    Jt[p] = J;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int cj = J * 16 + ocol(r);
                        old[p][r] = (ok[p] && ri[p] < m && cj <= ri[p]) ? A22[ri[p] + (int64_t)cj * lda] : 0.0;
                    }
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int k = 4 * kk + lk;
                        vj[p][kk] = ok[p] ? Vg[rj[p] + k * BF_MP] : 0.0;
                        vi[p][kk] = ok[p] ? Vg[ri[p] + k * BF_MP] : 0.0;
                    }
                }
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    if (!ok[p]) continue;
                    Acc acc = zacc<Acc>();
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) acc = mmx(vj[p][kk], Us[ri[p] + (4 * kk + lk) * BF_LDU], acc);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) acc = mmx(Us[rj[p] + (4 * kk + lk) * BF_LDU], vi[p][kk], acc);
                    if (ri[p] < m) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int cj = Jt[p] * 16 + ocol(r);
                            if (cj <= ri[p]) A22[ri[p] + (int64_t)cj * lda] = old[p][r] + acc[r];
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Band halvings: one wavefront per matrix, S = 64 / 2h teams.  LB: the
// matrix's band (n x (2b + 1) doubles, b = 2h) is moved into LDS when the
// wavefront takes the matrix, chased there, and the h + 1 diagonals the next
// stage needs are written out at the end; otherwise the chases work on the
// band in its global buffer.  The chases are the same either way.

template <int H>
constexpr int batched_band_lds_doubles() { return sbr::BATCH_NMAX * (4 * H + 1); }

// h = 8: two waves a SIMD (the register budget spills 76 values to scratch;
// 50.9 against 53.5 ms per 4096 matrices with one wave a SIMD and no spills).
template <int H, bool LB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(H == 8 ? 2 : 1))) void batched_band_kernel(const BatchDesc* __restrict__ desc, int count,
                                                          int* ticket) {
    constexpr int TEAM = 2 * H, S = 64 / TEAM, H2 = 2 * H, LDW = 4 * H + 1;
    extern __shared__ double bsm[];   // LB: the band, ld LDW
    __shared__ double scr_all[S * team_chase_scratch<H>()];
    __shared__ int psweep[S], pdone[S];
    __shared__ int mat_sh;
    const int t = threadIdx.x;
    const int tm = t / TEAM, u = t % TEAM;
    double* scr = scr_all + tm * team_chase_scratch<H>();

    while (true) {
        if (t == 0) mat_sh = atomicAdd(ticket, 1);
        team_sync<64>();
        const int mi = mat_sh;
        team_sync<64>();
        if (mi >= count) break;
        const BatchDesc dm = desc[mi];
        const int n = dm.n, b0 = dm.b0;
        if (b0 < 2 * H) continue;
        // stage index s = log2(b0 / b): even stages work in bandA, odd in bandB
        int stage = 0;
        for (int bb = b0; bb > 2 * H; bb >>= 1) ++stage;
        double* const gband = (stage & 1) ? dm.bandB : dm.bandA;
        double* next = (stage & 1) ? dm.bandA : dm.bandB;
        double* const band = LB ? bsm : gband;
        if (stage == 0) {
            // the lower band of the dense A (after full-to-band), headroom zero
            for (int64_t idx = t; idx < (int64_t)n * LDW; idx += 64) {
                const int d = (int)(idx % LDW), c = (int)(idx / LDW);
                band[idx] = (d <= H2 && c + d < n) ? dm.A[(c + d) + (int64_t)c * dm.lda] : 0.0;
            }
        } else if (LB) {
            for (int64_t idx = t; idx < (int64_t)n * LDW; idx += 64) band[idx] = gband[idx];
        }
        if (stage == 0 || LB) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            team_sync<64>();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        auto R = [&](int r, int c) -> double& { return band[(r - c) + (int64_t)c * LDW]; };
        const int nsweeps = (n - 2) / H;
        auto Jof = [&](int i) -> int { return (n - 2 - i * H) / H2 + 1; };
        if (u == 0 && tm < S) {
            psweep[tm] = tm + 1;
            pdone[tm] = 0;
        }
        team_sync<64>();
        while (true) {
            // state at the start of the step
            const int i = psweep[tm], jd = pdone[tm];
            bool act = (i <= nsweeps);
            const int j = jd + 1;
            if (act && i > 1) {
                const int sp = (tm + S - 1) % S;
                const int ip = psweep[sp], dp = pdone[sp];
                // sweep i-1 is finished once its team moved past it
                act = (ip > i - 1) || (ip == i - 1 && dp >= j + 2);
            }
            if (!__any(psweep[tm] <= nsweeps)) break;
            team_sync<64>();
            if (act) {
                const int o = i * H + (j - 1) * H2;
                const int nr = (n - o < H2) ? n - o : H2;
                const int cq = (j == 1) ? o - H : o - H2;
                int nbl = n - (o + H2);
                if (nbl > H2) nbl = H2;
                const int nbr = nbl > 0 ? nbl : 0;
                team_chase<H>(R, o, cq, nr, nbr, j, u, scr);
            }
            // band writes of this step complete before any team reads them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            team_sync<64>();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (act && u == 0) {
                if (j == Jof(i)) {
                    psweep[tm] = i + S;
                    pdone[tm] = 0;
                } else {
                    pdone[tm] = j;
                }
            }
            team_sync<64>();
        }
        // keep the h + 1 diagonals: into the next buffer with ld 2h + 1, or d
        // and e for the bisection after the last halving
        if (H == 1) {
            double* de = dm.de;
            for (int c = t; c < n; c += 64) {
                de[c] = band[(int64_t)c * LDW];
                de[n + c] = (c + 1 < n) ? band[1 + (int64_t)c * LDW] : 0.0;
            }
        } else {
            constexpr int LDN = 2 * H + 1;
            for (int64_t idx = t; idx < (int64_t)n * LDN; idx += 64) {
                const int d = (int)(idx % LDN), c = (int)(idx / LDN);
                next[idx] = (d <= H && c + d < n) ? band[d + (int64_t)c * LDW] : 0.0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        team_sync<64>();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// ---------------------------------------------------------------------------
// Sturm bisection per matrix (the same counts, interval and final width as
// the single-matrix kernels, by plain bisection from the whole interval).

constexpr int BB_NT = 64;   // one wavefront per matrix

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Sturm counts at xs[q] (scaled) for KQ chains per lane: SturmChain on the
// scaled d, e^2 in LDS; a wave with a chain whose minors came near underflow
// recounts all its chains with the guarded ratio recurrence.
template <int KQ>
__device__ __forceinline__ void sturm_counts_lanes(int n, const double* sd, const double* se, const double* xs,
                                                   int* cnt) {
    constexpr int U = 16;
    SturmChain ch[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) ch[q].start();
    int i = 0;
    for (; i + U <= n; i += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double di = sd[i + u], ei = se[i + u];
#pragma unroll
            for (int q = 0; q < KQ; ++q) ch[q].step(di - xs[q], ei);
        }
#pragma unroll
        for (int q = 0; q < KQ; ++q) ch[q].template close_block<U>();
    }
    for (; i < n; ++i) {
        const double di = sd[i], ei = se[i];
#pragma unroll
        for (int q = 0; q < KQ; ++q) ch[q].step_tail(di - xs[q], ei);
    }
    bool low = false;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        ch[q].finish();
        low |= ch[q].low;
        cnt[q] = ch[q].cnt;
    }
    if (__any(low)) {
        SturmRatio r[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) r[q].start();
        for (int j = 0; j < n; ++j) {
            const double di = sd[j], ei = se[j];
#pragma unroll
            for (int q = 0; q < KQ; ++q) r[q].step(di - xs[q], ei);
        }
#pragma unroll
        for (int q = 0; q < KQ; ++q)
            if (ch[q].low) cnt[q] = r[q].cnt;
    }
}

// KQ eigenvalue indices per lane (k = lane + 64 q), bisected in lockstep (KQ
// independent count recurrences per step).  First the counts at the M = 64 KQ
// points lo + (j + 1) (hi - lo) / (M + 1) (lane l, chain q: point l + 64 q),
// kept in LDS; each index starts from the cell whose end counts bracket it
// (a binary search), which holds its eigenvalue whatever rounding did to the
// counts, and bisects it for the halvings left.
template <int KQ>
__device__ __forceinline__ void bisect_lanes(int n, const double* sd, const double* se, double lo, double hi,
                                             double sc, int iters, double* w, int lane, int* gcnt) {
    constexpr int M = 64 * KQ;
    double a[KQ], c[KQ];
    bool live[KQ];
    const double gw = (hi - lo) / (double)(M + 1);
    if (iters > 0) {
        double xs[KQ];
        int cnt[KQ];
#pragma unroll
        for (int q = 0; q < KQ; ++q) xs[q] = (lo + (double)(lane + 64 * q + 1) * gw) * sc;
        sturm_counts_lanes<KQ>(n, sd, se, xs, cnt);
#pragma unroll
        for (int q = 0; q < KQ; ++q) gcnt[lane + 64 * q] = cnt[q];
    }
    team_sync<64>();
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        const int k = lane + 64 * q;
        a[q] = lo;
        c[q] = hi;
        live[q] = k < n;
        if (live[q] && iters > 0) {
            int jl = -1, jh = M;
            while (jh - jl > 1) {
                const int mid = (jl + jh) >> 1;
                if (gcnt[mid] > k) jh = mid;
                else jl = mid;
            }
            if (jl >= 0) a[q] = lo + (double)(jl + 1) * gw;
            if (jh < M) c[q] = lo + (double)(jh + 1) * gw;
        }
    }
    team_sync<64>();   // gcnt is rewritten by the next matrix
    // halvings left: (hi - lo) / ((M + 1) 2^r) below (hi - lo) / 2^iters
    const int rounds = iters > 0 ? (int)ceil((double)iters - log2((double)(M + 1))) : 0;
    for (int it = 0; it < rounds; ++it) {
        double x[KQ], xs[KQ];
        bool anyl = false;
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            x[q] = a[q] + 0.5 * (c[q] - a[q]);
            if (live[q] && (x[q] == a[q] || x[q] == c[q])) live[q] = false;
            anyl |= live[q];
            xs[q] = x[q] * sc;
        }
        if (!__any(anyl)) break;
        int cnt[KQ];
        sturm_counts_lanes<KQ>(n, sd, se, xs, cnt);
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            if (live[q]) {
                if (cnt[q] >= lane + 64 * q + 1) c[q] = x[q];
                else a[q] = x[q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q)
        if (lane + 64 * q < n) w[lane + 64 * q] = a[q] + 0.5 * (c[q] - a[q]);
}

__global__ __launch_bounds__(BB_NT) void batched_bisect_kernel(const BatchDesc* __restrict__ desc, int count,
                                                               int* ticket) {
    __shared__ double sd[sbr::BATCH_NMAX], se[sbr::BATCH_NMAX];
    __shared__ int gcnt[sbr::BATCH_NMAX];
    __shared__ int mat_sh;
    const int t = threadIdx.x;
    while (true) {
        if (t == 0) mat_sh = atomicAdd(ticket, 1);
        team_sync<64>();
        const int mi = mat_sh;
        team_sync<64>();
        if (mi >= count) break;
        const BatchDesc dm = desc[mi];
        const int n = dm.n;
        // d, e_{i-1} (from the last halving, or straight from A when n <= 2)
        double lo = DBL_MAX, hi = -DBL_MAX, emax2 = 1.0;
        for (int i = t; i < n; i += BB_NT) {
            double di, em, ep;
            if (dm.b0 >= 2) {
                di = dm.de[i];
                em = (i > 0) ? dm.de[n + i - 1] : 0.0;
                ep = (i + 1 < n) ? dm.de[n + i] : 0.0;
            } else {
                di = dm.A[i + (int64_t)i * dm.lda];
                em = (i > 0) ? dm.A[i + (int64_t)(i - 1) * dm.lda] : 0.0;
                ep = (i + 1 < n) ? dm.A[(i + 1) + (int64_t)i * dm.lda] : 0.0;
            }
            sd[i] = di;
            se[i] = em * em;
            const double rr = fabs(em) + fabs(ep);
            lo = fmin(lo, di - rr);
            hi = fmax(hi, di + rr);
            emax2 = fmax(emax2, em * em);
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        emax2 = wave_max(emax2);
        const double eps = DBL_EPSILON * 0.5;
        double tnorm = fmax(fabs(lo), fabs(hi));
        const double pivmin = DBL_MIN * emax2;
        const double widen = 2.1 * ((double)n * eps * tnorm + 2.0 * pivmin);
        const double l = lo - widen, h = hi + widen;
        tnorm = fmax(fabs(l), fabs(h));
        int iters = 0;
        if (h > l && tnorm > 0.0) {
            iters = (int)ceil(log2((h - l) / (eps * tnorm))) + 2;
            if (iters < 0) iters = 0;
        }
        // the Sturm data scaled so that the interval width is below one
        const double sc = (h > l) ? sturm_scale(h - l) : 1.0;
        team_sync<64>();
        for (int i = t; i < n; i += BB_NT) {
            sd[i] *= sc;
            se[i] *= sc * sc;
        }
        team_sync<64>();
        switch ((n + 63) / 64) {
            case 1: bisect_lanes<1>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
            case 2: bisect_lanes<2>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
            case 3: bisect_lanes<3>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
            case 4: bisect_lanes<4>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
            case 5: bisect_lanes<5>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
            case 6: bisect_lanes<6>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
            case 7: bisect_lanes<7>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
            default: bisect_lanes<8>(n, sd, se, l, h, sc, iters, dm.w, t, gcnt); break;
        }
        team_sync<64>();
    }
}

__global__ void batch_reset_kernel(int* tickets, int count) {
    if ((int)threadIdx.x < count) tickets[threadIdx.x] = 0;
}

}  // namespace

namespace sbr {

int64_t batch_scratch_doubles(int grid) { return (int64_t)grid * 2 * BF_MP * 16; }

int batch_f2b_grid() { return 512; }

void launch_batched(const BatchDesc* desc, int count, int max_b0, bool f32, int* tickets, double* scratch,
                    hipStream_t s) {
    if (count <= 0) return;
    batch_reset_kernel<<<1, 64, 0, s>>>(tickets, 8);
    const int gf = count < batch_f2b_grid() ? count : batch_f2b_grid();
    if (f32)
        batched_f2b_kernel<true><<<gf, BF_NT, BF_TOTAL * sizeof(double), s>>>(desc, count, tickets + 0, scratch);
    else
        batched_f2b_kernel<false><<<gf, BF_NT, BF_TOTAL * sizeof(double), s>>>(desc, count, tickets + 0, scratch);
    const int gb = count < 4096 ? count : 4096;
    // the last two halvings chase their band in LDS (20 and 37 KB at n = 512,
    // 8 and 4 matrices a CU); the bands of h = 4 and 8 (70 and 135 KB) would
    // leave 2 and 1 matrices a CU, which measured slower than chasing in the
    // global buffer with 16
    if (max_b0 >= 16) batched_band_kernel<8, false><<<gb, 64, 0, s>>>(desc, count, tickets + 1);
    if (max_b0 >= 8) batched_band_kernel<4, false><<<gb, 64, 0, s>>>(desc, count, tickets + 2);
    if (max_b0 >= 4)
        batched_band_kernel<2, true><<<gb, 64, batched_band_lds_doubles<2>() * sizeof(double), s>>>(desc, count,
                                                                                                  tickets + 3);
    if (max_b0 >= 2)
        batched_band_kernel<1, true><<<gb, 64, batched_band_lds_doubles<1>() * sizeof(double), s>>>(desc, count,
                                                                                                  tickets + 4);
    const int gs = count < 8192 ? count : 8192;
    batched_bisect_kernel<<<gs, BB_NT, 0, s>>>(desc, count, tickets + 5);
}

int init_batched_attributes() {
    hipError_t e = hipFuncSetAttribute((const void*)batched_f2b_kernel<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, BF_TOTAL * (int)sizeof(double));

    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)batched_f2b_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                BF_TOTAL * (int)sizeof(double));
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace sbr
