// sbr_band_tridiag.hip -- a symmetric band of width b (4, 8 or 16) reduced
// straight to tridiagonal form: Algorithm 4.2 with k = b, i.e. h = 1.
//
// Chase (i, j), i = 1 .. n-2, j = 1 .. J_i, has o = i + (j-1) b and works on
// rows [o, o + n_r), n_r = min(n - o, b).  Its "QR block" is a single column
// (column o - 1 for j = 1, o - b for j > 1), so the factorization is one
// Householder reflector H = I - tau v v^T with v_0 = 1; the block becomes
// [beta; 0].  With the reflector:
//   left block  X_L (rows [o, o+b), cols [o-b+1, o), j > 1): X_L <- H X_L
//   diagonal    D   (rows and cols [o, o+b)):                 D   <- H D H
//   below block X_B (rows [o+b, o+2b), cols [o, o+b)):        X_B <- X_B H
// which are the updates of Algorithm 4.2 with U = v, T = tau written for one
// reflector (H D H = D - v w^T - w v^T with p = tau D v,
// w = p - (tau/2)(v^T p) v).  The extents are those of the general-k model.
//
// Schedule (the sweep-group scheme of the small-b halvings, with h = 1): a
// work-group owns S consecutive sweeps and runs them in lock step, sweep s
// doing chase j = step - 2 s; a step is a QR phase (every active sweep forms
// its reflector and stores [beta; 0]) and an update phase, separated by a
// work-group barrier.  Consecutive sweeps two chases apart never write a
// common entry in the same phase, and a sweep's below block, which is the
// QR column and left block of its next chase, is touched by no other sweep in
// between (both checked by the schedule model), so it stays in registers.
//
// Lanes: a team of T lanes per sweep (T = 1 for b = 4), each holding b / T
// consecutive rows of the chase's blocks (the carried below block, the
// diagonal block as full symmetric rows, the new below block).  Column sums
// are team all-reduces and the QR column and w reach every lane of the team by
// DPP broadcasts.  The live
// band columns sit in an LDS ring (column c at slot c mod WC, its diagonals
// 0 .. 2b-1 contiguous: a chase reaches distance 2b - 1 at most), loaded from
// and written back to global memory in batches, with watermarks between
// consecutive groups as in the halving kernels.
#include "sbr_device.h"
#include "sbr_internal.h"

namespace {

// Launch shapes: lanes per sweep T (each holding R = B / T consecutive rows
// of the chase's blocks), sweeps per group S, steps per load / write-back
// batch.  Variant 0 is the default; the others are kept for tuning.
template <int B, int V> struct TriShape;
template <> struct TriShape<4, 0> { static constexpr int T = 4, S = 64, BATCH = 16; };
template <> struct TriShape<4, 1> { static constexpr int T = 2, S = 128, BATCH = 16; };
template <> struct TriShape<4, 2> { static constexpr int T = 1, S = 256, BATCH = 16; };
template <> struct TriShape<8, 0> { static constexpr int T = 8, S = 64, BATCH = 8; };
template <> struct TriShape<8, 1> { static constexpr int T = 4, S = 64, BATCH = 8; };
template <> struct TriShape<8, 2> { static constexpr int T = 2, S = 64, BATCH = 8; };
template <> struct TriShape<16, 0> { static constexpr int T = 16, S = 12, BATCH = 4; };
template <> struct TriShape<16, 1> { static constexpr int T = 8, S = 12, BATCH = 4; };
template <> struct TriShape<16, 2> { static constexpr int T = 16, S = 8, BATCH = 8; };
constexpr int TRI_VARIANTS = 3;

template <int B, int V>
struct TriCfg {
    static constexpr int T = TriShape<B, V>::T;
    static constexpr int S = TriShape<B, V>::S;
    static constexpr int BATCH = TriShape<B, V>::BATCH;
    static constexpr int R = B / T;
    static constexpr int NT = S * T;
    static constexpr int LAG = 2;                     // chases between consecutive sweeps
    // stored diagonals per ring column: 0 .. 2b - 1 are reached (a chase
    // reaches distance 2b - 1 at most); the odd stride spreads the windows of
    // the sweeps of a wavefront over the LDS banks
    static constexpr int LDW = 2 * B + 1;
    // ring columns: the active windows of the group span (LAG b - 1) per
    // sweep plus two chase windows, and one batch of columns loaded ahead
    static constexpr int WC = (LAG * B - 1) * S + B * (BATCH + 6);
    static constexpr int LDS_DOUBLES = WC * LDW;
    // prefetch registers: one batch of columns (b per step) spread over the block
    static constexpr int PFC = B * BATCH;
    static constexpr int PFN = (PFC * LDW + NT - 1) / NT;
    static_assert(64 % T == 0 && B % T == 0, "a team must sit inside one wavefront");
    static_assert(LDS_DOUBLES * 8 <= 160 * 1024, "ring must fit in LDS");
};

struct TriArgs {
    int64_t n;
    double* band;          // global band, ld = 2b + 1
    int ldg;               // 2b + 1
    int nsweeps;
    int ngroups;
    int* ticket;
    int* done;             // ngroups watermarks
    int* error;            // the plan's status word: nonzero stops every block
    uint64_t wait_ticks;
};

template <int B>
__device__ __forceinline__ int jcount(int n, int i) {
    return (n - 2 - i) / B + 1;
}

// Band element (o + r, o - B + x) of a chase window whose 2B columns occupy
// consecutive ring slots (FlatWin) or wrap around the ring's end (WrapWin);
// r - x + B is the element's diagonal, in [0, LDW).
template <int B, int LDW>
struct FlatWin {
    double* base;   // ring column of o - B
    __device__ __forceinline__ double& at(int r, int x) const { return base[x * LDW + (r - x + B)]; }
};
template <int B, int LDW, int WC>
struct WrapWin {
    double* ring;
    int sb;         // ring slot of column o - B
    __device__ __forceinline__ double& at(int r, int x) const {
        int sl = sb + x;
        sl -= (sl >= WC) ? WC : 0;
        return ring[sl * LDW + (r - x + B)];
    }
};

// What a chase's QR phase hands to its update phase (per lane: rows
// row0 .. row0 + R - 1 of the chase).
template <int B, int R>
struct StepRegs {
    double v[B];          // the reflector, v[0] = 1
    double dr[R][B];      // rows of the diagonal block
    double xb[R][B];      // rows of the below block
    double va[R];         // v at this lane's rows
    double tau;
};

// Lane SRC of each aligned team of T lanes (T in {2, 4, 8, 16}), in every
// lane of the team: quad_perm inside a quad; for 8 lanes the other quad's
// value comes over by row_half_mirror (lane i <-> 7 - i); row_newbcast for a
// 16-lane row.
template <int T, int SRC>
__device__ __forceinline__ double team_bcast(double v) {
    if constexpr (T == 2) {
        return dpp_d<SRC | (SRC << 2) | ((2 + SRC) << 4) | ((2 + SRC) << 6)>(v);
    } else if constexpr (T == 4) {
        return dpp_d<SRC | (SRC << 2) | (SRC << 4) | (SRC << 6)>(v);
    } else if constexpr (T == 8) {
        constexpr int Q = SRC & 3;
        const double a = dpp_d<Q | (Q << 2) | (Q << 4) | (Q << 6)>(v);
        const double b = dpp_d<0x141>(a);
        return (((threadIdx.x >> 2) & 1) == (SRC >> 2)) ? a : b;
    } else {
        static_assert(T == 16, "team size");
        return dpp_d<0x150 + SRC>(v);
    }
}

// Every lane of a team gets the B-vector whose entries u R .. u R + R - 1
// lane u of the team holds (R = B / T), by DPP broadcasts.
template <int B, int R>
__device__ __forceinline__ void team_gather(const double (&mine)[R], double (&all)[B]) {
    constexpr int T = B / R;
    if constexpr (T == 1) {
#pragma unroll
        for (int c = 0; c < B; ++c) all[c] = mine[c];
    } else {
        [&]<int... U>(std::integer_sequence<int, U...>) {
            (([&] {
#pragma unroll
                 for (int k = 0; k < R; ++k) all[U * R + k] = team_bcast<T, U>(mine[k]);
             }()),
             ...);
        }(std::make_integer_sequence<int, T>{});
    }
}

template <int T>
__device__ __forceinline__ double team_total(double v) {
    if constexpr (T == 1) return v;
    else return group_sum<T>(v);
}

// QR phase of one chase: the reflector of the QR column (column o - 1 for
// j = 1, the carried block's first column otherwise), [beta; 0] stored; the
// diagonal and below blocks loaded for the update phase (the concurrent QR
// phases of the other sweeps store only into their own QR columns, which meet
// this chase's blocks in one entry, the below block's last row and column,
// read after the barrier).  Every lane of the block runs it (act = false for
// the teams of inactive sweeps).  GUARD: a tail chase somewhere in the
// wavefront (rows or columns past the matrix end); otherwise every guard
// holds and is left out.
template <int B, int T, bool GUARD, class Win>
__device__ __forceinline__ void qr_phase(const Win& win, bool act, int j, int row0, int nr,
                                         const double (&cy)[B / T][B], StepRegs<B, B / T>& st) {
    constexpr int R = B / T;
    double x[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = row0 + k;
        const double xr = win.at(r, B - 1);
        x[k] = (j == 1) ? ((!GUARD || r < nr) ? xr : 0.0) : cy[k][0];
    }
    double xv[B];
    team_gather<B, R>(x, xv);
    double sq[B - 1];
#pragma unroll
    for (int c = 1; c < B; ++c) sq[c - 1] = xv[c] * xv[c];
    const double sig = tree_sum<B - 1>(sq);
    const double x0 = xv[0];
    double beta = x0, tau = 0.0, scal = 0.0;
    if (sig != 0.0) {
        // beta = -sgn(x0) ||x||, tau = 1 + |x0| / ||x||, v = x / (x0 - beta)
        // = sgn(x0) x / (|x0| + ||x||); Newton-refined estimates in range
        const double s2 = fma(x0, x0, sig);
        const double sg = (x0 >= 0.0) ? 1.0 : -1.0, ax = fabs(x0);
        if (s2 > 1e-290 && s2 < 1e290) {
            const double rs = sbr_rsqrt(s2);
            const double nrm = s2 * rs;
            beta = -sg * nrm;
            tau = fma(ax, rs, 1.0);
            scal = sg * sbr_recip(ax + nrm);
        } else {
            const double nrm = sqrt(s2);
            beta = -sg * nrm;
            tau = (beta - x0) / beta;
            scal = 1.0 / (x0 - beta);
        }
    }
    st.tau = tau;
    st.v[0] = 1.0;
#pragma unroll
    for (int c = 1; c < B; ++c) st.v[c] = xv[c] * scal;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = row0 + k;
        st.va[k] = (r == 0) ? 1.0 : x[k] * scal;
        if (act && (!GUARD || r < nr)) win.at(r, (j == 1) ? B - 1 : 0) = (r == 0) ? beta : 0.0;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = row0 + k;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            // diagonal block: element (o + max, o + min) of the lower storage
            const double dl = win.at(r, B + c);    // (o + r, o + c), c <= r
            const double du = win.at(c, B + r);    // (o + c, o + r), c > r
            const int lo = (r < c) ? r : c;
            const double dv = (c <= r) ? dl : du;
            st.dr[k][c] = (!GUARD || lo < nr) ? dv : 0.0;
            const double bv = win.at(B + r, B + c);   // (o + B + r, o + c)
            st.xb[k][c] = (!GUARD || c < nr) ? bv : 0.0;
        }
    }
}

// Update phase of one chase: left block (j > 1) H X_L, diagonal block H D H,
// below block X_B H (kept as the carry; stored at the sweep's last chase).
template <int B, int T, bool GUARD, class Win>
__device__ __forceinline__ void update_phase(const Win& win, bool act, int j, int J, int row0, int nr,
                                             int nbr, double (&cy)[B / T][B], StepRegs<B, B / T>& st) {
    constexpr int R = B / T;
    if (!act) return;
    const double tau = st.tau;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (row0 + k == B - 1 && (!GUARD || B - 1 < nr)) st.xb[k][B - 1] = win.at(2 * B - 1, 2 * B - 1);
    // left block (j > 1): rows o + r, columns o - B + c, c = 1 .. B-1
    if (j > 1) {
        double wl[B];
#pragma unroll
        for (int c = 1; c < B; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) acc = fma(st.va[k], cy[k][c], acc);
            wl[c] = team_total<T>(acc);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double tv = tau * st.va[k];
#pragma unroll
            for (int c = 1; c < B; ++c) win.at(row0 + k, c) = fma(-tv, wl[c], cy[k][c]);
        }
    }
    // diagonal block: p = tau D v, s = v^T p, w = p - (tau/2) s v,
    // D <- D - v w^T - w v^T (lower part stored)
    double p[R], sacc = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        double part[B];
#pragma unroll
        for (int c = 0; c < B; ++c) part[c] = st.dr[k][c] * st.v[c];
        p[k] = tau * tree_sum<B>(part);
        sacc = fma(p[k], st.va[k], sacc);
    }
    const double s = team_total<T>(sacc);
    double w[R];
#pragma unroll
    for (int k = 0; k < R; ++k) w[k] = fma(-0.5 * tau * s, st.va[k], p[k]);
    double wv[B];
    team_gather<B, R>(w, wv);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = row0 + k;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            const double nd = st.dr[k][c] - fma(st.va[k], wv[c], w[k] * st.v[c]);
            if (c <= r && (!GUARD || c < nr)) win.at(r, B + c) = nd;
        }
    }
    // below block: X_B <- X_B - tau (X_B v) v^T, carried into the next chase
#pragma unroll
    for (int k = 0; k < R; ++k) {
        double part[B];
#pragma unroll
        for (int c = 0; c < B; ++c) part[c] = st.xb[k][c] * st.v[c];
        const double q = tau * tree_sum<B>(part);
#pragma unroll
        for (int c = 0; c < B; ++c) cy[k][c] = fma(-q, st.v[c], st.xb[k][c]);
    }
    if (j == J) {
        // the sweep's last chase: its below block goes to the band
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c)
                if (row0 + k < nbr && c < nr) win.at(B + row0 + k, B + c) = cy[k][c];
    }
}

template <int B, int V>
__global__ __launch_bounds__((TriCfg<B, V>::NT)) void band_tridiag_kernel(TriArgs a) {
    typedef TriCfg<B, V> C;
    constexpr int S = C::S, WC = C::WC, LDW = C::LDW, LAG = C::LAG, T = C::T, R = C::R;
    extern __shared__ double ring[];
    __shared__ int g_sh, abort_sh, vis_sh;
    const int t = threadIdx.x;
    // sweep of the group: the teams of one wavefront take every NW-th sweep
    // (NW = wavefronts of the block), so their chase windows, NW (2b - 1)
    // ring columns apart, fall on different LDS banks
    constexpr int NW = C::NT / 64;
    const int tm = (C::NT % 64 == 0) ? ((t & 63) / T) * NW + (t >> 6) : t / T;
    const int row0 = (t % T) * R;         // first of this lane's rows of the chase
    const int n = (int)a.n;               // n (2b + 1) < 2^31 is checked on the host
    const int ldg = a.ldg;
    double* gband = a.band;

    while (true) {
        if (t == 0) {
            const bool failed = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            g_sh = failed ? a.ngroups : atomicAdd(a.ticket, 1);
            abort_sh = 0;
            vis_sh = 0;
        }
        __syncthreads();
        const int g = __builtin_amdgcn_readfirstlane(g_sh);
        __syncthreads();
        if (g >= a.ngroups) break;
        const int i0 = 1 + g * S;
        const int ns = (a.nsweeps - i0 + 1 < S) ? (a.nsweeps - i0 + 1) : S;
        // sweep s does its last chase at step f(s) = J(s) + LAG s, increasing in s
        auto Jof = [&](int s) -> int { return jcount<B>(n, i0 + s); };
        auto wstart = [&](int s, int j) -> int {
            const int o = i0 + s + (j - 1) * B;
            return (j == 1) ? o - 1 : o - B;
        };
        auto wend = [&](int s, int j) -> int {
            const int e = i0 + s + j * B;
            return e < n ? e : n;
        };
        const int tau_end = LAG * (ns - 1) + Jof(ns - 1);
        const int my_i = i0 + tm;
        const int my_J = (tm < ns) ? Jof(tm) : 0;
        double cy[R][B];               // this lane's rows of the last chase's below block
        int loaded = wstart(0, 1);     // ring holds columns [written, loaded)
        int written = loaded;
        int pub_pending = -1;          // watermark whose write-back is in flight
        int pf_lo = 0, pf_hi = 0;      // columns [pf_lo, pf_hi) prefetched into pf
        double pf[C::PFN];
        int s_lo = 0, f_lo = Jof(0);
        auto lowest_active = [&](int s0, int tau) {
            int sl = s0;
            while (sl < ns && Jof(sl) + LAG * sl < tau) ++sl;
            return sl;
        };
        auto need_through = [&](int sl, int tb) -> int {
            if (sl >= ns) return loaded;
            if (Jof(sl) + LAG * sl <= tb) return n;
            const int jj = tb - LAG * sl;
            return (jj >= 1) ? wend(sl, jj) : wend(sl, 1);
        };
        auto slot = [&](int c) { return c % WC; };
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c) cy[k][c] = 0.0;

        for (int tau_s = 1; tau_s <= tau_end; ++tau_s) {
            if (tau_s > f_lo && s_lo < ns) {
                s_lo = lowest_active(s_lo, tau_s);
                f_lo = (s_lo < ns) ? Jof(s_lo) + LAG * s_lo : tau_end;
            }
            // ---- columns needed within the next BATCH steps into the ring
            if (((tau_s - 1) % C::BATCH) == 0 && s_lo < ns) {
                const int need = need_through(s_lo, tau_s + C::BATCH - 1);
                if (pf_hi > pf_lo) {
                    const int cnt = (pf_hi - pf_lo) * LDW;
                    const int sl0 = slot(pf_lo);
#pragma unroll
                    for (int p = 0; p < C::PFN; ++p) {
                        const int idx = t + p * C::NT;
                        if (idx < cnt) {
                            const int k = idx / LDW, d = idx - k * LDW;
                            int sl = sl0 + k;
                            if (sl >= WC) sl -= WC;
                            ring[sl * LDW + d] = pf[p];
                        }
                    }
                    loaded = pf_hi;
                    pf_lo = pf_hi = 0;
                }
                if (need > loaded) {
                    if (g > 0) {
                        if (t == 0 && vis_sh < need) {
                            const uint64_t t0 = wall_clock64();
                            int d;
                            while ((d = __hip_atomic_load(&a.done[g - 1], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)) < need) {
                                __builtin_amdgcn_s_sleep(1);
                                if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                                    abort_sh = 1;
                                    break;
                                }
                                if (wall_clock64() - t0 > a.wait_ticks) {
                                    atomicOr(a.error, sbr::STATUS_STALLED);
                                    abort_sh = 1;
                                    break;
                                }
                            }
                            vis_sh = d;
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        }
                        __syncthreads();
                        if (abort_sh) return;
                    }
                    const int cnt = (need - loaded) * LDW;
                    const int sl0 = slot(loaded);
                    for (int idx = t; idx < cnt; idx += C::NT) {
                        const int k = idx / LDW, d = idx - k * LDW;
                        int sl = sl0 + k;
                        if (sl >= WC) sl -= WC;
                        ring[sl * LDW + d] = (loaded + k + d < n) ? gband[(int64_t)(loaded + k) * ldg + d] : 0.0;
                    }
                    loaded = need;
                }
                // prefetch the next batch's columns, as far as they are released
                {
                    const int sl2 = lowest_active(s_lo, tau_s + C::BATCH);
                    int want = need_through(sl2, tau_s + 2 * C::BATCH - 1);
                    if (want > loaded + C::PFC) want = loaded + C::PFC;
                    if (want > loaded && g > 0) {
                        if (t == 0 && vis_sh < want) {
                            const int d = __hip_atomic_load(&a.done[g - 1], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                            if (d > vis_sh) {
                                vis_sh = d;
                                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                            }
                        }
                        __syncthreads();
                        if (want > vis_sh) want = vis_sh;
                    }
                    if (want > loaded) {
                        const int cnt = (want - loaded) * LDW;
#pragma unroll
                        for (int p = 0; p < C::PFN; ++p) {
                            const int idx = t + p * C::NT;
                            if (idx < cnt) {
                                const int k = idx / LDW, d = idx - k * LDW;
                                pf[p] = (loaded + k + d < n) ? gband[(int64_t)(loaded + k) * ldg + d] : 0.0;
                            }
                        }
                        pf_lo = loaded;
                        pf_hi = want;
                    }
                }
                __syncthreads();
            }

            // ---- this step's chase of my sweep
            const int jl = tau_s - LAG * tm;
            const bool act = (tm < ns) && (jl >= 1) && (jl <= my_J);
            const int j = act ? jl : 1;
            const int o = my_i + (j - 1) * B;
            const int nr = (n - o < B) ? n - o : B;
            const int nbl = n - (o + B);
            const int nbr = nbl > B ? B : (nbl > 0 ? nbl : 0);
            // the chase's columns o - B .. o + B - 1 start at ring slot sb; when
            // they do not wrap around the ring's end, every element is at a
            // compile-time offset from one of two per-lane addresses
            int sb = slot(o) - B;
            sb += (sb < 0) ? WC : 0;
            const bool wraps = act && (sb + 2 * B > WC);
            const bool tail = act && (o + 2 * B > n);
            const bool fast = __ballot(wraps || tail) == 0;     // uniform per wavefront
            const FlatWin<B, LDW> fw{ring + sb * LDW};
            const WrapWin<B, LDW, WC> ww{ring, sb};
            StepRegs<B, R> st;
            if (fast) qr_phase<B, T, false>(fw, act, j, row0, nr, cy, st);
            else qr_phase<B, T, true>(ww, act, j, row0, nr, cy, st);
            __syncthreads();   // the update phase reads entries other QR phases stored
            if (fast) update_phase<B, T, false>(fw, act, j, my_J, row0, nr, nbr, cy, st);
            else update_phase<B, T, true>(ww, act, j, my_J, row0, nr, nbr, cy, st);
            __syncthreads();   // the next step reads what the neighbouring sweeps wrote

            // ---- write back columns no sweep of the group touches again
            const bool last = (tau_s == tau_end);
            if (last || (tau_s % C::BATCH) == 0) {
                int done = last ? loaded : n;
                if (!last) {
                    const int tn = tau_s + 1;
                    int s_hi = (tn - 1) / LAG;
                    if (s_hi > ns - 1) s_hi = ns - 1;
                    if (s_hi >= 0 && Jof(s_hi) + LAG * s_hi >= tn) {
                        const int st = wstart(s_hi, tn - LAG * s_hi);
                        done = st < done ? st : done;
                    }
                    if (s_hi + 1 < ns) {
                        const int st = wstart(s_hi + 1, 1);
                        done = st < done ? st : done;
                    }
                }
                if (done > loaded) done = loaded;
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (t == 0 && pub_pending >= 0 && !last) sbr_store_release(&a.done[g], pub_pending);
                if (done > written) {
                    const int cnt = (done - written) * LDW;
                    const int sl0 = slot(written);
                    for (int idx = t; idx < cnt; idx += C::NT) {
                        const int k = idx / LDW, d = idx - k * LDW;
                        int sl = sl0 + k;
                        if (sl >= WC) sl -= WC;
                        gband[(int64_t)(written + k) * ldg + d] = ring[sl * LDW + d];
                    }
                    written = done;
                    pub_pending = written;
                }
                if (last) {
                    __builtin_amdgcn_s_waitcnt(0);
                    __syncthreads();
                    if (t == 0) {
                        if (g > 0) {
                            const uint64_t t0 = wall_clock64();
                            while (__hip_atomic_load(&a.done[g - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n) {
                                __builtin_amdgcn_s_sleep(1);
                                if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                                if (wall_clock64() - t0 > a.wait_ticks) {
                                    atomicOr(a.error, sbr::STATUS_STALLED);
                                    break;
                                }
                            }
                        }
                        sbr_store_release(&a.done[g], n);
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int B, int V>
void launch_tri(int64_t n, double* band, const sbr::StageCtl& ctl, hipStream_t s) {
    typedef TriCfg<B, V> C;
    const int64_t nsweeps = n - 2;
    if (nsweeps < 1) return;
    const int64_t ngroups = (nsweeps + C::S - 1) / C::S;
    TriArgs a;
    a.n = n;
    a.band = band;
    a.ldg = 2 * B + 1;
    a.nsweeps = (int)nsweeps;
    a.ngroups = (int)ngroups;
    a.ticket = ctl.flags;
    a.done = ctl.flags + 1;
    a.error = ctl.status;
    a.wait_ticks = ctl.wait_ticks;
    sbr::launch_fill_int(ctl.flags, ngroups + 1, 0, s);
    int64_t grid = ngroups < 1024 ? ngroups : 1024;
    if (ctl.max_grid > 0 && grid > ctl.max_grid) grid = ctl.max_grid;
    band_tridiag_kernel<B, V><<<(unsigned)grid, C::NT, (size_t)C::LDS_DOUBLES * sizeof(double), s>>>(a);
}

template <int B>
void launch_tri_variant(int64_t n, double* band, const sbr::StageCtl& ctl, hipStream_t s) {
    switch (ctl.tri_variant) {
        case 1: launch_tri<B, 1>(n, band, ctl, s); break;
        case 2: launch_tri<B, 2>(n, band, ctl, s); break;
        default: launch_tri<B, 0>(n, band, ctl, s); break;
    }
}

template <int B, int V>
int set_tri_attr() {
    const int bytes = TriCfg<B, V>::LDS_DOUBLES * (int)sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)band_tridiag_kernel<B, V>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e == hipSuccess ? 0 : (int)e;
}

template <int B>
int set_tri_attrs() {
    return set_tri_attr<B, 0>() | set_tri_attr<B, 1>() | set_tri_attr<B, 2>();
}

}  // namespace

namespace sbr {

bool band_tridiag_supported(int b) { return b == 4 || b == 8 || b == 16; }

int band_tridiag_variants() { return TRI_VARIANTS; }

void launch_band_tridiag(int64_t n, double* band, int b, const StageCtl& ctl, hipStream_t s) {
    switch (b) {
        case 4: launch_tri_variant<4>(n, band, ctl, s); break;
        case 8: launch_tri_variant<8>(n, band, ctl, s); break;
        case 16: launch_tri_variant<16>(n, band, ctl, s); break;
        default: break;
    }
}

int init_band_tridiag_attributes() { return set_tri_attrs<4>() | set_tri_attrs<8>() | set_tri_attrs<16>(); }

}  // namespace sbr
