// sbr_band_group.hip -- band halving b -> h = b/2 (Algorithm 4.2, k = 2) for
// small bandwidths, with the active part of the band held in LDS.
//
// The chase mathematics is the one of sbr_band.hip (same offsets, extents and
// Eq. (4.1)-form update); what differs is the schedule.  A work-group owns a
// group of S consecutive sweeps i0 .. i0+S-1 and runs them as a pipeline of
// its own: at step tau sweep i0+s performs chase j = tau - 3s.  Chases that
// run in the same step are three chases apart in consecutive sweeps, so they
// write disjoint band columns (chase (i, j) writes columns [o-2h, o+2h),
// o = ih + (j-1)b, or [o-h, o+2h) for j = 1) and steps need only a work-group
// barrier.  One team of TEAM threads performs each chase.
//
// The group's live columns sit in an LDS ring buffer (column c at slot
// c mod WC, the 4h+1 stored diagonals contiguous, the same layout as the
// global band).  Columns are loaded from global memory in batches ahead of
// the leading sweep and written back once every sweep of the group is past
// them; the group then publishes a watermark done[g]: every column below it is
// final as far as sweeps <= i0+S-1 are concerned.  Group g+1 loads a column
// only below done[g]; this is the lag-3 rule between the last sweep of one
// group and the first sweep of the next, enforced at batch granularity (one
// agent-scope acquire per batch, not per chase).  Groups are taken from a
// ticket counter in order, so the group a block waits on is always running.
#include "sbr_device.h"
#include "sbr_internal.h"

namespace {

template <int H>
struct GroupCfg {
    // sweeps per group and threads per chase, sized so the ring plus the
    // per-team scratch stay near 110 KB of LDS
    static constexpr int S = (H == 1) ? 384 : (H == 2) ? 96 : (H == 4) ? 24 : 6;
    static constexpr int TEAM = (H == 1) ? 1 : (H == 2) ? 4 : (H == 4) ? 16 : 64;
    static constexpr int NT = S * TEAM;
    static constexpr int LDW = 4 * H + 1;        // stored diagonals per column
    static constexpr int BATCH = (H >= 8) ? 4 : 8;   // steps per load / write-back batch
    static constexpr int WC = 5 * H * S + 2 * H * (BATCH + 6);
    static constexpr int H2 = 2 * H;
    // per-team scratch (doubles)
    static constexpr int UB = 0;                 // 2H x H  QR block -> U
    static constexpr int TT = UB + H2 * H;       // H x H
    static constexpr int YY = TT + H * H;        // 2H x H  U T
    static constexpr int WR = YY + H2 * H;       // 2H x H  W / V of the qr rows
    static constexpr int GG = WR + H2 * H;       // H x H
    static constexpr int MM = GG + H * H;        // H x H
    static constexpr int WX = MM + H * H;        // 2H x H  W of the left / below block
    static constexpr int TAU = WX + H2 * H;      // H
    static constexpr int SCR = TAU + H;
    static constexpr int LDS_DOUBLES = WC * LDW + S * SCR;
};

struct GroupArgs {
    int64_t n;
    double* band;      // global band, ld = 4h + 1
    int nsweeps;
    int ngroups;
    int* ticket;
    int* done;         // ngroups watermarks
    int* error;
};

constexpr uint64_t GROUP_WAIT_LIMIT = 1000000000ull;   // 10 s of the 100 MHz clock

// A chase's team lies inside one wavefront (TEAM divides 64), whose lanes run
// in lock step and whose LDS accesses complete in program order, so inside a
// chase a compiler-level wavefront fence is all the synchronisation needed.
template <int TEAM>
__device__ __forceinline__ void team_sync() {
    static_assert(TEAM <= 64 && (64 % TEAM) == 0, "a team must sit inside one wavefront");
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int H>
__device__ __forceinline__ int64_t nchase_of(int64_t n, int64_t i) {
    return (n - 2 - i * H) / (2 * H) + 1;
}

template <int H>
__global__ __launch_bounds__(GroupCfg<H>::NT) void band_group_kernel(GroupArgs a) {
    typedef GroupCfg<H> C;
    constexpr int H2 = C::H2, TEAM = C::TEAM, S = C::S, WC = C::WC, LDW = C::LDW;
    extern __shared__ double smem[];
    double* ring = smem;
    __shared__ int g_sh, abort_sh, fresh_sh;
    __shared__ int64_t vis_sh;
    const int t = threadIdx.x;
    const int tm = t / TEAM, u = t % TEAM;
    double* scr = smem + WC * LDW + tm * C::SCR;
    double* Ub = scr + C::UB;
    double* Tm = scr + C::TT;
    double* Yb = scr + C::YY;
    double* Wr = scr + C::WR;
    double* Gm = scr + C::GG;
    double* Mm = scr + C::MM;
    double* Wx = scr + C::WX;
    double* tau = scr + C::TAU;
    const int64_t n = a.n;
    double* gband = a.band;

    // ring slot of column c for the current chase: window columns are
    // [cs, cs + 4h) and slot(cs) = sbase, so one compare wraps the index
    int cs = 0, sbase = 0;
    auto R = [&](int r, int c) -> double& {
        int sl = sbase + (c - cs);
        if (sl >= WC) sl -= WC;
        return ring[sl * LDW + (r - c)];
    };

    while (true) {
        if (t == 0) {
            const bool failed = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            g_sh = failed ? a.ngroups : atomicAdd(a.ticket, 1);
            abort_sh = 0;
            vis_sh = 0;
        }
        __syncthreads();
        const int g = g_sh;
        __syncthreads();
        if (g >= a.ngroups) break;
        const int64_t i0 = 1 + (int64_t)g * S;
        const int ns = (int)((a.nsweeps - i0 + 1 < S) ? (a.nsweeps - i0 + 1) : S);
        // Sweeps finish in order: sweep s does its last chase at step
        // f(s) = J_s + 3s, which increases with s.  At step tau the active
        // sweeps are s_lo(tau) .. s_hi(tau) with s_lo the first s with
        // f(s) >= tau and s_hi = min(ns-1, (tau-1)/3); window ends decrease
        // and window starts decrease with s, so the extremes are at s_lo
        // (end) and s_hi (start).
        auto Jof = [&](int s) -> int64_t { return nchase_of<H>(n, i0 + s); };
        auto wstart = [&](int s, int64_t j) -> int64_t {
            const int64_t o = (i0 + s) * H + (j - 1) * H2;
            return (j == 1) ? o - H : o - H2;
        };
        auto wend = [&](int s, int64_t j) -> int64_t {
            const int64_t e = (i0 + s) * H + j * H2;
            return e < n ? e : n;
        };
        const int64_t tau_end = 3 * (ns - 1) + Jof(ns - 1) > Jof(0) ? 3 * (ns - 1) + Jof(ns - 1) : Jof(0);
        // my sweep
        const int64_t my_i = i0 + tm;
        const int64_t my_J = (tm < ns) ? Jof(tm) : 0;
        int64_t loaded = wstart(0, 1);   // columns [written, loaded) are in the ring
        int64_t written = loaded;
        int s_lo = 0;

        for (int64_t tau_s = 1; tau_s <= tau_end; ++tau_s) {
            while (s_lo < ns && Jof(s_lo) + 3 * s_lo < tau_s) ++s_lo;
            // ---- columns needed within the next BATCH steps
            if (((tau_s - 1) % C::BATCH) == 0 && s_lo < ns) {
                const int64_t tb = tau_s + C::BATCH - 1;
                int64_t need;
                if (Jof(s_lo) + 3 * s_lo <= tb) {
                    need = n;                                   // a sweep ends inside the batch
                } else {
                    int64_t jj = tb - 3 * s_lo;
                    need = (jj >= 1) ? wend(s_lo, jj) : wend(s_lo, 1);
                }
                if (need > loaded) {
                    // wait until the previous group has released the columns
                    if (g > 0) {
                        if (t == 0) {
                            fresh_sh = 0;
                            if (vis_sh < need) {
                                const uint64_t t0 = wall_clock64();
                                int d;
                                while ((d = __hip_atomic_load(&a.done[g - 1], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT)) < need) {
                                    __builtin_amdgcn_s_sleep(2);
                                    if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                                        abort_sh = 1;
                                        break;
                                    }
                                    if (wall_clock64() - t0 > GROUP_WAIT_LIMIT) {
                                        atomicExch(a.error, 2 * H);
                                        abort_sh = 1;
                                        break;
                                    }
                                }
                                vis_sh = d;
                                fresh_sh = 1;
                            }
                        }
                        __syncthreads();
                        if (abort_sh) return;
                        if (fresh_sh) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                    // load [loaded, need) into the ring
                    const int cnt = (int)(need - loaded) * LDW;
                    const int sl0 = (int)(loaded % WC);
                    for (int idx = t; idx < cnt; idx += C::NT) {
                        const int k = idx / LDW, d = idx - k * LDW;
                        int sl = sl0 + k;
                        if (sl >= WC) sl -= WC;
                        ring[sl * LDW + d] = gband[(loaded + k) * (int64_t)LDW + d];
                    }
                    loaded = need;
                    __syncthreads();
                }
            }

            // ---- the chases of this step, one per team
            const int64_t jl = tau_s - 3 * tm;
            const bool act = (tm < ns) && (jl >= 1) && (jl <= my_J);
            const int j = act ? (int)jl : 0;
            const int o = act ? (int)(my_i * H + (int64_t)(j - 1) * H2) : 0;
            const int nr = act ? ((n - o < H2) ? (int)(n - o) : H2) : 0;
            const int cq = (j == 1) ? o - H : o - H2;
            int nbl = (int)(n - (o + H2));
            if (nbl > H2) nbl = H2;
            const int nbr = (act && nbl > 0) ? nbl : 0;
            cs = cq;
            sbase = act ? cs % WC : 0;

            // QR block into Ub
            if (act)
                for (int idx = u; idx < H2 * H; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    Ub[idx] = (r < nr) ? R(o + r, cq + c) : 0.0;
                }
            team_sync<TEAM>();
            for (int k = 0; k < H; ++k) {
                if (act && u == 0) {
                    double ss = 0.0;
                    for (int r = k + 1; r < H2; ++r) ss += Ub[r + k * H2] * Ub[r + k * H2];
                    const double xk = Ub[k + k * H2];
                    double beta, tk, scal;
                    if (ss == 0.0) {
                        beta = xk; tk = 0.0; scal = 0.0;
                    } else {
                        const double nrm = sqrt(xk * xk + ss);
                        beta = (xk >= 0.0) ? -nrm : nrm;
                        tk = (beta - xk) / beta;
                        scal = 1.0 / (xk - beta);
                    }
                    Ub[k + k * H2] = beta;
                    for (int r = k + 1; r < H2; ++r) Ub[r + k * H2] *= scal;
                    tau[k] = tk;
                }
                team_sync<TEAM>();
                if (act) {
                    const double tk = tau[k];
                    if (tk != 0.0)
                        for (int c = k + 1 + u; c < H; c += TEAM) {
                            double dot = Ub[k + c * H2];
                            for (int r = k + 1; r < H2; ++r) dot += Ub[r + k * H2] * Ub[r + c * H2];
                            const double f = tk * dot;
                            Ub[k + c * H2] -= f;
                            for (int r = k + 1; r < H2; ++r) Ub[r + c * H2] -= f * Ub[r + k * H2];
                        }
                }
                team_sync<TEAM>();
            }
            // R into the ring ([R; 0]), Ub becomes the explicit unit lower U
            if (act)
                for (int idx = u; idx < H2 * H; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    const double val = Ub[idx];
                    const bool refl = tau[c] != 0.0;
                    if (r < nr) R(o + r, cq + c) = (r <= c) ? val : 0.0;
                    Ub[idx] = (r < c) ? 0.0 : ((r == c) ? (refl ? 1.0 : 0.0) : (refl ? val : 0.0));
                }
            team_sync<TEAM>();
            // T: T[c][c] = tau_c, T[0:c, c] = -tau_c T[0:c, 0:c] (U^T U)[0:c, c]
            if (act)
                for (int idx = u; idx < H * H; idx += TEAM) {
                    const int ra = idx % H, c = idx / H;
                    double acc = 0.0;
                    if (ra < c)
                        for (int r = 0; r < H2; ++r) acc += Ub[r + ra * H2] * Ub[r + c * H2];
                    Gm[idx] = acc;
                    Tm[idx] = 0.0;
                }
            team_sync<TEAM>();
            for (int c = 0; c < H; ++c) {
                if (act)
                    for (int ra = u; ra <= c; ra += TEAM) {
                        if (ra == c) {
                            Tm[c + c * H] = tau[c];
                        } else {
                            double acc = 0.0;
                            for (int k = ra; k < c; ++k) acc += Tm[ra + k * H] * Gm[k + c * H];
                            Tm[ra + c * H] = -tau[c] * acc;
                        }
                    }
                team_sync<TEAM>();
            }
            // Y = U T ; W_R = D Y (D the symmetric diagonal block)
            if (act)
                for (int idx = u; idx < H2 * H; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    double acc = 0.0;
                    for (int k = 0; k <= c; ++k) acc += Ub[r + k * H2] * Tm[k + c * H];
                    Yb[idx] = acc;
                }
            team_sync<TEAM>();
            if (act)
                for (int idx = u; idx < H2 * H; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    double acc = 0.0;
                    if (r < nr)
                        for (int k = 0; k < nr; ++k) {
                            const double dv = (r >= k) ? R(o + r, o + k) : R(o + k, o + r);
                            acc += dv * Yb[k + c * H2];
                        }
                    Wr[idx] = acc;
                }
            team_sync<TEAM>();
            // G = U^T W_R ; M = T^T G ; V_R = 1/2 U M - W_R
            if (act)
                for (int idx = u; idx < H * H; idx += TEAM) {
                    const int ra = idx % H, c = idx / H;
                    double acc = 0.0;
                    for (int r = 0; r < H2; ++r) acc += Ub[r + ra * H2] * Wr[r + c * H2];
                    Gm[idx] = acc;
                }
            team_sync<TEAM>();
            if (act)
                for (int idx = u; idx < H * H; idx += TEAM) {
                    const int ra = idx % H, c = idx / H;
                    double acc = 0.0;
                    for (int k = 0; k <= ra; ++k) acc += Tm[k + ra * H] * Gm[k + c * H];
                    Mm[idx] = acc;
                }
            team_sync<TEAM>();
            if (act)
                for (int idx = u; idx < H2 * H; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    double acc = 0.0;
                    for (int k = 0; k < H; ++k) acc += Ub[r + k * H2] * Mm[k + c * H];
                    Wr[idx] = 0.5 * acc - Wr[idx];
                }
            team_sync<TEAM>();
            // diagonal block += U V_R^T + V_R U^T (lower part)
            if (act)
                for (int idx = u; idx < H2 * H2; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    if (r >= c && r < nr) {
                        double acc = 0.0;
                        for (int k = 0; k < H; ++k)
                            acc += Ub[r + k * H2] * Wr[c + k * H2] + Wr[r + k * H2] * Ub[c + k * H2];
                        R(o + r, o + c) += acc;
                    }
                }
            // left block (j > 1): X -= U (X^T Y)^T
            const bool left = act && (j > 1);
            if (left)
                for (int idx = u; idx < H * H; idx += TEAM) {
                    const int c = idx % H, k = idx / H;
                    double acc = 0.0;
                    for (int r = 0; r < nr; ++r) acc += R(o + r, o - H + c) * Yb[r + k * H2];
                    Wx[c + k * H] = acc;
                }
            team_sync<TEAM>();
            if (left)
                for (int idx = u; idx < H2 * H; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    if (r < nr) {
                        double acc = 0.0;
                        for (int k = 0; k < H; ++k) acc += Ub[r + k * H2] * Wx[c + k * H];
                        R(o + r, o - H + c) -= acc;
                    }
                }
            team_sync<TEAM>();
            // below block: X -= (X Y) U^T
            if (act && nbr > 0)
                for (int idx = u; idx < H2 * H; idx += TEAM) {
                    const int r = idx % H2, k = idx / H2;
                    double acc = 0.0;
                    if (r < nbr)
                        for (int c = 0; c < H2; ++c) acc += R(o + H2 + r, o + c) * Yb[c + k * H2];
                    Wx[idx] = acc;
                }
            team_sync<TEAM>();
            if (act && nbr > 0)
                for (int idx = u; idx < H2 * H2; idx += TEAM) {
                    const int r = idx % H2, c = idx / H2;
                    if (r < nbr) {
                        double acc = 0.0;
                        for (int k = 0; k < H; ++k) acc += Wx[r + k * H2] * Ub[c + k * H2];
                        R(o + H2 + r, o + c) -= acc;
                    }
                }
            team_sync<TEAM>();
            __syncthreads();   // next step reads columns the neighbouring sweeps wrote

            // ---- write back columns no sweep of the group will touch again
            const bool last = (tau_s == tau_end);
            if (last || (tau_s % C::BATCH) == 0) {
                int64_t done = last ? loaded : n;
                if (!last) {
                    // next step's active range: the smallest window start is at
                    // the highest started sweep; the next sweep to start (if
                    // any) begins at its first window
                    const int64_t tn = tau_s + 1;
                    int s_hi = (int)((tn - 1) / 3);
                    if (s_hi > ns - 1) s_hi = ns - 1;
                    if (s_hi >= 0 && Jof(s_hi) + 3 * s_hi >= tn) {
                        const int64_t st = wstart(s_hi, tn - 3 * s_hi);
                        done = st < done ? st : done;
                    }
                    if (s_hi + 1 < ns) {
                        const int64_t st = wstart(s_hi + 1, 1);
                        done = st < done ? st : done;
                    }
                }
                if (done > loaded) done = loaded;
                const bool moved = done > written;
                if (moved) {
                    const int cnt = (int)(done - written) * LDW;
                    const int sl0 = (int)(written % WC);
                    for (int idx = t; idx < cnt; idx += C::NT) {
                        const int k = idx / LDW, d = idx - k * LDW;
                        int sl = sl0 + k;
                        if (sl >= WC) sl -= WC;
                        gband[(written + k) * (int64_t)LDW + d] = ring[sl * LDW + d];
                    }
                    written = done;
                }
                if (moved || last) __threadfence();
                __syncthreads();
                if (t == 0 && (moved || last)) {
                    int pub = (int)written;
                    if (last) {
                        // everything this group loaded is back; columns it never
                        // loaded are final once the previous group is complete
                        if (g > 0) {
                            const uint64_t t0 = wall_clock64();
                            while (__hip_atomic_load(&a.done[g - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                                   (int)n) {
                                __builtin_amdgcn_s_sleep(2);
                                if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                                if (wall_clock64() - t0 > GROUP_WAIT_LIMIT) {
                                    atomicExch(a.error, 2 * H);
                                    break;
                                }
                            }
                        }
                        pub = (int)n;
                    }
                    sbr_store_release(&a.done[g], pub);
                }
            }
        }
        __syncthreads();
    }
}

template <int H>
void launch_group(int64_t n, double* band, int* flags, int* error, int max_grid, hipStream_t s) {
    typedef GroupCfg<H> C;
    const int64_t nsweeps = (n - 2) / H;
    if (nsweeps < 1) return;
    const int64_t ngroups = (nsweeps + C::S - 1) / C::S;
    GroupArgs a;
    a.n = n;
    a.band = band;
    a.nsweeps = (int)nsweeps;
    a.ngroups = (int)ngroups;
    a.ticket = flags;
    a.done = flags + 1;
    a.error = error;
    sbr::launch_fill_int(flags, ngroups + 1, 0, s);
    int64_t grid = ngroups < 256 ? ngroups : 256;
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    const size_t shm = (size_t)C::LDS_DOUBLES * sizeof(double);
    band_group_kernel<H><<<(unsigned)grid, C::NT, shm, s>>>(a);
}

template <int H>
int set_group_attr() {
    const int bytes = GroupCfg<H>::LDS_DOUBLES * (int)sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)band_group_kernel<H>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       bytes);
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace

namespace sbr {

bool band_group_supported(int b) { return b == 2 || b == 4 || b == 8 || b == 16; }

void launch_band_halve_group(int64_t n, double* band, int64_t ldband, int b, int* flags, int* error, int max_grid,
                             hipStream_t s) {
    (void)ldband;   // must equal 2b + 1 (checked by the caller)
    switch (b) {
        case 2: launch_group<1>(n, band, flags, error, max_grid, s); break;
        case 4: launch_group<2>(n, band, flags, error, max_grid, s); break;
        case 8: launch_group<4>(n, band, flags, error, max_grid, s); break;
        case 16: launch_group<8>(n, band, flags, error, max_grid, s); break;
        default: break;
    }
}

int init_band_group_attributes() {
    int rc = 0;
    rc |= set_group_attr<1>();
    rc |= set_group_attr<2>();
    rc |= set_group_attr<4>();
    rc |= set_group_attr<8>();
    return rc;
}

}  // namespace sbr
