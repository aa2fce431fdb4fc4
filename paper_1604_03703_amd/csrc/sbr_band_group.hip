// sbr_band_group.hip -- band halving b -> h = b/2 (Algorithm 4.2, k = 2) for
// small bandwidths, with the active part of the band held in LDS.
//
// The chase mathematics is the one of sbr_band.hip (same offsets, extents and
// Eq. (4.1)-form update); what differs is the schedule.  A work-group owns a
// group of S consecutive sweeps i0 .. i0+S-1 and runs them as a pipeline of
// its own: at step tau sweep i0+s performs chase j = tau - LAG s.  For h <= 4
// a chase is split in a QR phase and an update phase with a barrier between
// them, and LAG = 2: chases of one step are two chases apart in consecutive
// sweeps; the only entries two of them share are in the QR block of the
// upper sweep's chase, which its QR phase finishes before the lower sweep's
// update phase reads them.  For h = 8 (team_chase, one phase) LAG = 3: chases
// of one step write disjoint band columns (chase (i, j) writes columns
// [o-2h, o+2h), o = ih + (j-1)b, or [o-h, o+2h) for j = 1).
//
// The group's live columns sit in an LDS ring buffer (column c at slot
// c mod WC, the 4h+1 stored diagonals contiguous, the same layout as the
// global band).  Columns are loaded from global memory in batches ahead of
// the leading sweep and written back once every sweep of the group is past
// them; the group then publishes a watermark done[g]: every column below it is
// final as far as sweeps <= i0+S-1 are concerned.  Group g+1 loads a column
// only below done[g], which keeps the first sweep of one group behind the
// last sweep of the previous one, at batch granularity (one agent-scope
// acquire per batch, not per chase).  Groups are taken from a
// ticket counter in order, so the group a block waits on is always running.
#include "sbr_device.h"
#include "sbr_internal.h"
#include "sbr_team_chase.h"



namespace {

template <int H>
struct GroupCfg {
    // h = 1: one lane per sweep (lane_chase_qr / _update), one wave per
    // group, so a step's barriers are cheap.  h = 2: four lanes per sweep,
    // one band row each (team_lane_chase_qr / _update), 64 sweeps on four
    // waves; h = 4: four lanes per sweep, two rows each, 32 sweeps on two
    // waves (a row per lane there, eight lanes with ds_bpermute gathers,
    // measured 10 % slower).  All carry the bulge in registers.  h = 8 (used
    // only where the MFMA chase is not): one team of 2h lanes per chase
    // (team_chase, lane u holds band row u).  Sweeps per group are sized so
    // the ring (plus team_chase's scratch) stays in LDS.
    static constexpr bool LANE = (H <= 4);
    static constexpr int TEAM = (H == 1) ? 1 : (H == 2 ? 4 : (H == 4 ? 4 : 2 * H));
    static constexpr int NT = (H == 1) ? 64 : (H == 2 ? 256 : 128);
    static constexpr int S = NT / TEAM;
    static constexpr int LDW = 4 * H + 1;        // stored diagonals per column
    // steps per load / write-back batch
    static constexpr int BATCH = (H <= 2) ? 16 : (H == 4 ? 8 : 4);
    // steps between consecutive sweeps of the group: two with the two-phase
    // lane chases (a QR phase and an update phase per step), three with
    // team_chase, which does a whole chase between two barriers
    static constexpr int LAG = LANE ? 2 : 3;
    // ring columns: the active windows span (2 LAG - 1) h per sweep, plus
    // the columns loaded for one batch of steps ahead
    static constexpr int WC = (2 * LAG - 1) * H * S + 2 * H * (BATCH + 6);
    static constexpr int H2 = 2 * H;
    // per-team scratch (doubles): U rows (2h x h), a second 2h x h block
    // (the left block, then W, then V) and an h x h product
    // per-team scratch: the team_lane_chase gather buffers (16-lane teams),
    // or team_chase's blocks
    static constexpr int SCR = LANE ? (TEAM > 4 ? 4 * H : 0) : team_chase_scratch<H>();
    static constexpr int LDS_DOUBLES = WC * LDW + S * SCR;
    // prefetch registers: one batch of columns spread over the wave
    static constexpr int PFC = LANE ? 2 * H * BATCH : 0;
    static constexpr int PFN = LANE ? (PFC * LDW + NT - 1) / NT : 1;
};

struct GroupArgs {
    int64_t n;
    double* band;      // global band, ld = 4h + 1
    int nsweeps;
    int ngroups;
    int* ticket;
    int* done;         // ngroups watermarks
    int* error;        // the plan's status word: nonzero stops every block
    uint64_t wait_ticks;   // a wait gives up after this many ticks of the 100 MHz clock
};

template <int H>
__device__ __forceinline__ int nchase_of(int n, int i) {
    return (n - 2 - i * H) / (2 * H) + 1;
}

template <int H>
__global__ __launch_bounds__(GroupCfg<H>::NT) void band_group_kernel(GroupArgs a) {
    typedef GroupCfg<H> C;
    constexpr int H2 = C::H2, TEAM = C::TEAM, S = C::S, WC = C::WC, LDW = C::LDW, LAG = C::LAG;
    extern __shared__ double smem[];
    double* ring = smem;
    __shared__ int g_sh, abort_sh, fresh_sh;
    __shared__ int vis_sh;
    const int t = threadIdx.x;
    const int tm = t / TEAM, u = t % TEAM;
    double* scr = smem + WC * LDW + tm * C::SCR;
    // column and row indices fit in 32 bits (n * LDW < 2^31 is checked on the host)
    const int n = (int)a.n;
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
        // uniform across the block: keep the schedule arithmetic scalar
        const int g = __builtin_amdgcn_readfirstlane(g_sh);
        __syncthreads();
        if (g >= a.ngroups) break;
        const int i0 = 1 + g * S;
        const int ns = (a.nsweeps - i0 + 1 < S) ? (a.nsweeps - i0 + 1) : S;
        // Sweeps finish in order: sweep s does its last chase at step
        // f(s) = J_s + LAG s, which increases with s.  At step tau the active
        // sweeps are s_lo(tau) .. s_hi(tau) with s_lo the first s with
        // f(s) >= tau and s_hi = min(ns-1, (tau-1)/LAG); window ends decrease
        // and window starts decrease with s, so the extremes are at s_lo
        // (end) and s_hi (start).
        auto Jof = [&](int s) -> int { return nchase_of<H>(n, i0 + s); };
        auto wstart = [&](int s, int j) -> int {
            const int o = (i0 + s) * H + (j - 1) * H2;
            return (j == 1) ? o - H : o - H2;
        };
        auto wend = [&](int s, int j) -> int {
            const int e = (i0 + s) * H + j * H2;
            return e < n ? e : n;
        };
        const int tau_end = LAG * (ns - 1) + Jof(ns - 1) > Jof(0) ? LAG * (ns - 1) + Jof(ns - 1) : Jof(0);
        // my sweep
        const int my_i = i0 + tm;
        const int my_J = (tm < ns) ? Jof(tm) : 0;
        LaneCarry<H> carry;              // lane mode: the last chase's below block
        int loaded = wstart(0, 1);   // columns [written, loaded) are in the ring
        int written = loaded;
        int pub_pending = -1;        // watermark whose write-back is in flight
        int pf_lo = 0, pf_hi = 0;    // columns [pf_lo, pf_hi) prefetched into pf
        double pf[C::PFN];
        // lowest active sweep and the step of its last chase
        int s_lo = 0, f_lo = Jof(0);

        auto lowest_active = [&](int s0, int tau) {
            int sl = s0;
            while (sl < ns && Jof(sl) + LAG * sl < tau) ++sl;
            return sl;
        };
        // columns the group needs through step tb, given its lowest active sweep
        auto need_through = [&](int sl, int tb) -> int {
            if (sl >= ns) return loaded;
            if (Jof(sl) + LAG * sl <= tb) return n;   // a sweep ends by then: its window reaches n
            const int jj = tb - LAG * sl;
            return (jj >= 1) ? wend(sl, jj) : wend(sl, 1);
        };
        // ring slot of column c (any c inside [written, written + WC))
        auto slot = [&](int c) { return c % WC; };

        for (int tau_s = 1; tau_s <= tau_end; ++tau_s) {
            if (tau_s > f_lo && s_lo < ns) {
                s_lo = lowest_active(s_lo, tau_s);
                f_lo = (s_lo < ns) ? Jof(s_lo) + LAG * s_lo : tau_end;
            }
            // ---- columns needed within the next BATCH steps
            if (((tau_s - 1) % C::BATCH) == 0 && s_lo < ns) {
                const int need = need_through(s_lo, tau_s + C::BATCH - 1);
                // the columns prefetched a batch ago go to the ring (their loads
                // were waited for at the last write-back)
                if (pf_hi > pf_lo) {
                    const int cnt = (int)(pf_hi - pf_lo) * LDW;
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
                                    if (wall_clock64() - t0 > a.wait_ticks) {
                                        atomicOr(a.error, sbr::STATUS_STALLED);
                                        abort_sh = 1;
                                        break;
                                    }
                                }
                                vis_sh = d;
                                fresh_sh = 1;
                                // one acquire for the block (CU L1 + XCD L2)
                                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                            }
                        }
                        __syncthreads();
                        if (abort_sh) return;
                    }
                    // load [loaded, need) into the ring
                    const int cnt = (int)(need - loaded) * LDW;
                    const int sl0 = slot(loaded);
                    for (int idx = t; idx < cnt; idx += C::NT) {
                        const int k = idx / LDW, d = idx - k * LDW;
                        int sl = sl0 + k;
                        if (sl >= WC) sl -= WC;
                        ring[sl * LDW + d] = (loaded + k + d < n) ? gband[(loaded + k) * (int64_t)LDW + d] : 0.0;
                    }
                    loaded = need;
                }
                // prefetch what the next batch will need, as far as the previous
                // group has already released it: the loads run during this batch
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
                        const int cnt = (int)(want - loaded) * LDW;
#pragma unroll
                        for (int p = 0; p < C::PFN; ++p) {
                            const int idx = t + p * C::NT;
                            if (idx < cnt) {
                                const int k = idx / LDW, d = idx - k * LDW;
                                // entries past the matrix end read as zero
                                pf[p] = (loaded + k + d < n) ? gband[(loaded + k) * (int64_t)LDW + d] : 0.0;
                            }
                        }
                        pf_lo = loaded;
                        pf_hi = want;
                    }
                }
                __syncthreads();
            }

            // ---- the chases of this step, one per team (or lane)
            const int jl = tau_s - LAG * tm;
            const bool act = (tm < ns) && (jl >= 1) && (jl <= my_J);
            const int j = act ? (int)jl : 0;
            const int o = act ? my_i * H + (j - 1) * H2 : 0;
            const int nr = act ? ((n - o < H2) ? (int)(n - o) : H2) : 0;
            const int cq = (j == 1) ? o - H : o - H2;
            int nbl = (int)(n - (o + H2));
            if (nbl > H2) nbl = H2;
            const int nbr = (act && nbl > 0) ? nbl : 0;
            if constexpr (!C::LANE) {
                cs = cq;
                sbase = act ? cs % WC : 0;
            }

            if constexpr (C::LANE) {
                // columns past the matrix end can only be touched once
                // o + 2h > n (never for h = 1: o <= n - 2)
                const bool guard = act && (o + H2 > n);
                if constexpr (TEAM == 1) {
                    LaneRot rot;
                    if (act) lane_chase_qr<WC, LDW>(ring, o, j == 1, carry, rot);
                    __syncthreads();   // the update phases read QR blocks of the neighbours
                    if (act) lane_chase_update<WC, LDW>(ring, o, j == 1, carry, rot);
                } else {
                    TeamRefl<H, TEAM> rf;
                    if (act) {
                        if (!guard) team_lane_chase_qr<H, TEAM, WC, LDW, false>(ring, o, j == 1, nr, u, carry, rf);
                        else team_lane_chase_qr<H, TEAM, WC, LDW, true>(ring, o, j == 1, nr, u, carry, rf);
                    }
                    __syncthreads();
                    if (act) {
                        if (!guard)
                            team_lane_chase_update<H, TEAM, WC, LDW, false>(ring, o, j == 1, nr, nbr, u, carry, rf,
                                                                            scr);
                        else
                            team_lane_chase_update<H, TEAM, WC, LDW, true>(ring, o, j == 1, nr, nbr, u, carry, rf,
                                                                           scr);
                    }
                }
            } else {
                if (act) team_chase<H>(R, o, cq, nr, nbr, j, u, scr);
            }
            team_sync<TEAM>();
            __syncthreads();   // next step reads columns the neighbouring sweeps wrote

            // ---- write back columns no sweep of the group will touch again.
            // The stores of one batch are published at the next batch end (or
            // at the group's end), by when they have long completed, so the
            // wave never stalls on a store round trip.
            const bool last = (tau_s == tau_end);
            if (last || (tau_s % C::BATCH) == 0) {
                int done = last ? loaded : n;
                if (!last) {
                    // next step's active range: the smallest window start is at
                    // the highest started sweep; the next sweep to start (if
                    // any) begins at its first window
                    const int tn = tau_s + 1;
                    int s_hi = (int)((tn - 1) / LAG);
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
                // the previous batch's stores (and the prefetch loads) are done
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (t == 0 && pub_pending >= 0 && !last) sbr_store_release(&a.done[g], (int)pub_pending);
                if (done > written) {
                    const int cnt = (int)(done - written) * LDW;
                    const int sl0 = slot(written);
                    for (int idx = t; idx < cnt; idx += C::NT) {
                        const int k = idx / LDW, d = idx - k * LDW;
                        int sl = sl0 + k;
                        if (sl >= WC) sl -= WC;
                        gband[(written + k) * (int64_t)LDW + d] = ring[sl * LDW + d];
                    }
                    written = done;
                    pub_pending = written;
                }
                if (last) {
                    // stores complete to L2; thread 0's release below writes the L2 back
                    __builtin_amdgcn_s_waitcnt(0);
                    __syncthreads();
                    if (t == 0) {
                        // everything this group loaded is back; columns it never
                        // loaded are final once the previous group is complete
                        if (g > 0) {
                            const uint64_t t0 = wall_clock64();
                            while (__hip_atomic_load(&a.done[g - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                                   (int)n) {
                                __builtin_amdgcn_s_sleep(2);
                                if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                                if (wall_clock64() - t0 > a.wait_ticks) {
                                    atomicOr(a.error, sbr::STATUS_STALLED);
                                    break;
                                }
                            }
                        }
                        sbr_store_release(&a.done[g], (int)n);
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int H>
void launch_group(int64_t n, double* band, const sbr::StageCtl& ctl, hipStream_t s) {
    typedef GroupCfg<H> C;
    const int64_t nsweeps = (n - 2) / H;
    if (nsweeps < 1) return;
    const int64_t ngroups = (nsweeps + C::S - 1) / C::S;
    GroupArgs a;
    a.n = n;
    a.band = band;
    a.nsweeps = (int)nsweeps;
    a.ngroups = (int)ngroups;
    a.ticket = ctl.flags;
    a.done = ctl.flags + 1;
    a.error = ctl.status;
    a.wait_ticks = ctl.wait_ticks;
    sbr::launch_fill_int(ctl.flags, ngroups + 1, 0, s);
    int64_t grid = ngroups < (C::LANE ? 1024 : 256) ? ngroups : (C::LANE ? 1024 : 256);
    if (ctl.max_grid > 0 && grid > ctl.max_grid) grid = ctl.max_grid;
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

void launch_band_halve_group(int64_t n, double* band, int b, const StageCtl& ctl, hipStream_t s) {
    switch (b) {
        case 2: launch_group<1>(n, band, ctl, s); break;
        case 4: launch_group<2>(n, band, ctl, s); break;
        case 8: launch_group<4>(n, band, ctl, s); break;
        case 16: launch_group<8>(n, band, ctl, s); break;
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
