// sbr_bisect.hip -- eigenvalues of the final tridiagonal by Sturm-sequence
// bisection (the last step of Algorithm 4.3, "compute the eigenvalues of the
// thin band", done here on the tridiagonal reached by the halvings).
//
// The count of eigenvalues below x is the number of sign changes of the
// leading principal minors of T - x I (SturmChain: the three-term recurrence
// on data scaled by a power of two, rescaled every 16 steps; a chain whose
// minors come near underflow is recounted with the guarded ratio recurrence
// q_i = (d_i - x) - e_{i-1}^2 / q_{i-1}, SturmRatio).  The interval is the
// Gershgorin interval widened by 2.1 (n eps |T| + 2 pivmin); every index ends
// no wider than the bisection of that interval by
// I = ceil(log2((hi - lo) / (eps max(|lo|, |hi|)))) + 2 halvings would leave
// it, stopping early when no point falls strictly inside.
//
// Two passes share the work of the first halvings, which is the same for all
// indices: the counts at 2n evenly spaced points of the interval (one thread
// a point), after which each index starts from the grid cell that holds its
// eigenvalue (a binary search in the counts), about log2(2n) halvings in one
// pass; then multisection inside the cell (G lanes per index).  d and e^2 are
// streamed through LDS in chunks that every thread of the block reads at the
// same address (broadcast).
//
// A tridiagonal with a NaN or an infinity has no meaningful Sturm counts: the
// setup kernel flags it (and raises the non-finite bit of the plan's status
// word when there is one) and every eigenvalue comes out NaN; so does every
// eigenvalue of a call whose band stage was abandoned (status word nonzero).
#include <float.h>

#include <mutex>

#include "sbr_device.h"
#include "sbr_internal.h"

// Fixed device scratch of the allocation-free tridiagonal entry point: e^2
// (NOALLOC_MAX_N doubles) and the grid counts (2 NOALLOC_MAX_N ints), then
// the setup record.  One copy per GPU, held
// until the process ends.  Host code must not use this name as an address (it
// names a host-side stand-in): the device address comes from
// hipGetSymbolAddress, see noalloc_scratch below.
constexpr int64_t NOALLOC_E2_DOUBLES = 2 * sbr::NOALLOC_MAX_N;
constexpr int64_t NOALLOC_SETUP_DOUBLES = (sizeof(sbr::BisectSetup) + sizeof(double) - 1) / sizeof(double);
static __device__ __align__(256) double scratch[NOALLOC_E2_DOUBLES + NOALLOC_SETUP_DOUBLES];

namespace {

constexpr int PREP_NT = 256;
// lanes per eigenvalue index in the multisection pass
constexpr int BISECT_LANES = 2;

__global__ __launch_bounds__(PREP_NT) void bisect_prep_kernel(int64_t n, const double* __restrict__ d,
                                                               const double* __restrict__ e,
                                                               double* __restrict__ e2p,
                                                               sbr::BisectSetup* setup, int* status) {
    __shared__ double s_lo[PREP_NT], s_hi[PREP_NT], s_e2[PREP_NT];
    const int t = threadIdx.x;
    double lo = DBL_MAX, hi = -DBL_MAX, emax2 = 1.0;
    bool bad = false;
    for (int64_t i = t; i < n; i += PREP_NT) {
        const double em = (i > 0) ? e[i - 1] : 0.0;
        const double ep = (i + 1 < n) ? e[i] : 0.0;
        const double r = fabs(em) + fabs(ep);
        bad |= !isfinite(d[i]) || !isfinite(em);
        lo = fmin(lo, d[i] - r);
        hi = fmax(hi, d[i] + r);
        e2p[i] = em * em;
        emax2 = fmax(emax2, em * em);
    }
    s_lo[t] = lo;
    s_hi[t] = hi;
    s_e2[t] = emax2;
    const int anybad = __syncthreads_or(bad);
    for (int o = PREP_NT / 2; o > 0; o >>= 1) {
        if (t < o) {
            s_lo[t] = fmin(s_lo[t], s_lo[t + o]);
            s_hi[t] = fmax(s_hi[t], s_hi[t + o]);
            s_e2[t] = fmax(s_e2[t], s_e2[t + o]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double pivmin = DBL_MIN * s_e2[0];
        double l = s_lo[0], h = s_hi[0];
        const double eps = DBL_EPSILON * 0.5;
        double tnorm = fmax(fabs(l), fabs(h));
        const double widen = 2.1 * ((double)n * eps * tnorm + 2.0 * pivmin);
        l -= widen;
        h += widen;
        tnorm = fmax(fabs(l), fabs(h));
        int iters = 0;
        if (h > l && tnorm > 0.0) {
            iters = (int)ceil(log2((h - l) / (eps * tnorm))) + 2;
            if (iters < 0) iters = 0;
        }
        setup->lo = l;
        setup->hi = h;
        setup->pivmin = pivmin;
        setup->scale = (h > l) ? sturm_scale(h - l) : 1.0;
        setup->iters = anybad ? 0 : iters;
        setup->nonfinite = anybad;
        if (anybad && status) atomicOr(status, sbr::STATUS_NONFINITE);
    }
}

// Sturm count at xs (scaled) for every thread of the block: d and e^2 pass
// through LDS scaled by sc, sc^2 in chunks of CH, each thread runs one
// chain; if any chain of the block came near underflow, the block recounts
// with the guarded ratio recurrence and those chains take that count.
// Called by every thread of the block (it synchronises).
template <int NT, int CH>
__device__ __forceinline__ int sturm_count(int n, const double* __restrict__ d, const double* __restrict__ e2p,
                                           double sc, double xs, double2* sde) {
    constexpr int U = 16;
    static_assert(CH % U == 0, "chunks hold whole blocks");
    const int t = threadIdx.x;
    const double sc2 = sc * sc;
    SturmChain ch;
    ch.start();
    for (int s0 = 0; s0 < n; s0 += CH) {
        const int len = (n - s0 < CH) ? (n - s0) : CH;
        __syncthreads();
        for (int i = t; i < len; i += NT) sde[i] = make_double2(d[s0 + i] * sc, e2p[s0 + i] * sc2);
        __syncthreads();
        int i = 0;
        for (; i + U <= len; i += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double2 de = sde[i + u];
                ch.step(de.x - xs, de.y);
            }
            ch.template close_block<U>();
        }
        for (; i < len; ++i) {   // only the last chunk has a partial block
            const double2 de = sde[i];
            ch.step_tail(de.x - xs, de.y);
        }
    }
    ch.finish();
    if (!__syncthreads_or(ch.low)) return ch.cnt;
    SturmRatio r;
    r.start();
    for (int s0 = 0; s0 < n; s0 += CH) {
        const int len = (n - s0 < CH) ? (n - s0) : CH;
        __syncthreads();
        for (int i = t; i < len; i += NT) sde[i] = make_double2(d[s0 + i] * sc, e2p[s0 + i] * sc2);
        __syncthreads();
        for (int i = 0; i < len; ++i) {
            const double2 de = sde[i];
            r.step(de.x - xs, de.y);
        }
    }
    return ch.low ? r.cnt : ch.cnt;
}

// Point j (0 <= j < M) of the grid of M interior points of [lo, hi]; the
// same expression in both passes, so a cell's ends are the points counted.
__device__ __forceinline__ double grid_point(double lo, double hi, int M, int j) {
    return lo + (double)(j + 1) * ((hi - lo) / (double)(M + 1));
}

// First pass: counts at the M grid points, one thread each.
template <int NT, int CH>
__global__ __launch_bounds__(NT) void sturm_grid_kernel(int64_t n, int M, const double* __restrict__ d,
                                                        const double* __restrict__ e2p,
                                                        const sbr::BisectSetup* __restrict__ setup,
                                                        int* __restrict__ gcnt) {
    __shared__ double2 sde[CH];
    if (setup->iters == 0) return;   // the whole grid: no interval to search
    const int j = (int)blockIdx.x * NT + (int)threadIdx.x;
    const double x = grid_point(setup->lo, setup->hi, M, j < M ? j : M - 1);
    const double sc = setup->scale;
    const int cnt = sturm_count<NT, CH>((int)n, d, e2p, sc, x * sc, sde);
    if (j < M) gcnt[j] = cnt;
}

// Second pass, multisection: G lanes per eigenvalue index, lane g counts at
// x_g = a + (g + 1) (c - a) / (G + 1); the interval then shrinks to the piece
// between the last point with count <= k and the next one, a factor G + 1
// per round.  Several lanes per index keep every SIMD busy when there are few
// indices per SIMD.  The start interval is the grid cell [x_jl, x_jh] with
// count(x_jl) <= k < count(x_jh) (x_{-1} = lo, x_M = hi), found by binary
// search; it holds the eigenvalue whatever rounding did to the counts.
template <int NT, int CH, int G>
__global__ __launch_bounds__(NT) void bisect_kernel(int64_t n, int M, const double* __restrict__ d,
                                                    const double* __restrict__ e2p,
                                                    const sbr::BisectSetup* __restrict__ setup,
                                                    const int* __restrict__ gcnt, double* __restrict__ w,
                                                    const int* status) {
    static_assert(G == 2 || G == 4 || G == 8, "lanes per index");
    __shared__ double2 sde[CH];
    const int t = threadIdx.x, g = t % G;
    const int64_t k = (int64_t)blockIdx.x * (NT / G) + t / G;   // 0-based: the (k+1)-th smallest
    const double lo = setup->lo, hi = setup->hi, sc = setup->scale;
    const int iters = setup->iters;
    double a = lo, c = hi;
    bool live = (k < n);
    int rounds = 0;
    if (iters > 0) {
        if (live) {
            int jl = -1, jh = M;
            while (jh - jl > 1) {
                const int mid = (jl + jh) >> 1;
                if (gcnt[mid] > k) jh = mid;
                else jl = mid;
            }
            a = (jl < 0) ? lo : grid_point(lo, hi, M, jl);
            c = (jh >= M) ? hi : grid_point(lo, hi, M, jh);
        }
        // rounds so that (hi - lo) / ((M + 1) (G + 1)^rounds) is below the
        // bisection's final width (hi - lo) / 2^iters
        const double need = (double)iters - log2((double)M + 1.0);
        rounds = need > 0.0 ? (int)ceil(need / log2((double)(G + 1))) : 0;
    }
    for (int it = 0; it < rounds; ++it) {
        const double x = a + (double)(g + 1) * ((c - a) / (double)(G + 1));
        const bool act = live && (c - a) > 0.0 && (x > a) && (x < c);
        if (!__syncthreads_or(act)) break;
        const int cnt = sturm_count<NT, CH>((int)n, d, e2p, sc, x * sc, sde);   // n < 2^31 (entry points)
        // p = number of points left of the eigenvalue (count <= k); the
        // counts are monotone in x up to rounding, so the eigenvalue lies in
        // [x_{p-1}, x_p] (x_{-1} = a, x_G = c).  The lanes of a group hold
        // the same a, c and evaluate the same formula for the points, so
        // they agree on the ends.
        double left = (cnt <= k) ? 1.0 : 0.0;
        double any = act ? 1.0 : 0.0;
        left += dpp_d<0xB1>(left);
        any += dpp_d<0xB1>(any);
        if (G >= 4) {
            left += dpp_d<0x4E>(left);
            any += dpp_d<0x4E>(any);
        }
        if (G >= 8) {
            left += dpp_d<0x141>(left);
            any += dpp_d<0x141>(any);
        }
        if (live) {
            if (any > 0.0) {
                const int p = (int)left;
                const double step = (c - a) / (double)(G + 1);
                const double na = (p == 0) ? a : a + (double)p * step;
                const double nc = (p == G) ? c : a + (double)(p + 1) * step;
                a = na;
                c = nc;
            } else {
                live = false;   // no point of the group strictly inside: converged
            }
        }
    }
    if (k < n && g == 0) {
        const bool failed = setup->nonfinite || (status && *status != 0);
        w[k] = failed ? __builtin_nan("") : a + 0.5 * (c - a);
    }
}

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

}  // namespace

namespace sbr {

int noalloc_scratch(int device, double** e2p, BisectSetup** setup) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        // the caller has made `device` current: its own copy of the array
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        g_scratch_ptr[device] = (double*)ptr;
    }
    *e2p = g_scratch_ptr[device];
    *setup = (BisectSetup*)(g_scratch_ptr[device] + NOALLOC_E2_DOUBLES);
    return 0;
}

void launch_tridiag_eigvals(int64_t n, const double* d, const double* e, double* e2p, BisectSetup* setup,
                            double* w, int* status, hipStream_t s) {
    if (n <= 0) return;
    bisect_prep_kernel<<<1, PREP_NT, 0, s>>>(n, d, e, e2p, setup, status);
    constexpr int NT = 256, CH = 2048, G = BISECT_LANES;
    // the grid counts fill the workspace's second n doubles (2n ints)
    const int M = (int)(n < (int64_t{1} << 29) ? 2 * n : (int64_t{1} << 30));
    int* gcnt = (int*)(e2p + n);
    sturm_grid_kernel<NT, CH><<<(unsigned)((M + NT - 1) / NT), NT, 0, s>>>(n, M, d, e2p, setup, gcnt);
    const unsigned blocks = (unsigned)((n + NT / G - 1) / (NT / G));
    bisect_kernel<NT, CH, G><<<blocks, NT, 0, s>>>(n, M, d, e2p, setup, gcnt, w, status);
}

}  // namespace sbr
