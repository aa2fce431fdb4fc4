// sbr_band.hip -- band-to-band reduction (Algorithm 4.2 with k = 2) and the
// band storage helpers.
//
// Band storage: lower band, column-major by column: band[d + j*ldb] holds
// B(j + d, j).  A halving stage on bandwidth b = 2h needs ldb >= 2b + 1: a
// chase fills entries up to distance 2b - 1 below the diagonal.
//
// One halving b -> h.  Sweep i (1-based) eliminates columns [(i-1)h, ih)
// below the h-th sub-diagonal and chases the bulge down; chase (i, j) has
//   o = o_qr.r = ih + (j-1)b,
//   QR block  rows [o, o + n_r) x cols [o - h, o) for j = 1, [o - b, o - b + h)
//             for j > 1, n_r = min(n - o, b);
//   update    rows [o, o + n_r) x cols [o, o + 2b) for j = 1 and
//             [o - h, o + 2b) for j > 1 (the exact extents; clipped at n);
// with [U, T, R] = QR(block), the block set to [R; 0], W = B[upd, qr] U T,
// V = -W, V[qr rows] += 1/2 U T^T U^T W[qr rows], B[qr, upd] += U V^T and
// B[upd, qr] += V U^T.  Sweep i has chases while o <= n - 2; sweeps run
// while ih <= n - 2.
//
// In lower storage the update splits into the "left" block B[qr, o-h:o]
// (j > 1), the diagonal block B[qr, qr] and the "below" block
// B[o+b:o+2b, qr].
//
// Pipelining: a persistent grid takes sweeps in increasing order from a
// ticket counter; chase (i, j) starts after chase (i, j-1) (same block) and
// after sweep i-1 has finished chase j + 2 (or the whole sweep).  Every
// pair of chases that writes a common entry is then ordered as in the
// sequential loop nest (a new panel may start once the previous bulge has
// been chased three times; two is not enough because chase (i-1, j+2)
// factors entries that chase (i, j) updates).
#include "sbr_device.h"
#include "sbr_internal.h"

namespace {

__global__ void dense_to_band_kernel(int64_t n, const double* __restrict__ A, int64_t lda, int b,
                                     double* __restrict__ band, int64_t ldb) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * ldb) return;
    const int64_t d = idx % ldb, j = idx / ldb;
    double v = 0.0;
    if (d <= b && j + d < n) v = A[(j + d) + j * lda];
    band[idx] = v;
}

__global__ void band_copy_kernel(int64_t n, const double* __restrict__ src, int64_t lds, int keep,
                                 double* __restrict__ dst, int64_t ldd) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * ldd) return;
    const int64_t d = idx % ldd, j = idx / ldd;
    double v = 0.0;
    if (d <= keep && d < lds && j + d < n) v = src[d + j * lds];
    dst[idx] = v;
}

__global__ void band_to_tridiag_kernel(int64_t n, const double* __restrict__ band, int64_t ldb,
                                       double* __restrict__ d, double* __restrict__ e) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    d[j] = band[j * ldb];
    if (j + 1 < n) e[j] = band[1 + j * ldb];
}

__global__ void fill_int_kernel(int* p, int64_t count, int v) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < count) p[idx] = v;
}

struct ChaseArgs {
    int64_t n;
    double* band;
    int64_t ldb;
    int nsweeps;
    int* ticket;       // one int
    int* progress;     // nsweeps + 1 ints; progress[i] = chases of sweep i done
    double* gscratch;  // per-block scratch (global variant)
    int64_t scratch_stride;
    int* error;        // set to 1 if a wait gave up; every block then exits
};

// A wait for the previous sweep gives up after this many ticks of the
// 100 MHz wall clock (10 s): the schedule guarantees progress, so this only
// bounds the kernel's lifetime should that guarantee ever be broken.
constexpr uint64_t WAIT_LIMIT_TICKS = 1000000000ull;

constexpr int SWEEP_DONE = 1 << 30;

__device__ __forceinline__ double bget(const double* band, int64_t ldb, int64_t r, int64_t c) {
    const int64_t d = r - c;   // caller guarantees r >= c
    return (d < ldb) ? band[d + c * ldb] : 0.0;
}
__device__ __forceinline__ void bput(double* band, int64_t ldb, int64_t r, int64_t c, double v) {
    const int64_t d = r - c;
    if (d < ldb) band[d + c * ldb] = v;
}

template <int H>
struct ChaseLayout {
    static constexpr int H2 = 2 * H;
    static constexpr int QB = 0;                 // 2H x H   QR block, then U
    static constexpr int DB = QB + H2 * H;       // 2H x 2H  diagonal block (full)
    static constexpr int TT = DB + H2 * H2;      // H x H    T
    static constexpr int YY = TT + H * H;        // 2H x H   Y = U T
    static constexpr int WR = YY + H2 * H;       // 2H x H   W of the qr rows, then V; W of "below" rows
    static constexpr int GG = WR + H2 * H;       // H x H    U^T U, then U^T W
    static constexpr int MM = GG + H * H;        // H x H    T^T U^T W, then W of the "left" block
    static constexpr int XX = MM + H * H;        // 2H x 2H  left / below block staging
    static constexpr int TAU = XX + H2 * H2;     // H
    static constexpr int VB = TAU + H;           // 2 x 2H   reflector staging for the QR
    static constexpr int TOTAL = VB + 2 * H2;
};

// lanes per column in the chase QR: at most 8 (DPP group sums), at most 2h
template <int H, int NT>
constexpr int chase_tpcq() {
    return (NT / H < 2 * H) ? ((NT / H < 8) ? NT / H : 8) : ((2 * H < 8) ? 2 * H : 8);
}

// Register blocks of the chase's small products: MH = 2h x h outputs,
// HH = h x h, MM = 2h x 2h (256 threads).
template <int H> struct ChaseTiles {
    static constexpr int MH_M = 1, MH_N = 1, HH_M = 1, HH_N = 1, MM_M = 1, MM_N = 1;
};
template <> struct ChaseTiles<64> {
    static constexpr int MH_M = 4, MH_N = 4, HH_M = 4, HH_N = 4, MM_M = 4, MM_N = 4;
};
template <> struct ChaseTiles<32> {
    static constexpr int MH_M = 2, MH_N = 4, HH_M = 2, HH_N = 2, MM_M = 4, MM_N = 4;
};
template <> struct ChaseTiles<16> {
    static constexpr int MH_M = 1, MH_N = 2, HH_M = 1, HH_N = 1, MM_M = 2, MM_N = 2;
};

template <int H, int NT, bool LDS>
__global__ __launch_bounds__(NT) void chase_kernel(ChaseArgs a) {
    typedef ChaseLayout<H> L;
    constexpr int H2 = 2 * H;
    constexpr int TPCQ = chase_tpcq<H, NT>();
    constexpr int NQ = H * TPCQ;
    constexpr int RPT = H2 / TPCQ;
    static_assert(TPCQ >= 2 && TPCQ <= 64 && (TPCQ & (TPCQ - 1)) == 0 && RPT >= 1 && NQ <= NT, "qr layout");
    extern __shared__ double dyn_smem[];
    double* sm = LDS ? dyn_smem : (a.gscratch + (int64_t)blockIdx.x * a.scratch_stride);
    double* Qb = sm + L::QB;
    double* Db = sm + L::DB;
    double* Tm = sm + L::TT;
    double* Yb = sm + L::YY;
    double* Wr = sm + L::WR;
    double* Gm = sm + L::GG;
    double* Mm = sm + L::MM;
    double* Xb = sm + L::XX;
    double* tau = sm + L::TAU;
    double* vbuf = sm + L::VB;
    __shared__ int sweep_sh;
    __shared__ int abort_sh;

    const int t = threadIdx.x;
    const int64_t n = a.n, ldb = a.ldb;
    double* band = a.band;
    const int qc = t / TPCQ, qs = t % TPCQ;

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
        const int64_t nchase = (n - 2 - (int64_t)i * H) / H2 + 1;
        for (int64_t j = 1; j <= nchase; ++j) {
            if (i > 1) {
                if (t == 0) {
                    const int need = (int)(j + 2);
                    const uint64_t t0 = wall_clock64();
                    // spin on relaxed loads (an acquire per poll would invalidate
                    // the L2 each time); one acquire fence once the flag is seen
                    while (__hip_atomic_load(&a.progress[i - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                           need) {
                        __builtin_amdgcn_s_sleep(2);
                        if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            abort_sh = 1;
                            break;
                        }
                        if (wall_clock64() - t0 > WAIT_LIMIT_TICKS) {
                            atomicExch(a.error, 2 * H);   // the stage (its bandwidth b) that stalled
                            abort_sh = 1;
                            break;
                        }
                    }
                    // one acquire for the block: it invalidates this CU's L1 and
                    // the XCD's L2, which every wave of the block reads through
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                __syncthreads();
                if (abort_sh) return;
            }
            const int64_t o = (int64_t)i * H + (j - 1) * H2;
            const int nr = (int)((n - o < H2) ? (n - o) : H2);
            const int64_t cq = (j == 1) ? o - H : o - H2;
            int64_t nb64 = n - (o + H2);
            if (nb64 > H2) nb64 = H2;
            const int nbr = nb64 > 0 ? (int)nb64 : 0;

            // ---- QR block straight into registers (column groups), diagonal block into Db
            double x[RPT];
            if (t < NQ) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int row = qs + TPCQ * r;
                    x[r] = (row < nr) ? bget(band, ldb, o + row, cq + qc) : 0.0;
                }
            }
            for (int idx = t; idx < H2 * H2; idx += NT) {
                const int r = idx % H2, c = idx / H2;
                double v = 0.0;
                if (r < nr && c < nr) v = (r >= c) ? bget(band, ldb, o + r, o + c) : bget(band, ldb, o + c, o + r);
                Db[idx] = v;
            }

            // ---- Householder QR of the block: one barrier per reflector, column
            // sums inside each TPCQ-lane group
            for (int k = 0; k < H; ++k) {
                double* v = vbuf + (k & 1) * H2;
                if (t < NQ && qc == k) {
                    double ss = 0.0, xk = 0.0;
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int row = qs + TPCQ * r;
                        if (row > k) ss += x[r] * x[r];
                        else if (row == k) xk = x[r];
                    }
                    ss = group_sum<TPCQ>(ss);
                    xk = group_sum<TPCQ>(xk);
                    double beta, tk, scal;
                    if (ss == 0.0) {
                        beta = xk; tk = 0.0; scal = 0.0;
                    } else {
                        const double nrm = sqrt(xk * xk + ss);
                        beta = (xk >= 0.0) ? -nrm : nrm;
                        tk = (beta - xk) / beta;
                        scal = 1.0 / (xk - beta);
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
                if (t < NQ && qc > k) {
                    const double tk = tau[k];
                    if (tk != 0.0) {
                        double d = 0.0;
#pragma unroll
                        for (int r = 0; r < RPT; ++r) d += v[qs + TPCQ * r] * x[r];
                        d = group_sum<TPCQ>(d);
                        const double f = tk * d;
#pragma unroll
                        for (int r = 0; r < RPT; ++r) x[r] -= f * v[qs + TPCQ * r];
                    }
                }
            }
            // U into Qb (unit lower, a zero column where no reflector was
            // applied), [R; 0] into the band
            if (t < NQ) {
                const double tk = tau[qc];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int row = qs + TPCQ * r;
                    double u = 0.0;
                    if (tk != 0.0) u = (row == qc) ? 1.0 : ((row > qc) ? x[r] : 0.0);
                    Qb[row + qc * H2] = u;
                    if (row < nr) bput(band, ldb, o + row, cq + qc, (row <= qc) ? x[r] : 0.0);
                }
            }
            __syncthreads();

            typedef ChaseTiles<H> TL;
            auto U = [&](int i, int k) -> double { return Qb[i + k * H2]; };
            auto Ut = [&](int i, int k) -> double { return Qb[k + i * H2]; };
            // ---- T (forward, columnwise): G = U^T U (strict upper), then
            // T[c][c] = tau_c, T[0:c, c] = -tau_c T[0:c, 0:c] G[0:c, c]
            block_gemm<H, H, H2, TL::HH_M, TL::HH_N, NT>(
                t, Ut, U, [&](int i, int jj, double v) {
                    Gm[i + jj * H] = (i < jj) ? v : 0.0;
                    Tm[i + jj * H] = 0.0;
                });
            __syncthreads();
            for (int c = 0; c < H; ++c) {
                const double tc = tau[c];
                for (int ra = t; ra <= c; ra += NT) {
                    if (ra == c) {
                        Tm[c + c * H] = tc;
                    } else {
                        double acc = 0.0;
                        for (int k = ra; k < c; ++k) acc += Tm[ra + k * H] * Gm[k + c * H];
                        Tm[ra + c * H] = -tc * acc;
                    }
                }
                __syncthreads();
            }
            // ---- Y = U T
            block_gemm<H2, H, H, TL::MH_M, TL::MH_N, NT>(
                t, U, [&](int k, int jj) -> double { return Tm[k + jj * H]; },
                [&](int i, int jj, double v) { Yb[i + jj * H2] = v; });
            __syncthreads();
            // ---- W_R = D Y
            block_gemm<H2, H, H2, TL::MH_M, TL::MH_N, NT>(
                t, [&](int i, int k) -> double { return Db[i + k * H2]; },
                [&](int k, int jj) -> double { return Yb[k + jj * H2]; },
                [&](int i, int jj, double v) { Wr[i + jj * H2] = v; });
            __syncthreads();
            // ---- G = U^T W_R ; M = T^T G ; V_R = 1/2 U M - W_R
            block_gemm<H, H, H2, TL::HH_M, TL::HH_N, NT>(
                t, Ut, [&](int k, int jj) -> double { return Wr[k + jj * H2]; },
                [&](int i, int jj, double v) { Gm[i + jj * H] = v; });
            __syncthreads();
            block_gemm<H, H, H, TL::HH_M, TL::HH_N, NT>(
                t, [&](int i, int k) -> double { return Tm[k + i * H]; },
                [&](int k, int jj) -> double { return Gm[k + jj * H]; },
                [&](int i, int jj, double v) { Mm[i + jj * H] = v; });
            __syncthreads();
            block_gemm<H2, H, H, TL::MH_M, TL::MH_N, NT>(
                t, U, [&](int k, int jj) -> double { return Mm[k + jj * H]; },
                [&](int i, int jj, double v) { Wr[i + jj * H2] = 0.5 * v - Wr[i + jj * H2]; });
            __syncthreads();
            // ---- diagonal block: B += [U, V_R] [V_R, U]^T (lower part)
            block_gemm<H2, H2, H2, TL::MM_M, TL::MM_N, NT>(
                t, [&](int i, int k) -> double { return (k < H) ? Qb[i + k * H2] : Wr[i + (k - H) * H2]; },
                [&](int k, int jj) -> double { return (k < H) ? Wr[jj + k * H2] : Qb[jj + (k - H) * H2]; },
                [&](int i, int jj, double v) {
                    if (i >= jj && i < nr) bput(band, ldb, o + i, o + jj, Db[i + jj * H2] + v);
                });
            __syncthreads();
            // ---- left block (j > 1): X -= U (X^T Y)^T
            if (j > 1) {
                for (int idx = t; idx < H2 * H; idx += NT) {
                    const int r = idx % H2, c = idx / H2;
                    Xb[idx] = (r < nr) ? bget(band, ldb, o + r, o - H + c) : 0.0;
                }
                __syncthreads();
                block_gemm<H, H, H2, TL::HH_M, TL::HH_N, NT>(
                    t, [&](int c, int r) -> double { return Xb[r + c * H2]; },
                    [&](int r, int k) -> double { return Yb[r + k * H2]; },
                    [&](int c, int k, double v) { Mm[c + k * H] = v; });
                __syncthreads();
                block_gemm<H2, H, H, TL::MH_M, TL::MH_N, NT>(
                    t, U, [&](int k, int c) -> double { return Mm[c + k * H]; },
                    [&](int i, int c, double v) {
                        if (i < nr) bput(band, ldb, o + i, o - H + c, Xb[i + c * H2] - v);
                    });
                __syncthreads();
            }
            // ---- below block: X -= (X Y) U^T
            if (nbr > 0) {
                for (int idx = t; idx < H2 * H2; idx += NT) {
                    const int r = idx % H2, c = idx / H2;
                    Xb[idx] = (r < nbr) ? bget(band, ldb, o + H2 + r, o + c) : 0.0;
                }
                __syncthreads();
                block_gemm<H2, H, H2, TL::MH_M, TL::MH_N, NT>(
                    t, [&](int i, int c) -> double { return Xb[i + c * H2]; },
                    [&](int c, int k) -> double { return Yb[c + k * H2]; },
                    [&](int i, int k, double v) { Wr[i + k * H2] = v; });
                __syncthreads();
                block_gemm<H2, H2, H, TL::MM_M, TL::MM_N, NT>(
                    t, [&](int i, int k) -> double { return Wr[i + k * H2]; },
                    [&](int k, int c) -> double { return Qb[c + k * H2]; },
                    [&](int i, int c, double v) {
                        if (i < nbr) bput(band, ldb, o + H2 + i, o + c, Xb[i + c * H2] - v);
                    });
            }
            // ---- publish: every wave's stores complete to L2, then one
            // agent-scope release (L2 write-back) by thread 0 covers the block
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (t == 0) sbr_store_release(&a.progress[i], (j == nchase) ? SWEEP_DONE : (int)j);
        }
    }
}

template <int H>
constexpr int chase_nt() { return H <= 4 ? 64 : (H == 8 ? 128 : 256); }

template <int H>
constexpr bool chase_in_lds() { return H <= 32; }

template <int H>
int chase_grid(int64_t n) {
    const int64_t nsweeps = (n - 2) / H;
    const int64_t cap = chase_in_lds<H>() ? 1024 : 256;
    int64_t g = nsweeps < cap ? nsweeps : cap;
    return (int)(g < 1 ? 1 : g);
}

template <int H>
void launch_chase(int64_t n, double* band, int64_t ldb, double* scratch, int* flags, int* error, int max_grid,
                  hipStream_t s) {
    const int64_t nsweeps = (n - 2) / H;
    if (nsweeps < 1) return;
    constexpr int NT = chase_nt<H>();
    constexpr bool LDS = chase_in_lds<H>();
    ChaseArgs a;
    a.n = n;
    a.band = band;
    a.ldb = ldb;
    a.nsweeps = (int)nsweeps;
    a.ticket = flags;
    a.progress = flags + 1;
    a.gscratch = scratch;
    a.scratch_stride = ChaseLayout<H>::TOTAL;
    a.error = error;
    const int64_t nflags = nsweeps + 2;
    fill_int_kernel<<<(unsigned)((nflags + 255) / 256), 256, 0, s>>>(flags, nflags, 0);
    int grid = chase_grid<H>(n);
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    const size_t shm = LDS ? (size_t)ChaseLayout<H>::TOTAL * sizeof(double) : 0;
    chase_kernel<H, NT, LDS><<<grid, NT, shm, s>>>(a);
}

template <int H>
int set_chase_attr() {
    constexpr int NT = chase_nt<H>();
    if (!chase_in_lds<H>()) return 0;
    const int bytes = ChaseLayout<H>::TOTAL * (int)sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)chase_kernel<H, NT, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace

namespace sbr {

void launch_dense_to_band(int64_t n, const double* A, int64_t lda, int b, double* band, int64_t ldband,
                          hipStream_t s) {
    const int64_t tot = n * ldband;
    if (tot <= 0) return;
    dense_to_band_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(n, A, lda, b, band, ldband);
}

void launch_band_copy(int64_t n, const double* src, int64_t ldsrc, int keep, double* dst, int64_t lddst,
                      hipStream_t s) {
    const int64_t tot = n * lddst;
    if (tot <= 0) return;
    band_copy_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(n, src, ldsrc, keep, dst, lddst);
}

int64_t chase_workspace_doubles(int64_t n, int b, int* grid_out) {
    int64_t per = 0;
    int grid = 1;
    (void)per;
    if (grid_out) *grid_out = grid;
    return band_mfma_workspace_doubles(n, b);
}

int64_t chase_flag_ints(int64_t n, int b) {
    const int h = b / 2;
    if (h < 1) return 0;
    return (n - 2) / h + 2 > 2 ? (n - 2) / h + 2 : 2;
}

void launch_band_halve(int64_t n, double* band, int64_t ldband, int b, bool f32, double* scratch, int* flags,
                       int* error, int max_grid, hipStream_t s) {
    (void)f32;
    if (band_mfma_supported(b)) {
        launch_band_halve_mfma(n, band, ldband, b, scratch, flags, error, max_grid, s);
        return;
    }
    // the group kernel indexes the band with 32-bit integers
    if (band_group_supported(b) && ldband == 2 * b + 1 && n * (int64_t)ldband < (int64_t)INT32_MAX) {
        launch_band_halve_group(n, band, ldband, b, flags, error, max_grid, s);
        return;
    }
    switch (b) {
        case 2: launch_chase<1>(n, band, ldband, scratch, flags, error, max_grid, s); break;
        case 4: launch_chase<2>(n, band, ldband, scratch, flags, error, max_grid, s); break;
        case 8: launch_chase<4>(n, band, ldband, scratch, flags, error, max_grid, s); break;
        case 16: launch_chase<8>(n, band, ldband, scratch, flags, error, max_grid, s); break;
        case 32: launch_chase<16>(n, band, ldband, scratch, flags, error, max_grid, s); break;
        case 64: launch_chase<32>(n, band, ldband, scratch, flags, error, max_grid, s); break;
        case 128: launch_chase<64>(n, band, ldband, scratch, flags, error, max_grid, s); break;
        default: break;
    }
}

void launch_fill_int(int* p, int64_t count, int v, hipStream_t s) {
    if (count <= 0) return;
    fill_int_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(p, count, v);
}

void launch_band_to_tridiag(int64_t n, const double* band, int64_t ldband, double* d, double* e, hipStream_t s) {
    if (n <= 0) return;
    band_to_tridiag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, band, ldband, d, e);
}

int init_band_attributes() {
    int rc = 0;
    rc |= set_chase_attr<1>();
    rc |= set_chase_attr<2>();
    rc |= set_chase_attr<4>();
    rc |= set_chase_attr<8>();
    rc |= set_chase_attr<16>();
    rc |= set_chase_attr<32>();
    return rc;
}

}  // namespace sbr
