// sbr_internal.h -- host-side launchers shared between the translation units
// of the SBR library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbr {

// ---- sbr_gemm.hip ---------------------------------------------------------
void launch_gemm(bool f32, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 const double* Cin, int64_t ldci, double* Cout, int64_t ldco, hipStream_t s);
int gemm_splits(int64_t M, int64_t N, int64_t K);
void launch_gemm_splitk(bool f32, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                        const double* Cin, int64_t ldci, double* Cout, int64_t ldco, double* part,
                        int splits, hipStream_t s);
// Whether a bulk SYR2K launch over m rows uses 128 x 128 tiles (else 64 x 64).
bool syr2k_big_tiles(int64_t m);
void launch_syr2k_lower(bool f32, int64_t m, int64_t K, const double* U, int64_t ldu, const double* V,
                        int64_t ldv, double* C, int64_t ldc, hipStream_t s);
// The columns j < nc of the same update (all rows, lower triangle only).
void launch_syr2k_lower_cols(bool f32, int64_t m, int64_t nc, int64_t K, const double* U, int64_t ldu,
                             const double* V, int64_t ldv, double* C, int64_t ldc, hipStream_t s);
int symm_splits(int64_t m, int64_t nb);
// M = T^T (U^T W) for b x b T (b <= 128), U and W m x b: split-K partials of
// U^T W in part (splits slices of b x b), then one kernel sums them and
// multiplies by T^T.
void launch_ttuw(int b, int64_t m, const double* U, int64_t ldu, const double* W, int64_t ldw, const double* T,
                 int64_t ldt, double* M, double* part, int splits, hipStream_t s);
// The symmetric product's 32-bit buffer offsets cover the operands
// (lda, ldy up to about 2^20 doubles).
bool symm_offsets_fit(int64_t m, int64_t lda, int64_t ldy, int64_t elem);
// FP32-storage form: C / A are an FP32 copy of the trailing matrix (FP32
// MFMA products, FP32 accumulation into FP32 storage).
void launch_syr2k_lower_f32s(int64_t m, int64_t K, const double* U, int64_t ldu, const double* V, int64_t ldv,
                             float* C, int64_t ldc, hipStream_t s);
void launch_syr2k_lower_cols_f32s(int64_t m, int64_t nc, int64_t K, const double* U, int64_t ldu, const double* V,
                                  int64_t ldv, float* C, int64_t ldc, hipStream_t s);
void launch_symm_lower_f32s(int64_t m, int64_t nb, const float* A, int64_t lda, const double* Y, int64_t ldy,
                            double* W, int64_t ldw, double* part, int splits, hipStream_t s);
// The same with FP32 copies of the skinny operands (half the bytes per
// operand load; the products round to FP32 anyway).
void launch_syr2k_lower_f32s(int64_t m, int64_t K, const float* U, int64_t ldu, const float* V, int64_t ldv,
                             float* C, int64_t ldc, hipStream_t s);
void launch_syr2k_lower_cols_f32s(int64_t m, int64_t nc, int64_t K, const float* U, int64_t ldu, const float* V,
                                  int64_t ldv, float* C, int64_t ldc, hipStream_t s);
void launch_symm_lower_f32s(int64_t m, int64_t nb, const float* A, int64_t lda, const float* Y, int64_t ldy,
                            double* W, int64_t ldw, double* part, int splits, hipStream_t s);
// X (m x nc, ld ldx) rounded to FP32 into Xs (ld lds).
void launch_block_to_f32(int64_t m, int64_t nc, const double* X, int64_t ldx, float* Xs, int64_t lds, hipStream_t s);
// Lower triangle of A's m x m block -> As (FP32); the first nc columns of As's
// m x m block (lower part) -> A (FP64).
void launch_lower_to_f32(int64_t m, const double* A, int64_t lda, float* As, int64_t lds, hipStream_t s);
void launch_cols_to_f64(int64_t m, int64_t nc, const float* As, int64_t lds, double* A, int64_t lda, hipStream_t s);
void launch_symm_lower(bool f32, int64_t m, int64_t nb, const double* A, int64_t lda, const double* Y,
                       int64_t ldy, double* W, int64_t ldw, double* part, int splits, hipStream_t s);
// W = A Y from Yt = Y^T (nb x m, ld ldyt = 128) for full 128 x 128 tiles:
// whether (m, nb, lda) qualify for elements of elem bytes, and the launches
// (same splits and partials): FP64, and the FP32-storage form (A the FP32
// copy, Yt an FP32 copy of Y^T).
bool symm_yt_ok(int64_t m, int64_t nb, int64_t lda, int64_t elem);
void launch_symm_lower_yt(int64_t m, int64_t nb, const double* A, int64_t lda, const double* Yt, int64_t ldyt,
                          double* W, int64_t ldw, double* part, int splits, hipStream_t s);
void launch_symm_lower_yt_f32s(int64_t m, int64_t nb, const float* A, int64_t lda, const float* Yt, int64_t ldyt,
                               double* W, int64_t ldw, double* part, int splits, hipStream_t s);

// ---- sbr_tsqr.hip ---------------------------------------------------------
// TSQR tree over an m x b panel (m >= b): leaves of b rows (the last one takes
// the remainder, < 2b rows), binary tree of stacked b x b R factors.
struct TsqrTree {
    int b = 0;
    int64_t m = 0;
    int levels = 0;               // number of levels; level 0 = leaves
    int count[40];                // nodes per level
    double* slots[40];            // R slots per level, b x b each (ld b)
    double* tau[40];              // b Householder scalars per node
};
// Host-side sizing: doubles needed for the slots and taus of a panel of m rows.
int64_t tsqr_workspace_doubles(int64_t m, int b);
void tsqr_plan(TsqrTree& tr, int64_t m, int b, double* ws);
// Factor the panel P (m x b, ld ldp; overwritten by the leaf reflectors) and
// write the explicit thin Q (m x b, ld ldq).  The R factor is left in
// tsqr_root_r(tr).
bool tsqr_supported(int b);
void launch_tsqr(const TsqrTree& tr, double* P, int64_t ldp, double* Q, int64_t ldq, hipStream_t s);
const double* tsqr_root_r(const TsqrTree& tr);
// Householder reconstruction (single work-group): from Q1 = Q[0:b, 0:b]
// writes U1 (unit lower, into U rows 0..b-1, ld ldu), T (b x b), W1^{-1}
// (b x b) and S (b signs).
void launch_reconstruct(int b, const double* Q, int64_t ldq, double* U, int64_t ldu, double* T, int64_t ldt,
                        double* W1inv, double* S, hipStream_t s);
void launch_zero_block(int64_t m, int64_t nc, double* X, int64_t ldx, hipStream_t s);
// Largest panel width factored by one TSQR tree; wider panels are factored
// recursively (left half, block-reflector update of the right half, lower
// right half, then the merged T).
constexpr int TSQR_MAX_B = 64;
// Band block of the panel: P[0:b, :] = diag(S) R (upper), P[b:m, :] = 0.
void launch_panel_writeback(int64_t m, int b, double* P, int64_t ldp, const double* R, const double* S,
                            hipStream_t s);
// Ragged last panel (m < b rows below the band): unblocked Householder on the
// panel and two-sided application to the trailing m x m block.
void launch_f2b_tail(int64_t m, int b, double* P, int64_t ldp, double* A22, int64_t lda, hipStream_t s);
int init_tsqr_attributes();

// ---- sbr_band.hip ---------------------------------------------------------
void launch_dense_to_band(int64_t n, const double* A, int64_t lda, int b, double* band, int64_t ldband,
                          hipStream_t s);
void launch_band_copy(int64_t n, const double* src, int64_t ldsrc, int keep, double* dst, int64_t lddst,
                      hipStream_t s);
// Workspace (doubles) of one halving stage for bandwidth b and n.
int64_t chase_workspace_doubles(int64_t n, int b);
// Ints of flag/counter storage for one halving stage.
int64_t chase_flag_ints(int64_t n, int b);
// Status bits of the plan's device status word (the values of the public
// SBR_STATUS_* bits).
constexpr int STATUS_STALLED = 1;     // a pipelined wait gave up; the stage was abandoned
constexpr int STATUS_NONFINITE = 2;   // the tridiagonal reached by the reductions is not finite
// Control of one pipelined band stage: flags / tickets (chase_flag_ints of
// them), the status word (status[0], watched by the kernels: once it is
// nonzero every block exits), how long one wait may spin (ticks of the
// 100 MHz clock), and a cap on the grid (0 = automatic, 1 = the sequential
// sweep order).  Bands b <= group_max_b (and b <= 16) go to the sweep-group
// kernel when its layout allows, wider ones to the MFMA chase.
struct StageCtl {
    int* flags;
    int* status;
    uint64_t wait_ticks;
    int max_grid;
    int group_max_b;
    int tri_variant;     // launch shape of the direct band-to-tridiagonal kernel
};
constexpr int DEFAULT_GROUP_MAX_B = 8;
// Bands b <= this (and b in {4, 8, 16}) go straight to the tridiagonal in one
// stage instead of being halved further (0: always halve).  Measured at
// n = 32768: 4 -> 1 direct 129 ms against 4 -> 2 -> 1 138 ms; 8 -> 1 direct
// 237 ms against 238 ms; 16 -> 1 direct 517 ms against 385 ms.
constexpr int DEFAULT_TRIDIAG_FROM_B = 4;
// Built-in next band width from 128, 64 and 32 (the rest halve, and bands
// <= DEFAULT_TRIDIAG_FROM_B go straight to the tridiagonal).  Measured at
// n = 32768 (ms per stage): 128 -> 64 / 32 / 16: 164 / 188 / 283; 64 -> 32 /
// 16 / 8: 70 / 73 / 122; 32 -> 16 / 8: 77 / 117; 16 -> 8: 155; 8 -> 4: 99;
// 4 -> 1: 117.  So 128 -> 64 -> 8 -> 4 -> 1 (502 ms) against 566 ms for
// 128 -> 64 -> 32 -> 8 -> ... and 520 ms for 128 -> 32 -> 8 -> ...
constexpr int DEFAULT_NEXT_FROM_128 = 64;
constexpr int DEFAULT_NEXT_FROM_64 = 8;
constexpr int DEFAULT_NEXT_FROM_32 = 8;
constexpr uint64_t DEFAULT_WAIT_TICKS = 1000000000ull;   // 10 s
// Whether launch_band_halve handles (n, ldband, b).
bool band_halve_supported(int64_t n, int64_t ldband, int b);
void launch_band_halve(int64_t n, double* band, int64_t ldband, int b, bool f32, double* scratch,
                       const StageCtl& ctl, hipStream_t s);
// One reduction b -> h (Algorithm 4.2 with k = b / h): a halving (any kernel
// above), h = 1 (the direct band-to-tridiagonal kernel, ld = 2b + 1) or
// another k on the MFMA chase kernel.  Band ld >= 2b + 1.
bool band_reduce_supported(int64_t n, int64_t ldband, int b, int h);
void launch_band_reduce(int64_t n, double* band, int64_t ldband, int b, int h, bool f32, double* scratch,
                        const StageCtl& ctl, hipStream_t s);
// status[1] |= status[0]; status[0] = 0 (device side, capturable).
void launch_status_rearm(int* status, hipStream_t s);
void launch_fill_int(int* p, int64_t count, int v, hipStream_t s);
// ---- sbr_batched.hip: many matrices (n <= BATCH_NMAX), one work-group each --
constexpr int BATCH_NMAX = 512;
struct BatchDesc {
    double* A;        // n x n, column-major, lda (overwritten)
    int64_t lda;
    double* w;        // n eigenvalues out
    double* bandA;    // n * (2 b0 + 1) doubles: even halving stages
    double* bandB;    // n * (b0 + 1) doubles: odd halving stages
    double* de;       // 2n doubles: d, then e, of the final tridiagonal
    int32_t n;
    int32_t b0;       // initial band (power of two, <= 16; 1 when n <= 2)
};
int64_t batch_scratch_doubles(int grid);
int batch_f2b_grid();
// Every kernel of the batched form, in order, on stream s (capturable: the
// tickets are reset by a kernel).  desc is a device array of count entries,
// ordered by decreasing n; tickets: 8 ints.
// f32: the full-to-band trailing updates on FP32 MFMA (panel QR, T, the
// halvings and the bisection FP64)
void launch_batched(const BatchDesc* desc, int count, int max_b0, bool f32, int* tickets, double* scratch,
                    hipStream_t s);
int init_batched_attributes();

// ---- sbr_chase_mfma.hip: b in {16, 32, 64, 128}, chase products on FP64 MFMA
bool band_mfma_supported(int b);
// b -> h with h = b / k, k a power of two, h >= 8
bool band_reduce_mfma_supported(int b, int h);
int64_t band_mfma_workspace_doubles(int64_t n, int b);
// f32: the WY applications (every product after T is formed) on FP32 MFMA
// with FP32 accumulation; QR, tau, U^T U and T stay FP64
void launch_band_halve_mfma(int64_t n, double* band, int64_t ldband, int b, bool f32, double* scratch,
                            const StageCtl& ctl, hipStream_t s);
void launch_band_reduce_mfma(int64_t n, double* band, int64_t ldband, int b, int h, bool f32, double* scratch,
                             const StageCtl& ctl, hipStream_t s);
int init_band_mfma_attributes();
// ---- sbr_band_tridiag.hip: band b in {4, 8, 16} straight to tridiagonal ----
// (Algorithm 4.2 with k = b).  Band ld = 2b + 1, n (2b + 1) < 2^31.
bool band_tridiag_supported(int b);
int band_tridiag_variants();
void launch_band_tridiag(int64_t n, double* band, int b, const StageCtl& ctl, hipStream_t s);
int init_band_tridiag_attributes();
// ---- sbr_band_group.hip: small bandwidths, sweep groups with LDS windows --
bool band_group_supported(int b);
// band ld = 2b + 1, n (2b + 1) < 2^31
void launch_band_halve_group(int64_t n, double* band, int b, const StageCtl& ctl, hipStream_t s);
int init_band_group_attributes();
void launch_band_to_tridiag(int64_t n, const double* band, int64_t ldband, double* d, double* e,
                            hipStream_t s);

// ---- sbr_bisect.hip -------------------------------------------------------
struct BisectSetup {
    double lo, hi, pivmin;
    double scale;     // power of two putting the interval width in [1/2, 1)
    int iters;
    int nonfinite;    // d or e holds a NaN or an infinity
};
// Doubles of bisection workspace for order n: e^2 (n) and the Sturm counts
// at the 2n points of the shared first grid (2n ints).
inline int64_t bisect_workspace_doubles(int64_t n) { return 2 * n; }
// e may be null when n == 1.  e2p (bisect_workspace_doubles(n)) and setup
// are workspace.
// status: null, or the plan's status word: its STATUS_NONFINITE bit is set
// for a non-finite tridiagonal, and when status[0] is nonzero (a stage of
// the call was abandoned, or the input is not finite) every w is NaN.
void launch_tridiag_eigvals(int64_t n, const double* d, const double* e, double* e2p, BisectSetup* setup,
                            double* w, int* status, hipStream_t s);
// Largest order of the allocation-free tridiagonal entry point.
constexpr int64_t NOALLOC_MAX_N = 1 << 18;
// Device addresses (for `device`, which must be current) of the fixed scratch
// of the allocation-free entry point: e^2 (NOALLOC_MAX_N doubles) and the
// setup record.  Looked up once per device.  0 or a hipError_t.
int noalloc_scratch(int device, double** e2p, BisectSetup** setup);

}  // namespace sbr
