/*
 * sbr_stages.h -- stage-level entry points of the SBR eigensolver library.
 *
 * These expose the individual steps of the hot path (for component tests and
 * per-phase measurement).  Conventions are those of sbr.h: FP64 device
 * buffers, column-major, asynchronous on `stream`, 0 / -i / SBR_E* returns.
 */
#ifndef SBR_STAGES_H
#define SBR_STAGES_H

#include "sbr.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Full-to-band reduction (Algorithm 4.1, right-looking: every panel's
 * two-sided update, Eq. (4.1), is applied to the whole trailing matrix).
 * A (n x n, lower triangle) is overwritten: on return A[i + j*lda] for
 * 0 <= i - j <= b holds the band matrix with the eigenvalues of the input,
 * and A[i + j*lda] = 0 for i - j > b.  The strict upper triangle is scratch.
 * b: power of two, 2 <= b <= 128.  SBR_ENOTSUP when (n + 128 lda) * 8
 * reaches 2^31 (the symmetric products' 32-bit offsets; lda beyond ~2^20).
 */
int sbr_full_to_band(sbr_plan_t plan, int64_t n, double* A, int64_t lda,
                     int32_t b, sbr_precision prec, sbr_stream_t stream);

/*
 * Copy the lower band of a dense matrix into band storage:
 * band[d + j*ldband] = A[(j+d) + j*lda] for 0 <= d <= b and j + d < n,
 * and 0 for every other d < ldband.  Requires ldband >= b + 1.
 */
int sbr_dense_to_band(int64_t n, const double* A, int64_t lda, int32_t b,
                      double* band, int64_t ldband, sbr_stream_t stream);

/*
 * One band-to-band halving (Algorithm 4.2 with k = 2): the symmetric band
 * matrix of bandwidth b held in `band` (lower band storage as above, with
 * ldband >= 2b + 1 because the chase fills up to distance 2b - 1; the rows
 * at distances b+1 .. 2b must hold zeros on entry, as sbr_dense_to_band
 * leaves them) is reduced in place to bandwidth b/2.  On return the entries
 * at distance > b/2 are exactly zero.  b: power of two, 2 <= b <= 128.
 * prec = SBR_FP32_MFMA: for b >= 16 the WY applications of every chase
 * run on FP32 MFMA with FP32 accumulation (QR, tau and T in FP64); b <= 8
 * is FP64 in both forms.  For b <= 8 with
 * ldband != 2b + 1 the band goes through the plan's band buffer (two
 * copies).  SBR_ENOTSUP for n >= 2^31.
 */
int sbr_band_halve(sbr_plan_t plan, int64_t n, double* band, int64_t ldband,
                   int32_t b, sbr_precision prec, sbr_stream_t stream);

/*
 * Band of width b straight to tridiagonal form (Algorithm 4.2 with k = b,
 * i.e. h = 1: every chase is one Householder reflector of length b).  Same
 * storage conventions as sbr_band_halve (ldband >= 2b + 1, rows b+1 .. 2b
 * zero on entry); on return the entries at distance > 1 are exactly zero.
 * b in {4, 8, 16} (-5 otherwise); FP64.  SBR_ENOTSUP when n (2b + 1) reaches
 * 2^31.
 */
int sbr_band_to_tridiag(sbr_plan_t plan, int64_t n, double* band, int64_t ldband, int32_t b,
                        sbr_stream_t stream);

/*
 * One band-to-band reduction b -> h (Algorithm 4.2 with k = b / h, Section
 * 4.2): same storage conventions as sbr_band_halve (ldband >= 2b + 1, rows
 * b+1 .. 2b zero on entry); on return the entries at distance > h are
 * exactly zero.  Kernels exist for h = b/2 (as sbr_band_halve), for h = 1
 * with b in {4, 8, 16} (as sbr_band_to_tridiag) and for b in {16, 32, 64, 128}
 * with h = b/k >= 8 (one work-group per sweep, chase products on MFMA);
 * -5 for any other (b, h).  Every sweep eliminates h columns, so a stage with
 * k > 2 does in one pipeline what log2(k) halvings do in several.  prec as
 * for sbr_band_halve (h = 1 is FP64 in both forms).  SBR_ENOTSUP for n >= 2^31, and for h = 1 when
 * n (2b + 1) reaches 2^31.
 */
int sbr_band_reduce(sbr_plan_t plan, int64_t n, double* band, int64_t ldband, int32_t b, int32_t h,
                    sbr_precision prec, sbr_stream_t stream);

/*
 * Panel QR of the m x b panel P (m >= b) by the TSQR tree of Algorithm 3.2
 * followed by Householder reconstruction (Corollary 3.7).  Outputs (device):
 *   Q  m x b explicit orthonormal factor (ld = m), P = Q R,
 *   R  b x b upper triangular (ld = b),
 *   U  m x b, unit lower trapezoidal (ld = m), T b x b upper (ld = b),
 *   S  b signs with (I - U T U^T)[:, :b] = Q diag(S).
 * P is left unchanged.
 */
int sbr_panel_qr(sbr_plan_t plan, int64_t m, int32_t b, const double* P,
                 int64_t ldp, double* Q, double* R, double* U, double* T,
                 double* S, sbr_stream_t stream);

/* C = alpha op(A) op(B) + beta C on the MFMA tile engine (transa/transb:
 * 0 = N, 1 = T); prec chooses FP64 or FP32-MFMA arithmetic. */
int sbr_gemm(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
             double alpha, const double* A, int64_t lda, const double* B,
             int64_t ldb, double beta, double* C, int64_t ldc,
             sbr_precision prec, sbr_stream_t stream);

/* Lower triangle of C += U V^T + V U^T (C m x m, U and V m x k). */
int sbr_syr2k_lower(int64_t m, int64_t k, const double* U, int64_t ldu,
                    const double* V, int64_t ldv, double* C, int64_t ldc,
                    sbr_precision prec, sbr_stream_t stream);

/* W = A Y with A symmetric (m x m, lower triangle read), Y m x k.
 * The kernel addresses A and Y with 32-bit byte offsets: returns
 * SBR_ENOTSUP when (m + 128 lda) * 8 or (16 + 127 ldy) * 8 reaches 2^31
 * (leading dimensions beyond about 2^20). */
int sbr_symm_lower(int64_t m, int64_t k, const double* A, int64_t lda,
                   const double* Y, int64_t ldy, double* W, int64_t ldw,
                   sbr_precision prec, sbr_stream_t stream);

/* Per-phase timing of the last call made through `plan` with timing enabled
 * (hipEvents recorded on the call's stream; reading them synchronises). */
typedef struct {
    double ms_total;          /* whole call */
    double ms_f2b;            /* full-to-band */
    double ms_band;           /* all band-to-band halvings */
    double ms_bisect;         /* tridiagonal extraction + bisection */
    double ms_update_kernels; /* sum over launches of the SYMM + SYR2K kernels */
    int64_t update_launches;  /* number of those launches */
    double ms_syr2k;          /* bulk SYR2K launches only: the trailing update
                                 minus the next panel's column block */
    int64_t syr2k_launches;
    double ms_symm;           /* SYMM launches only */
    int64_t symm_launches;
    double ms_stage[8];       /* per band-to-band stage, in order (the widths
                                 come from sbr_plan_get_band_stages) */
    int32_t n_stages;
    double ms_syr2k_big;      /* the bulk SYR2K launches on 128 x 128 tiles
                                 (the first ones; the last, small trailing
                                 matrices use 64 x 64 tiles) */
    int64_t syr2k_big_launches;
} sbr_timing;

/* enable: 0 off; 1 every pair above; 2 the phase totals and the bulk SYR2K
 * launches only (no events around the SYMM launches, which sit on the
 * full-to-band critical path: each recorded event costs the stream a few
 * microseconds); ms_symm and symm_launches are then 0. */
int sbr_plan_set_timing(sbr_plan_t plan, int enable);

/* Cap on the number of work-groups of the pipelined band-to-band kernels
 * (0 = automatic).  With 1, a halving b >= 16 runs its chases one at a time
 * in the sequential (sweep-major) order of Algorithm 4.2, and a halving
 * b <= 8 runs its groups of consecutive sweeps one after another (inside a
 * group the sweeps still advance in lock step, a fixed lag apart).  The
 * result is bitwise the same at any cap: every chase does the same
 * arithmetic on the same data. */
int sbr_plan_set_chase_blocks(sbr_plan_t plan, int32_t max_blocks);

/* Bandwidths b <= this value (at most 16) are halved by the sweep-group
 * kernel (bulges in registers, live band in LDS), wider ones by the MFMA
 * chase kernel (default 8). */
int sbr_plan_set_group_max_band(sbr_plan_t plan, int32_t b);

/* In a solve, bands b <= this value (b in {4, 8, 16}) are reduced straight
 * to the tridiagonal by one stage of sbr_band_to_tridiag's kind instead of
 * further halvings (0: halve down to 1; the default is 4).  variant (0 .. 2) picks the launch
 * shape of that kernel (lanes per sweep, sweeps per work-group) for it and
 * for sbr_band_to_tridiag; 0 is the default.  -3 for an unknown variant. */
int sbr_plan_set_tridiag_band(sbr_plan_t plan, int32_t b, int32_t variant);

/* Band widths of a solve's band-to-band stages (Algorithm 4.3 leaves the
 * choice of k per stage to the machine): widths[0 .. count) strictly
 * decreasing powers of two.  From the current width b a solve goes to the
 * largest listed width below b that sbr_band_reduce takes for b (halving when
 * none does), and it ends with a width of 1.  count = 0 restores the built-in
 * sequence (chosen by measurement on gfx950).  -2 for a bad count, -3 for a
 * list that is not strictly decreasing powers of two >= 1. */
int sbr_plan_set_band_stages(sbr_plan_t plan, int32_t count, const int32_t* widths);

/* The band widths after each band-to-band stage of a solve of order n from
 * band b0 with the plan's current settings (at most cap of them written to
 * widths); returns the number of stages or a negative argument error. */
int sbr_plan_get_band_stages(sbr_plan_t plan, int64_t n, int32_t b0, int32_t* widths, int32_t cap);

/* How long (ticks of the 100 MHz device clock) a pipelined band kernel waits
 * for the previous sweep before it abandons the stage and raises
 * SBR_STATUS_STALLED (0 = the default, 10^9 ticks = 10 s).  The schedule
 * always makes progress, so the limit only bounds a kernel's lifetime; a
 * tiny limit forces the abandon path from the host (for tests). */
int sbr_plan_set_wait_limit(sbr_plan_t plan, int64_t ticks);

/* CUs kept free of the bulk trailing-update launches of the full-to-band
 * stage (default 32; 0 = none).  The next panel is factored concurrently on
 * another stream (Section 4 lookahead); a trailing-update grid that covers the
 * whole chip would hold every CU until it drains, so the bulk launch goes to
 * a stream restricted to the other CUs (CUs 0 .. cus-1 of the logical
 * numbering, which interleaves the XCDs, are left out) and the panel kernels
 * start at once.  Synchronises the device when the
 * value changes.  Returns 0, -1 (null plan), -2 (cus < 0) or SBR_EHIP.  Where
 * CU-masked streams are unavailable the setting has no effect. */
int sbr_plan_set_panel_cus(sbr_plan_t plan, int32_t cus);

/* Number of consecutive full-to-band panels whose two-sided updates are
 * aggregated before one trailing update (default 1).  Section 4, Eq. (4.2):
 * the update X + U V^T + V U^T need not be applied before the next panel,
 * since the product that panel needs is (X + U V^T + V U^T) Y =
 * X Y + U (V^T Y) + V (U^T Y).  With depth D, the panels of a group take
 * their W = A22 Y from the matrix as it stood at the start of the group plus
 * those skinny corrections, each next panel's columns get the pending
 * updates before its factorization, and one SYR2K of rank 2 D b per group
 * updates the trailing matrix (the next group's first panel is factored
 * beside it, as with depth 1).  Applies to the FP64 form (the FP32-MFMA form
 * keeps depth 1).  Depth > 1 allocates 4 n_max D b + 2 D b^2 doubles of
 * aggregation buffers, here for the plan's current size and again when a
 * larger problem grows the plan.  Returns 0, -1 (null plan), -2 (depth
 * outside 1 .. 4) or SBR_ENOMEM. */
int sbr_plan_set_update_depth(sbr_plan_t plan, int32_t depth);

/* Blocking (waits for the device): the SBR_STATUS_* bits raised by the calls
 * made through the plan since the previous sbr_plan_status, then clears
 * them.  Every call starts with a clear live word, so a stage abandoned by
 * one call does not affect the next; the eigenvalues of a call that raised
 * a bit are NaN. */
int sbr_plan_status(sbr_plan_t plan, int32_t* status);
int sbr_plan_get_timing(sbr_plan_t plan, sbr_timing* out);

#ifdef __cplusplus
}
#endif

#endif /* SBR_STAGES_H */
