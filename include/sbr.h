/*
 * sbr.h -- C ABI of the MI355X (gfx950) successive-band-reduction symmetric
 * eigenvalue solver.
 *
 * Method: Solomonik, Ballard, Demmel, Hoefler, "A communication-avoiding
 * parallel algorithm for the symmetric eigenvalue problem".  A dense symmetric
 * matrix is reduced to band form (Algorithm 4.1: panel QR by a TSQR tree,
 * Algorithm 3.2, Householder reconstruction, Corollary 3.7, and the two-sided
 * rank-2b trailing update of Eq. (4.1)); the band is then halved b -> b/2 by
 * bulge chasing (Algorithm 4.2 with k = 2) down to tridiagonal form; the
 * eigenvalues come from Sturm-sequence bisection (the final step of
 * Algorithm 4.3: "compute the eigenvalues of the thin band").
 *
 * Conventions shared by every entry point:
 *  - Matrices are column-major FP64 in DEVICE memory; element (i, j) of A is
 *    A[i + j * lda].  Only the lower triangle (i >= j) is read.
 *  - Calls are asynchronous on the given HIP stream (NULL = legacy default
 *    stream).  Argument errors are detected on the host before anything is
 *    enqueued.  A fault inside a kernel surfaces at the caller's next
 *    synchronisation.
 *  - Return value: 0 on success; -i if the i-th argument is invalid (LAPACK
 *    convention); a positive SBR_E* code otherwise.  sbr_last_hip_error()
 *    returns the hipError_t behind SBR_EHIP.
 *  - Eigenvalues are written to a caller-owned device array in ascending
 *    order.
 */
#ifndef SBR_H
#define SBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* sbr_stream_t;     /* same object as hipStream_t */
typedef struct sbr_plan_s* sbr_plan_t;         /* opaque: workspace + tuning */

typedef enum {
    SBR_FP64 = 0,        /* every step in FP64 */
    SBR_FP32_MFMA = 1    /* full-to-band trailing updates on FP32 MFMA with
                            FP32 accumulation into an FP32 copy of the
                            trailing matrix (n^2 floats of plan workspace;
                            FP64 storage with FP32 products if it cannot be
                            allocated); each panel's column block returns to
                            FP64 before its QR, so the panel QR, Householder
                            norms, R factor and Sturm counts stay FP64.  In
                            the band stages of width b >= 16 the WY
                            applications of every chase (the products after
                            T is formed) run on FP32 MFMA with FP32
                            accumulation; the QR of the bulge, tau and T stay
                            FP64, the band stays FP64 storage.  Bands b <= 8
                            (no matrix products) and the batched kernels
                            compute in FP64 in both forms. */
} sbr_precision;

enum {
    SBR_OK = 0,
    SBR_ENOMEM = 1,      /* device workspace could not be allocated */
    SBR_EHIP = 2,        /* a HIP runtime call failed */
    SBR_ENOTSUP = 3      /* valid but unsupported parameter combination */
};

/*
 * Conditions found on the device while a call runs.  Calls return before the
 * device has done the work, so these are not return codes: they are bits of
 * the plan's status word, read (and cleared) by sbr_plan_status in
 * sbr_stages.h, and every eigenvalue of the affected call is NaN.
 */
enum {
    SBR_STATUS_STALLED = 1,    /* a pipelined band stage stopped waiting for
                                  the previous sweep and was abandoned */
    SBR_STATUS_NONFINITE = 2   /* the tridiagonal reached by the reductions
                                  holds a NaN or an infinity (non-finite
                                  input) */
};

/*
 * Eigenvalues of a dense symmetric matrix (Algorithm 4.3's problem: A in,
 * the eigenvalue vector D out), plain FP64 form.
 *   n      order of A, n >= 0.
 *   A      device pointer, n x n, lda >= max(1, n); lower triangle read.
 *          OVERWRITTEN: on return it holds no meaningful values.
 *   lda    leading dimension of A.
 *   b0     band width of the full-to-band stage: a power of two with
 *          2 <= b0 <= 128, or 0 to pick it from n.  Any n is allowed (no
 *          divisibility by b0 is required).
 *   stream HIP stream all work is enqueued on.
 *   w      device pointer, n doubles: the eigenvalues, ascending.
 * Uses an internal plan cached per device (allocates on first use and when
 * n or b0 grows).
 */
int sbr_syev_eigvals(int64_t n, double* A, int64_t lda, int32_t b0,
                     sbr_stream_t stream, double* w);

/* As sbr_syev_eigvals, with an explicit plan and precision form.  Once the
 * plan holds workspace for (n, b0, prec) the call allocates nothing and does
 * not wait for the device, so it can be captured in a HIP graph; a plan is
 * not safe for calls that overlap (on two streams or two threads). */
int sbr_syev_eigvals_ex(sbr_plan_t plan, int64_t n, double* A, int64_t lda,
                        int32_t b0, sbr_precision prec, sbr_stream_t stream,
                        double* w);

/*
 * Eigenvalues of `batch` independent symmetric matrices of different orders
 * (the sequence of matrices of a self-consistent-field loop, Section 1).
 *   n, lda   HOST arrays of length batch (n[k] >= 1, lda[k] >= n[k]).
 *   A        HOST array of batch DEVICE pointers (each overwritten).
 *   b0       band width for every matrix, or 0 for the tuned choice per size.
 *   w        HOST array of batch DEVICE pointers, w[k] holds n[k] doubles.
 * Matrices with n[k] <= 512 (and b0 <= 16) are reduced by the batched
 * kernels, one work-group per matrix, largest first: full-to-band with
 * panels of width b (when b0 = 0: the plan's band table, see
 * sbr_plan_set_batch_bands, else 8 for n <= 96 and 16 above), the halvings
 * b -> 1 and bisection.  Their launch sequence is captured once per batch
 * shape (the pointers, orders and bands) and replayed by later calls with the
 * same shape; a new shape uploads the descriptors and captures again (the
 * host then waits for the previous upload).  Larger matrices, or b0 >= 32,
 * go through sbr_syev_eigvals_ex one after another on the same stream.  The
 * per-matrix band buffers grow on demand (allocation on the first call of a
 * larger batch).  prec = SBR_FP32_MFMA: the batched full-to-band runs
 * its trailing updates (W = A22 U T, U^T W, V and A22 += U V^T + V U^T) on
 * FP32 MFMA with FP32 accumulation, added into the FP64 matrix; its panel QR,
 * tau and T, the halvings and the bisection stay FP64.  prec also applies to
 * the matrices that go through sbr_syev_eigvals_ex.
 */
int sbr_syev_eigvals_batched(sbr_plan_t plan, int32_t batch, const int64_t* n,
                             double* const* A, const int64_t* lda, int32_t b0,
                             sbr_precision prec, sbr_stream_t stream,
                             double* const* w);

/*
 * Band per size bucket for the batched form with b0 = 0 (the tuned choice):
 * a matrix of order n gets bands[q] for the first q with n <= n_max[q]
 * (n_max ascending, bands powers of two <= 16), the built-in rule (8 up to
 * n = 96, 16 above) beyond the last bucket; nbuckets = 0 restores the
 * built-in rule.  Host-side only (the next batched call captures its launch
 * again when a band changes).  -3 / -4 for a malformed table.
 */
int sbr_plan_set_batch_bands(sbr_plan_t plan, int32_t nbuckets, const int32_t* n_max,
                             const int32_t* bands);

/*
 * Eigenvalues of the symmetric tridiagonal matrix with diagonal d[0..n-1]
 * and off-diagonal e[0..n-2] (device pointers; e may be NULL when n == 1),
 * by Sturm-sequence bisection; w (device, n doubles) ascending, every entry
 * NaN if d or e holds a NaN or an infinity.  SBR_ENOTSUP for n >= 2^31 (the
 * Sturm counts are 32-bit).
 */
int sbr_tridiag_eigvals(int64_t n, const double* d, const double* e,
                        sbr_stream_t stream, double* w);

/*
 * sbr_tridiag_eigvals without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels and results as
 * sbr_tridiag_eigvals; its scratch (e^2, the Sturm counts of the first grid
 * and the bisection setup, about 4 MiB) is a fixed array in the library's device image, one per GPU, held
 * until the process ends.  n <= 262144 (2^18), else SBR_ENOTSUP before
 * anything is enqueued.  All calls on one GPU share that array: calls that
 * overlap on one GPU (concurrent streams or threads) race and must be
 * serialised by the caller.
 */
int sbr_tridiag_eigvals_noalloc(int64_t n, const double* d, const double* e,
                                sbr_stream_t stream, double* w);

/* Plan owning the device workspace for problems up to n_max (and batches up
 * to batch_max matrices).  Creating a plan allocates; calls made through an
 * existing plan within its limits do not. */
int sbr_plan_create(sbr_plan_t* plan, int64_t n_max, int32_t batch_max,
                    sbr_precision prec);
/* Waits for the device (work enqueued with the plan may still run), then
 * frees the plan's memory, streams, events and captured launches. */
int sbr_plan_destroy(sbr_plan_t plan);

/* Device workspace bytes sbr_syev_eigvals_ex needs for (n, b0, prec). */
int sbr_workspace_size(int64_t n, int32_t b0, sbr_precision prec, size_t* bytes);

/* Band width chosen for order n when b0 = 0 is passed. */
int32_t sbr_default_band(int64_t n);

/* hipError_t of the last SBR_EHIP failure on the calling thread. */
int sbr_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SBR_H */
