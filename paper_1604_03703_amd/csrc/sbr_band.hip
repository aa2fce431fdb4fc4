// sbr_band.hip -- band-to-band reductions (Algorithm 4.2, b -> h = b / k) and
// the band storage helpers.
//
// Band storage: lower band, column-major by column: band[d + j*ldb] holds
// B(j + d, j).  A stage on bandwidth b needs ldb >= 2b + 1: a chase fills
// entries up to distance 2b - 1 below the diagonal.
//
// One reduction b -> h.  Sweep i (1-based) eliminates columns [(i-1)h, ih)
// below the h-th sub-diagonal and chases the bulge down; chase (i, j) has
//   o = o_qr.r = ih + (j-1)b,
//   QR block  rows [o, o + n_r) x cols [o - h, o) for j = 1, [o - b, o - b + h)
//             for j > 1, n_r = min(n - o, b);
//   update    rows [o, o + n_r) x cols [o, o + 2b) for j = 1 and
//             [o - b + h, o + 2b) for j > 1 (the exact extents; clipped at n);
// with [U, T, R] = QR(block), the block set to [R; 0], W = B[upd, qr] U T,
// V = -W, V[qr rows] += 1/2 U T^T U^T W[qr rows], B[qr, upd] += U V^T and
// B[upd, qr] += V U^T.  Sweep i has chases while o <= n - 2; sweeps run
// while ih <= n - 2.
//
// In lower storage the update splits into the "left" block B[qr, o-b+h:o]
// (j > 1), the diagonal block B[qr, qr] and the "below" block
// B[o+b:o+2b, qr].
//
// The chase kernels themselves are in sbr_chase_mfma.hip (b >= 16, one
// work-group per sweep, products on MFMA, any k with h >= 8),
// sbr_band_group.hip (halvings of b <= 8, a group of consecutive sweeps per
// work-group with the live band in LDS) and sbr_band_tridiag.hip (b <= 16
// straight to the tridiagonal); this file holds the storage kernels and the
// dispatch.
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

// status[1] |= status[0]; status[0] = 0: the flags a call raised move to the
// sticky word the host reads, and the live word the pipelined kernels watch
// starts clear, so one abandoned stage does not stop the sweeps of later calls
__global__ void status_rearm_kernel(int* status) {
    status[1] |= status[0];
    status[0] = 0;
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

int64_t chase_workspace_doubles(int64_t n, int b) { return band_mfma_workspace_doubles(n, b); }

int64_t chase_flag_ints(int64_t n, int b) {
    const int h = b / 2;
    if (h < 1) return 0;
    return (n - 2) / h + 2 > 2 ? (n - 2) / h + 2 : 2;
}

// the small-b group kernel indexes the band with 32-bit integers and expects
// ld = 2b + 1
static bool group_fits(int64_t n, int64_t ldband, int b) {
    return band_group_supported(b) && ldband == 2 * (int64_t)b + 1 && n * ldband < (int64_t)INT32_MAX;
}

bool band_halve_supported(int64_t n, int64_t ldband, int b) {
    return band_mfma_supported(b) || group_fits(n, ldband, b);
}

void launch_band_halve(int64_t n, double* band, int64_t ldband, int b, bool f32, double* scratch,
                       const StageCtl& ctl, hipStream_t s) {
    // f32: the MFMA chase's WY applications on FP32 MFMA; the small-b group
    // kernels (no matrix products) are FP64 in both forms
    const bool group = group_fits(n, ldband, b) && (b <= ctl.group_max_b || !band_mfma_supported(b));
    if (group)
        launch_band_halve_group(n, band, b, ctl, s);
    else if (band_mfma_supported(b))
        launch_band_halve_mfma(n, band, ldband, b, f32, scratch, ctl, s);
}

bool band_reduce_supported(int64_t n, int64_t ldband, int b, int h) {
    if (h < 1 || h >= b || b % h) return false;
    if (2 * h == b) return band_halve_supported(n, ldband, b);
    if (h == 1) return band_tridiag_supported(b) && ldband == 2 * (int64_t)b + 1 && n * ldband < (int64_t)INT32_MAX;
    return band_reduce_mfma_supported(b, h);
}

void launch_band_reduce(int64_t n, double* band, int64_t ldband, int b, int h, bool f32, double* scratch,
                        const StageCtl& ctl, hipStream_t s) {
    if (2 * h == b)
        launch_band_halve(n, band, ldband, b, f32, scratch, ctl, s);
    else if (h == 1)
        launch_band_tridiag(n, band, b, ctl, s);
    else
        launch_band_reduce_mfma(n, band, ldband, b, h, f32, scratch, ctl, s);
}

void launch_fill_int(int* p, int64_t count, int v, hipStream_t s) {
    if (count <= 0) return;
    fill_int_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(p, count, v);
}

void launch_band_to_tridiag(int64_t n, const double* band, int64_t ldband, double* d, double* e, hipStream_t s) {
    if (n <= 0) return;
    band_to_tridiag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, band, ldband, d, e);
}

void launch_status_rearm(int* status, hipStream_t s) { status_rearm_kernel<<<1, 1, 0, s>>>(status); }

}  // namespace sbr
