/*
 * oracle.c -- FP64 CPU oracle for the symmetric eigenvalue problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may link, load or call this file; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
 * with the GPU path.
 *
 * What it computes: the sorted eigenvalues of a dense symmetric matrix, which
 * is exactly what the successive-band-reduction eigensolver returns (its
 * full-to-band and band-to-band stages are orthogonal similarity transforms,
 * Section 4, Algorithms 4.1-4.3, so they preserve the spectrum).  The route is
 * deliberately a different one from the GPU path:
 *
 *  1. unblocked Householder reduction straight to tridiagonal form -- the
 *     direct b = 1 reduction of Section 4 that the paper contrasts with
 *     successive band reduction (each column needs one product with the
 *     trailing matrix); one reflector at a time, Eq. (4.1) with U = v, T = tau;
 *  2. Sturm-sequence bisection on the tridiagonal (d, e) for every index,
 *     with Kahan's zero-pivot guard (pivmin) so the count stays monotone.
 *
 * Pins (tests/test_oracle_pins.py): Toeplitz closed form 2cos(k pi/(n+1)),
 * prescribed spectra Q diag(lam) Q^T, trace / Frobenius invariance of (d, e),
 * brute-force cyclic Jacobi for n <= 16, LAPACK (numpy / scipy) cross-checks.
 *
 * Storage: column-major, A[i + j*lda]; only the lower triangle is read.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(A, lda, i, j) (A)[(size_t)(i) + (size_t)(j) * (size_t)(lda)]

static double now_seconds(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Euclidean norm with scaling (no overflow / underflow of the squares). */
static double scaled_norm(int64_t m, const double* x) {
    double scale = 0.0, ssq = 1.0;
    for (int64_t i = 0; i < m; ++i) {
        double a = fabs(x[i]);
        if (a == 0.0) continue;
        if (scale < a) {
            ssq = 1.0 + ssq * (scale / a) * (scale / a);
            scale = a;
        } else {
            ssq += (a / scale) * (a / scale);
        }
    }
    return scale * sqrt(ssq);
}

/*
 * Householder tridiagonalisation of the n x n symmetric matrix held in the
 * lower triangle of A (overwritten).  Outputs d[0..n-1] (diagonal) and
 * e[0..n-2] (sub-diagonal).
 *
 * For column j: x = A[j+1:n, j]; alpha = -sgn(x_0) |x| (sgn(0) = +1);
 * v = x - alpha e_0; tau = 2 / (v^T v); then with X = A[j+1:n, j+1:n]:
 * p = tau X v, w = p - (tau/2)(p^T v) v, X <- X - v w^T - w v^T, which is
 * (I - tau v v^T) X (I - tau v v^T) written as a symmetric rank-2 update
 * (Eq. (4.1) with a single reflector).  If x_1.. are already zero, no
 * reflector is applied and e_j = x_0.
 */
int oracle_tridiagonalize(int64_t n, double* A, int64_t lda, double* d, double* e) {
    if (n < 0 || lda < (n > 1 ? n : 1) || (n > 0 && (!A || !d)) || (n > 1 && !e)) return -1;
    if (n == 0) return 0;
    double* v = (double*)malloc(sizeof(double) * (size_t)n);
    double* p = (double*)malloc(sizeof(double) * (size_t)n);
    if (!v || !p) { free(v); free(p); return -2; }
    for (int64_t j = 0; j + 2 < n; ++j) {
        const int64_t m = n - j - 1;          /* length of x */
        double* x = &AT(A, lda, j + 1, j);
        double tail = scaled_norm(m - 1, x + 1);
        d[j] = AT(A, lda, j, j);
        if (tail == 0.0) {                    /* already reduced */
            e[j] = x[0];
            continue;
        }
        double xn = hypot(x[0], tail);
        double alpha = (x[0] >= 0.0) ? -xn : xn;
        v[0] = x[0] - alpha;
        for (int64_t i = 1; i < m; ++i) v[i] = x[i];
        double vtv = v[0] * v[0];
        for (int64_t i = 1; i < m; ++i) vtv += v[i] * v[i];
        double tau = 2.0 / vtv;
        e[j] = alpha;
        x[0] = alpha;
        for (int64_t i = 1; i < m; ++i) x[i] = 0.0;

        double* X = &AT(A, lda, j + 1, j + 1);
        /* p = tau * X v, X symmetric stored lower: column sweep, private sums */
        memset(p, 0, sizeof(double) * (size_t)m);
#pragma omp parallel
        {
            double* pl = (double*)calloc((size_t)m, sizeof(double));
#pragma omp for schedule(dynamic, 32)
            for (int64_t k = 0; k < m; ++k) {
                const double* col = X + (size_t)k * (size_t)lda;
                double s = col[k] * v[k];
                const double vk = v[k];
                for (int64_t i = k + 1; i < m; ++i) {
                    s += col[i] * v[i];
                    pl[i] += col[i] * vk;
                }
                pl[k] += s;
            }
#pragma omp critical
            for (int64_t i = 0; i < m; ++i) p[i] += pl[i];
            free(pl);
        }
        double ptv = 0.0;
        for (int64_t i = 0; i < m; ++i) { p[i] *= tau; ptv += p[i] * v[i]; }
        const double c = 0.5 * tau * ptv;
        for (int64_t i = 0; i < m; ++i) p[i] -= c * v[i];      /* p is now w */
#pragma omp parallel for schedule(dynamic, 32)
        for (int64_t k = 0; k < m; ++k) {
            double* col = X + (size_t)k * (size_t)lda;
            const double vk = v[k], wk = p[k];
            for (int64_t i = k; i < m; ++i) col[i] -= v[i] * wk + p[i] * vk;
        }
    }
    if (n >= 2) {
        d[n - 2] = AT(A, lda, n - 2, n - 2);
        e[n - 2] = AT(A, lda, n - 1, n - 2);
    }
    d[n - 1] = AT(A, lda, n - 1, n - 1);
    free(v);
    free(p);
    return 0;
}

/* Safe minimum pivot: smallest normal number scaled by max(1, max e_i^2). */
double oracle_pivmin(int64_t n, const double* e) {
    double emax2 = 1.0;
    for (int64_t i = 0; i + 1 < n; ++i) {
        double t = e[i] * e[i];
        if (t > emax2) emax2 = t;
    }
    return DBL_MIN * emax2;
}

/*
 * Sturm count: number of negative pivots of T - x I, i.e. (with the guard)
 * the number of eigenvalues below x.  q_0 = d_0 - x,
 * q_i = (d_i - x) - e_{i-1}^2 / q_{i-1}; a pivot with |q| < pivmin is replaced
 * by -pivmin (Kahan; keeps the count monotone in x).
 */
int64_t oracle_sturm_count(int64_t n, const double* d, const double* e, double x, double pivmin) {
    if (n <= 0) return 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int64_t cnt = (q < 0.0);
    for (int64_t i = 1; i < n; ++i) {
        q = (d[i] - x) - (e[i - 1] * e[i - 1]) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

/*
 * Gershgorin interval of the tridiagonal, widened as in LAPACK's bisection
 * (2.1 * (n eps |T| + 2 pivmin)), and the fixed iteration count
 * I = ceil(log2((hi - lo) / (eps * max(|lo|, |hi|)))) + 2.
 */
int oracle_bisect_setup(int64_t n, const double* d, const double* e,
                        double* lo_out, double* hi_out, double* pivmin_out, int* iters_out) {
    if (n <= 0) return -1;
    double lo = d[0], hi = d[0];
    for (int64_t i = 0; i < n; ++i) {
        double r = 0.0;
        if (i > 0) r += fabs(e[i - 1]);
        if (i + 1 < n) r += fabs(e[i]);
        if (d[i] - r < lo) lo = d[i] - r;
        if (d[i] + r > hi) hi = d[i] + r;
    }
    double pivmin = oracle_pivmin(n, e);
    double tnorm = fmax(fabs(lo), fabs(hi));
    const double eps = DBL_EPSILON * 0.5;
    const double fudge = 2.1;
    lo -= fudge * ((double)n * eps * tnorm + 2.0 * pivmin);
    hi += fudge * ((double)n * eps * tnorm + 2.0 * pivmin);
    tnorm = fmax(fabs(lo), fabs(hi));
    int iters = 0;
    if (hi > lo && tnorm > 0.0) {
        iters = (int)ceil(log2((hi - lo) / (eps * tnorm))) + 2;
        if (iters < 0) iters = 0;
    }
    *lo_out = lo;
    *hi_out = hi;
    *pivmin_out = pivmin;
    *iters_out = iters;
    return 0;
}

/* All n eigenvalues of tridiag(e, d, e), ascending, by bisection per index. */
int oracle_bisect_all(int64_t n, const double* d, const double* e, double* w) {
    if (n < 0 || (n > 0 && (!d || !w))) return -1;
    if (n == 0) return 0;
    double lo, hi, pivmin;
    int iters;
    oracle_bisect_setup(n, d, e, &lo, &hi, &pivmin, &iters);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 1; k <= n; ++k) {
        double a = lo, c = hi;
        for (int it = 0; it < iters; ++it) {
            double mid = a + 0.5 * (c - a);
            if (mid == a || mid == c) break;
            if (oracle_sturm_count(n, d, e, mid, pivmin) >= k) c = mid; else a = mid;
        }
        w[k - 1] = a + 0.5 * (c - a);
    }
    return 0;
}

/*
 * Eigenvalues of the dense symmetric matrix (lower triangle of A read; A is
 * not modified -- a private copy is reduced).  seconds[0] receives the time of
 * the tridiagonalisation, seconds[1] that of the bisection (may be NULL).
 */
int oracle_eigvalsh(int64_t n, const double* A, int64_t lda, double* w, double* seconds) {
    if (n < 0 || lda < (n > 1 ? n : 1) || (n > 0 && (!A || !w))) return -1;
    if (n == 0) return 0;
    double* C = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double* d = (double*)malloc(sizeof(double) * (size_t)n);
    double* e = (double*)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    if (!C || !d || !e) { free(C); free(d); free(e); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i < n; ++i) C[(size_t)i + (size_t)j * (size_t)n] = AT(A, lda, i, j);
    double t0 = now_seconds();
    int rc = oracle_tridiagonalize(n, C, n, d, e);
    double t1 = now_seconds();
    if (rc == 0) rc = oracle_bisect_all(n, d, e, w);
    double t2 = now_seconds();
    if (seconds) { seconds[0] = t1 - t0; seconds[1] = t2 - t1; }
    free(C); free(d); free(e);
    return rc;
}
