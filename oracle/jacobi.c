/*
 * Test infrastructure only -- the CPU oracle for singular values.
 *
 * Only the test suite, the smoke check and the bench's cpu_baseline leg load
 * this file's library; the GPU product path never links or calls it.
 *
 * What it computes: the singular values of a dense real matrix, in float64,
 * by one-sided (Hestenes) Jacobi.  The paper's method (two-stage reduction:
 * dense -> band -> bidiagonal -> diagonal, Section "Algorithm" of the
 * evaluation, Algorithm 1) only applies orthogonal transformations, which
 * leave the singular values unchanged; so the plain definition of its result
 * is the multiset of singular values of A, and that is what this file
 * computes, without any tiling, band form or bulge chasing.
 *
 * Method (Hestenes 1958; accuracy: Demmel & Veselic 1992):
 *   1. W = A (or A^T if m < n), column-major, float64.
 *   2. Scale W by 2^e so that max|w| lies in [0.5, 1): exact.
 *   3. Repeat sweeps (at most max_sweeps).  A sweep is n'-1 rounds of a
 *      round-robin tournament over the columns (n' = n rounded up to even,
 *      the extra index is a dummy); each round has n'/2 disjoint pairs.
 *      For a pair (p, q): alpha = |w_p|^2, beta = |w_q|^2, gamma = w_p.w_q.
 *      If |gamma| > tol*sqrt(alpha)*sqrt(beta), rotate the two columns by
 *      the plane rotation that makes them orthogonal.
 *   4. Stop after a sweep with no rotation.
 *   5. sigma_j = |w_j| * 2^-e, sorted descending; return min(m, n) values.
 *
 * Each pair is handled start-to-finish by one thread with sums in a fixed
 * order, so the result is bitwise independent of the OpenMP thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Return codes. */
#define ORACLE_OK 0
#define ORACLE_BAD_ARG -1
#define ORACLE_NONFINITE -2
#define ORACLE_NO_CONVERGENCE -3
#define ORACLE_NO_MEMORY -4

static int cmp_desc(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* Rotate one pair; returns 1 if a rotation was applied. */
static int jacobi_pair(double *W, int64_t m, int64_t p, int64_t q, double tol, double *offmax) {
    double *wp = W + p * m, *wq = W + q * m;
    double alpha = 0.0, beta = 0.0, gamma = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        alpha += wp[i] * wp[i];
        beta += wq[i] * wq[i];
        gamma += wp[i] * wq[i];
    }
    *offmax = 0.0;
    if (alpha == 0.0 || beta == 0.0) return 0;
    double scale = sqrt(alpha) * sqrt(beta);
    double rel = fabs(gamma) / scale;
    *offmax = rel;
    if (fabs(gamma) <= tol * scale) return 0;
    /* t solves t^2 + 2 zeta t - 1 = 0 (smaller root): columns become orthogonal. */
    double zeta = (beta - alpha) / (2.0 * gamma);
    double t;
    if (fabs(zeta) > 1e150) {
        t = 1.0 / (2.0 * zeta);
    } else {
        double sg = zeta >= 0.0 ? 1.0 : -1.0;
        t = sg / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    }
    double c = 1.0 / sqrt(1.0 + t * t);
    double s = c * t;
    for (int64_t i = 0; i < m; ++i) {
        double x = wp[i], y = wq[i];
        wp[i] = c * x - s * y;
        wq[i] = s * x + c * y;
    }
    return 1;
}

/*
 * oracle_svd_values: singular values of the m x n column-major float64 matrix
 * A (leading dimension lda >= max(1, m)), written descending into S[min(m,n)].
 * nthreads <= 0 uses the OpenMP default.  sweeps_out (may be NULL) receives the
 * number of sweeps; offmax_out (may be NULL) the largest |gamma|/sqrt(alpha beta)
 * seen in the last sweep.
 */
int oracle_svd_values(const double *A, int64_t m, int64_t n, int64_t lda, double *S,
                      int max_sweeps, int nthreads, int *sweeps_out, double *offmax_out) {
    if (m < 0 || n < 0) return ORACLE_BAD_ARG;
    int64_t k = m < n ? m : n;
    if (k == 0) return ORACLE_OK;
    if (!A || !S || lda < (m > 1 ? m : 1)) return ORACLE_BAD_ARG;
    int transpose = m < n;
    int64_t M = transpose ? n : m, N = transpose ? m : n;
    double *W = (double *)malloc(sizeof(double) * (size_t)M * (size_t)N);
    if (!W) return ORACLE_NO_MEMORY;
    double amax = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double v = A[i + j * lda];
            if (!isfinite(v)) { free(W); return ORACLE_NONFINITE; }
            if (fabs(v) > amax) amax = fabs(v);
            if (transpose) W[j + i * M] = v; else W[i + j * M] = v;
        }
    if (amax == 0.0) {
        for (int64_t j = 0; j < k; ++j) S[j] = 0.0;
        free(W);
        return ORACLE_OK;
    }
    int e;
    frexp(amax, &e); /* amax = f * 2^e, f in [0.5, 1) */
    for (int64_t i = 0; i < M * N; ++i) W[i] = ldexp(W[i], -e);

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double tol = sqrt((double)M) * ldexp(1.0, -53);
    int64_t Np = N + (N & 1); /* players incl. dummy */
    int64_t npairs = Np / 2;
    int sweep = 0, converged = 0;
    double last_off = 0.0;
    if (N == 1) converged = 1;
    while (!converged && sweep < max_sweeps) {
        int64_t rotations = 0;
        double sweep_off = 0.0;
        for (int64_t r = 0; r < Np - 1; ++r) {
            /* Circle method: index Np-1 is fixed, the others rotate. */
#pragma omp parallel for schedule(static) reduction(+ : rotations) reduction(max : sweep_off)
            for (int64_t i = 0; i < npairs; ++i) {
                int64_t p, q;
                if (i == 0) {
                    p = r;
                    q = Np - 1;
                } else {
                    p = (r + i) % (Np - 1);
                    q = (r - i + (Np - 1)) % (Np - 1);
                }
                if (p >= N || q >= N) continue;
                if (p > q) { int64_t t = p; p = q; q = t; }
                double off;
                rotations += jacobi_pair(W, M, p, q, tol, &off);
                if (off > sweep_off) sweep_off = off;
            }
        }
        ++sweep;
        last_off = sweep_off;
        if (rotations == 0) converged = 1;
    }
    if (sweeps_out) *sweeps_out = sweep;
    if (offmax_out) *offmax_out = last_off;
    if (!converged) { free(W); return ORACLE_NO_CONVERGENCE; }
    double *sv = (double *)malloc(sizeof(double) * (size_t)N);
    if (!sv) { free(W); return ORACLE_NO_MEMORY; }
    for (int64_t j = 0; j < N; ++j) {
        double acc = 0.0;
        const double *w = W + j * M;
        for (int64_t i = 0; i < M; ++i) acc += w[i] * w[i];
        sv[j] = ldexp(sqrt(acc), e);
    }
    qsort(sv, (size_t)N, sizeof(double), cmp_desc);
    for (int64_t j = 0; j < k; ++j) S[j] = sv[j];
    free(sv);
    free(W);
    return ORACLE_OK;
}
