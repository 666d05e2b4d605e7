/*
 * FP64 CPU oracle: one-sided (Hestenes) Jacobi SVD.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * What it computes.  The soft-thresholding operator of the paper (section 2,
 * Eq. (1)) is defined through the SVD A = U Sigma V^T.  This file produces
 * that SVD the slow, obviously correct way: rotate pairs of columns of a
 * working copy W = A until every pair is orthogonal (to a relative tolerance),
 * accumulating the same rotations into V.  Then sigma_j = ||w_j||,
 * u_j = w_j / sigma_j, and A = U diag(sigma) V^T.  The thresholding itself
 * (Eq. (1)), the polar factors (section 2) and the rank-r truncation
 * (Corollary 1) are formed from these factors by the Python wrapper.
 *
 * Pair order: round-robin ("circle method") tournament, so that the n/2
 * pairs of one round touch disjoint columns and may be rotated in parallel
 * (OpenMP).  Any cyclic order converges; the order changes only rounding.
 *
 * Rotation for a pair (p, q) with alpha = w_p.w_p, beta = w_q.w_q,
 * gamma = w_p.w_q:  zeta = (beta - alpha) / (2 gamma),
 * t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1+t^2), s = c t,
 * (w_p, w_q) <- (c w_p - s w_q, s w_p + c w_q).  This is the rotation that
 * makes the new pair orthogonal (the smaller root of t^2 + 2 zeta t - 1 = 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Pair (p, q) of slot k in round r of a round-robin tournament of N players
 * (N even): player N-1 is fixed, the others rotate. */
static void tournament_pair(int64_t N, int64_t r, int64_t k, int64_t *p, int64_t *q)
{
    int64_t a, b;
    if (k == 0) {
        a = N - 1;
        b = r;
    } else {
        a = (r + k) % (N - 1);
        b = (r - k + (N - 1)) % (N - 1);
    }
    *p = a < b ? a : b;
    *q = a < b ? b : a;
}

/* Rotate one column pair; returns 1 if a rotation was applied. */
static int rotate_pair(int64_t m, int64_t n, double *W, double *V, int64_t p, int64_t q, double tol)
{
    double *wp = W + p * m, *wq = W + q * m;
    double alpha = 0.0, beta = 0.0, gamma = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        alpha += wp[i] * wp[i];
        beta += wq[i] * wq[i];
        gamma += wp[i] * wq[i];
    }
    if (alpha == 0.0 || beta == 0.0) return 0;
    if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) return 0;
    double zeta = (beta - alpha) / (2.0 * gamma);
    double t;
    if (fabs(zeta) > 1e150)
        t = 1.0 / (2.0 * zeta); /* sqrt(1+zeta^2) ~ |zeta|: avoid overflow */
    else
        t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    double c = 1.0 / sqrt(1.0 + t * t);
    double s = c * t;
    for (int64_t i = 0; i < m; ++i) {
        double x = wp[i], y = wq[i];
        wp[i] = c * x - s * y;
        wq[i] = s * x + c * y;
    }
    double *vp = V + p * n, *vq = V + q * n;
    for (int64_t i = 0; i < n; ++i) {
        double x = vp[i], y = vq[i];
        vp[i] = c * x - s * y;
        vq[i] = s * x + c * y;
    }
    return 1;
}

/*
 * oracle_svd: thin SVD of a real m x n matrix with m >= n >= 1.
 *   A   row-major m x n, leading dimension lda (>= n), FP64, read only.
 *   U   out, row-major m x n: left singular vectors (columns); a column whose
 *       singular value is below the rank tolerance is left zero.
 *   s   out, n singular values, descending; those below the rank tolerance
 *       max(m,n) * 2^-52 * s[0] are reported as 0.
 *   V   out, row-major n x n: right singular vectors (columns).
 *   nthreads  OpenMP threads (<= 0: runtime default).
 * Returns the number of sweeps used (>= 1), -1 if 60 sweeps did not
 * converge, -2 on a bad argument, -3 if memory ran out.
 */
int oracle_svd(int64_t m, int64_t n, const double *A, int64_t lda, double *U, double *s, double *V,
               int nthreads)
{
    if (m < n || n < 1 || lda < n || !A || !U || !s || !V) return -2;
    double *W = (double *)malloc(sizeof(double) * m * n);   /* column-major m x n */
    double *Vc = (double *)malloc(sizeof(double) * n * n);  /* column-major n x n */
    double *nrm = (double *)malloc(sizeof(double) * n);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * n);
    if (!W || !Vc || !nrm || !order) {
        free(W); free(Vc); free(nrm); free(order);
        return -3;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) W[j * m + i] = A[i * lda + j];
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) Vc[j * n + i] = (i == j) ? 1.0 : 0.0;

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* Orthogonality tolerance relative to ||w_p|| ||w_q||: the rounding noise
     * of a length-m dot product is about sqrt(m) ulps. */
    const double tol = 4.0 * sqrt((double)m) * 0x1p-52;
    const int64_t N = (n % 2 == 0) ? n : n + 1; /* odd n: one dummy player */
    int sweeps = 0, converged = 0;
    if (n == 1) converged = 1;
    while (!converged && sweeps < 60) {
        ++sweeps;
        long rotations = 0;
        for (int64_t r = 0; r < N - 1; ++r) {
#pragma omp parallel for reduction(+ : rotations) schedule(static)
            for (int64_t k = 0; k < N / 2; ++k) {
                int64_t p, q;
                tournament_pair(N, r, k, &p, &q);
                if (q >= n) continue;
                rotations += rotate_pair(m, n, W, Vc, p, q, tol);
            }
        }
        if (rotations == 0) converged = 1;
    }
    if (n == 1) sweeps = 1;

    /* singular values = column norms; sort descending (insertion sort on an
     * index array keeps the code plain) */
    for (int64_t j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int64_t i = 0; i < m; ++i) acc += W[j * m + i] * W[j * m + i];
        nrm[j] = sqrt(acc);
        order[j] = j;
    }
    for (int64_t a = 1; a < n; ++a) {
        int64_t key = order[a], b = a - 1;
        while (b >= 0 && nrm[order[b]] < nrm[key]) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = key;
    }
    const double smax = nrm[order[0]];
    const double rank_tol = (double)m * 0x1p-52 * smax;
    for (int64_t jj = 0; jj < n; ++jj) {
        int64_t j = order[jj];
        double sj = nrm[j];
        int keep = sj > rank_tol && sj > 0.0;
        s[jj] = keep ? sj : 0.0;
        for (int64_t i = 0; i < m; ++i) U[i * n + jj] = keep ? W[j * m + i] / sj : 0.0;
        for (int64_t i = 0; i < n; ++i) V[i * n + jj] = Vc[j * n + i];
    }
    free(W); free(Vc); free(nrm); free(order);
    return converged ? sweeps : -1;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
