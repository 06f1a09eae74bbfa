/*
 * FP64 CPU oracle of the ERX detector.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: it is used by the test-suite, by the smoke check and by
 * the CPU-baseline leg of the benchmark, and shares no code, header, table
 * or helper with the GPU library.
 *
 * It computes, for one stream of scan lines X_t in R^{p x b} (pixels x bands,
 * band index fastest), exactly what Sec. III of the paper defines, in double
 * precision, in the order the paper gives:
 *
 *   line mean                mu_hat_t = (1/p) sum_i x_i                  Sec. III-C, Eq. (18)
 *   line covariance          K_hat_t = 1/(p-1) sum_i (x_i-mu_hat)(x_i-mu_hat)^T
 *                                                                         Sec. III-C, Eq. (19)
 *   exponential moving avg   mu_t = (1-a) mu_{t-1} + a mu_hat_t
 *                            K_t  = (1-a) K_{t-1}  + a K_hat_t            Sec. III-C, Eqs. (20)-(21)
 *                            with the first line's statistics as the
 *                            initial background (a = 1 on the first line)
 *   ridge + Cholesky         L_t L_t^T = K_t + eps I                      Sec. III-D
 *   forward substitution     L_t m_i = x_i - mu_t,  delta_i = sqrt(m.m)   Sec. III-D, Eqs. (22)-(23)
 *   line normalisation       (delta_i - mean) / std over the line         Sec. III-E, Eq. (24)
 *
 * Readings taken where the text is ambiguous (documented with the design):
 *   - the ridge is added to the covariance itself (the factor is of
 *     K_t + eps I, not of an inverse), otherwise the forward substitution
 *     would not give a Mahalanobis distance;
 *   - each line is scored with the background AFTER its own update, which is
 *     what makes momentum 1 mean "only the current line's statistics";
 *   - m is the column vector L^{-1}(x - mu);
 *   - the normalisation uses the population standard deviation over the p
 *     pixels of the line; a zero deviation gives 0;
 *   - a pivot <= 0 (possible only without ridge on a singular covariance)
 *     marks the line "not positive definite" and its scores NaN.
 *
 * Plain loops, no BLAS, no blocking.  OpenMP is used only to spread
 * independent pixels or matrix rows across threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ERO_EXPORT __attribute__((visibility("default")))

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

ERO_EXPORT int ero_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sec. III-C, Eq. (18): mean over the p pixels of one line. */
ERO_EXPORT void ero_line_mean(int b, int p, const double *X, double *mu_hat)
{
    for (int j = 0; j < b; ++j) mu_hat[j] = 0.0;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < b; ++j) mu_hat[j] += X[(size_t)i * b + j];
    for (int j = 0; j < b; ++j) mu_hat[j] /= (double)p;
}

/* Sec. III-C, Eq. (19): covariance of one line, centred on its own mean,
 * normalised by p-1.  Output is the full symmetric b x b matrix. */
ERO_EXPORT void ero_line_cov(int b, int p, const double *X, const double *mu_hat,
                             double *K_hat, int nthreads)
{
    set_threads(nthreads);
    double *Ct = (double *)malloc(sizeof(double) * (size_t)b * (size_t)p);
    /* centred data, transposed so that each band is one contiguous row */
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < b; ++j)
            Ct[(size_t)j * p + i] = X[(size_t)i * b + j] - mu_hat[j];
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < b; ++r) {
        const double *cr = Ct + (size_t)r * p;
        for (int c = 0; c <= r; ++c) {
            const double *cc = Ct + (size_t)c * p;
            double s = 0.0;
            for (int i = 0; i < p; ++i) s += cr[i] * cc[i];
            s /= (double)(p - 1);
            K_hat[(size_t)r * b + c] = s;
            K_hat[(size_t)c * b + r] = s;
        }
    }
    free(Ct);
}

/* Textbook Cholesky (row by row), lower factor with positive diagonal.
 * Returns 0 on success, k+1 if the k-th pivot is not positive (the factor
 * is then incomplete).  A NaN pivot is not reported: it propagates. */
ERO_EXPORT int ero_cholesky(int b, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)b * (size_t)b);
    for (int i = 0; i < b; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[(size_t)i * b + j];
            for (int k = 0; k < j; ++k) s -= L[(size_t)i * b + k] * L[(size_t)j * b + k];
            if (i == j) {
                if (s <= 0.0) return i + 1;
                L[(size_t)i * b + i] = sqrt(s);
            } else {
                L[(size_t)i * b + j] = s / L[(size_t)j * b + j];
            }
        }
    }
    return 0;
}

/* Sec. III-D, Eqs. (22)-(23): solve L m = r by forward substitution and
 * return sqrt(m . m).  m has room for b values. */
ERO_EXPORT double ero_mahalanobis(int b, const double *L, const double *r, double *m)
{
    double ss = 0.0;
    for (int i = 0; i < b; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * b + k] * m[k];
        m[i] = s / L[(size_t)i * b + i];
        ss += m[i] * m[i];
    }
    return sqrt(ss);
}

/* Sec. III-E, Eq. (24): line-wise standardisation with the population
 * standard deviation; a zero deviation maps every score to 0. */
ERO_EXPORT void ero_normalise(int p, const double *delta, double *out)
{
    double mean = 0.0, var = 0.0;
    for (int i = 0; i < p; ++i) mean += delta[i];
    mean /= (double)p;
    for (int i = 0; i < p; ++i) var += (delta[i] - mean) * (delta[i] - mean);
    var /= (double)p;
    double sd = sqrt(var);
    for (int i = 0; i < p; ++i) out[i] = (sd > 0.0) ? (delta[i] - mean) / sd : (sd == 0.0 ? 0.0 : sd);
}

/*
 * Run the detector over n lines of one stream.
 *
 *   state:   *t     number of lines already absorbed (0 for a new stream)
 *            mu[b]  background mean after line *t   (ignored when *t == 0)
 *            K[b*b] background covariance after line *t (full, symmetric)
 *   X:       [n][p][b] lines
 *   delta:   [n][p] Mahalanobis distance of every pixel (after its line's update)
 *   delta_n: optional [n][p] line-normalised scores (NULL to skip)
 *   mu_hist, K_hist: optional per-line copies of the background after each
 *            line ([n][b], [n][b*b]; NULL to skip)
 *   notpd:   optional [n] flags, 1 where K_t + eps I had a non-positive pivot
 *
 * Returns the number of not-positive-definite lines, or -1 on invalid
 * arguments (b < 1, p < 2, momentum outside (0, 1], eps < 0, n < 0).
 */
ERO_EXPORT long long ero_push(int b, int p, double alpha, double eps,
                              long long *t, double *mu, double *K,
                              const double *X, long long n,
                              double *delta, double *delta_n,
                              double *mu_hist, double *K_hist, int *notpd,
                              int nthreads)
{
    if (b < 1 || p < 2 || !(alpha > 0.0 && alpha <= 1.0) || !(eps >= 0.0) || n < 0) return -1;
    set_threads(nthreads);
    const size_t bb = (size_t)b * (size_t)b;
    double *mu_hat = (double *)malloc(sizeof(double) * (size_t)b);
    double *K_hat = (double *)malloc(sizeof(double) * bb);
    double *A = (double *)malloc(sizeof(double) * bb);
    double *L = (double *)malloc(sizeof(double) * bb);
    long long bad = 0;

    for (long long l = 0; l < n; ++l) {
        const double *x = X + (size_t)l * (size_t)p * (size_t)b;
        ero_line_mean(b, p, x, mu_hat);
        ero_line_cov(b, p, x, mu_hat, K_hat, nthreads);
        /* the first line's statistics are the initial background;
         * later lines are blended in with momentum alpha */
        if (*t == 0) {
            memcpy(mu, mu_hat, sizeof(double) * (size_t)b);
            memcpy(K, K_hat, sizeof(double) * bb);
        } else {
            for (int j = 0; j < b; ++j) mu[j] = (1.0 - alpha) * mu[j] + alpha * mu_hat[j];
            for (size_t e = 0; e < bb; ++e) K[e] = (1.0 - alpha) * K[e] + alpha * K_hat[e];
        }
        *t += 1;
        if (mu_hist) memcpy(mu_hist + (size_t)l * b, mu, sizeof(double) * (size_t)b);
        if (K_hist) memcpy(K_hist + (size_t)l * bb, K, sizeof(double) * bb);

        /* ridge, then the Cholesky factor of the regularised covariance */
        memcpy(A, K, sizeof(double) * bb);
        for (int j = 0; j < b; ++j) A[(size_t)j * b + j] += eps;
        const int fail = ero_cholesky(b, A, L);
        if (notpd) notpd[l] = fail ? 1 : 0;
        double *dl = delta + (size_t)l * p;
        if (fail) {
            ++bad;
            for (int i = 0; i < p; ++i) dl[i] = NAN;
        } else {
#pragma omp parallel
            {
                double *r = (double *)malloc(sizeof(double) * (size_t)b);
                double *m = (double *)malloc(sizeof(double) * (size_t)b);
#pragma omp for schedule(static)
                for (int i = 0; i < p; ++i) {
                    const double *xi = x + (size_t)i * b;
                    for (int j = 0; j < b; ++j) r[j] = xi[j] - mu[j];
                    dl[i] = ero_mahalanobis(b, L, r, m);
                }
                free(r);
                free(m);
            }
        }
        if (delta_n) ero_normalise(p, dl, delta_n + (size_t)l * p);
    }
    free(mu_hat);
    free(K_hat);
    free(A);
    free(L);
    return bad;
}
