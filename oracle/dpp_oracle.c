/*
 * FP64 CPU oracle for the factorization-based DPP sampler.
 *
 * TEST INFRASTRUCTURE ONLY. This file exists to check the GPU library
 * against the paper; it is not part of the product path. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Poulson, "High-performance sampling of generic
 * Determinantal Point Processes", Sec. 2, Theorem 2 and the unblocked
 * right-looking sampler listing that follows it):
 *
 *   A := K
 *   for j = 0 .. n-1:
 *     d_j := A[j,j]                      (conditional inclusion probability)
 *     keep j iff u_j < d_j, else A[j,j] := d_j - 1
 *     A[j+1:n, j] /= A[j,j]
 *     A[j+1:n, j+1:n] -= A[j+1:n, j] * A[j, j+1:n]
 *
 * The keep branch preserves the loop invariant by Prop. 3 (condition on
 * inclusion) and the reject branch by Prop. 4 (condition on exclusion of one
 * element). On return A holds, in place, the unpivoted factorization of
 * K - 1_{Y^c}; the likelihood of the sample is the product of the absolute
 * values of the final pivots (Theorem 2 and the alternate proof of Prop. 1
 * that follows the listing), so loglik = sum_j ln|A[j,j]|.
 *
 * The Hermitian variant uses the symmetric specialization the paper points
 * to (Sec. 2, the paragraph on LDL^H specializations): only the lower
 * triangle is read and written, and the row A[j, j+1:n] of the update is the
 * (real) mirror of the not-yet-scaled column A[j+1:n, j]. On return the
 * strict lower triangle holds the unit-lower L and the diagonal holds D of
 * K - 1_{Y^c} = L D L^T.
 *
 * Conventions (readings of points the paper leaves open):
 *   - one uniform u_j per index, consumed in index order; keep iff u_j < d_j
 *     (strict), so u_j = d_j rejects;
 *   - d_j is compared as computed, without clamping to [0,1];
 *   - loglik is the natural logarithm;
 *   - info = j+1 for the first pivot that is exactly zero or NaN after the
 *     decision (0 if none); the values after such a pivot are unspecified.
 *
 * Storage is column-major with leading dimension lda >= n.
 * The rank-one update is parallelized over columns with OpenMP: every
 * element still receives exactly the updates of the listing, in the same
 * order, so the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(A, lda, i, k) ((A)[(size_t)(i) + (size_t)(k) * (size_t)(lda)])

/* Bernoulli decision and pivot modification of one index (Theorem 2). */
static double decide(double d, double u, uint8_t* keep)
{
    if (u < d) {
        *keep = 1;
        return d;
    }
    *keep = 0;
    return d - 1.0;
}

/*
 * Non-Hermitian sampler: the unblocked listing as written, on all of A.
 * npiv limits the run to the first npiv pivots (npiv <= 0 or >= n: all);
 * the outputs for indices >= npiv are then left untouched and loglik sums
 * only the processed pivots. predec (may be NULL) receives d_j before the
 * decision.
 */
int dpp_oracle_lu(double* A, int64_t n, int64_t lda, const double* u, int64_t npiv,
                  uint8_t* mask, double* pivots, double* predec, double* loglik,
                  int32_t* info)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || !A || !u || !mask || !pivots || !loglik || !info)
        return 1;
    if (npiv <= 0 || npiv > n) npiv = n;
    double ll = 0.0;
    int32_t inf = 0;
    for (int64_t j = 0; j < npiv; ++j) {
        double d = AT(A, lda, j, j);
        if (predec) predec[j] = d;
        double dp = decide(d, u[j], &mask[j]);
        AT(A, lda, j, j) = dp;
        pivots[j] = dp;
        ll += log(fabs(dp));
        if (inf == 0 && (dp == 0.0 || isnan(dp))) inf = (int32_t)(j + 1);
        /* A[j+1:n, j] /= A[j,j] */
        for (int64_t i = j + 1; i < n; ++i) AT(A, lda, i, j) /= dp;
        /* A[j+1:n, j+1:n] -= A[j+1:n, j] * A[j, j+1:n] */
#pragma omp parallel for schedule(static)
        for (int64_t k = j + 1; k < n; ++k) {
            const double ujk = AT(A, lda, j, k);
            double* colk = &AT(A, lda, 0, k);
            const double* colj = &AT(A, lda, 0, j);
            for (int64_t i = j + 1; i < n; ++i) colk[i] -= colj[i] * ujk;
        }
    }
    *loglik = ll;
    *info = inf;
    return 0;
}

/*
 * Hermitian (real symmetric) sampler: the same listing on the lower triangle.
 * The upper triangle of A is neither read nor written. The row A[j, j+1:n]
 * that the listing's update uses is, by symmetry, the column A[j+1:n, j]
 * before it is scaled; it is saved in row_j (n doubles of scratch owned by
 * the caller) before the column is scaled, and the update then follows the
 * listing: A[i,k] -= A[i,j] * A[j,k] for j < k <= i.
 */
int dpp_oracle_ldlh(double* A, int64_t n, int64_t lda, const double* u, int64_t npiv,
                    uint8_t* mask, double* pivots, double* predec, double* loglik,
                    int32_t* info, double* row_j)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || !A || !u || !mask || !pivots || !loglik || !info ||
        !row_j)
        return 1;
    if (npiv <= 0 || npiv > n) npiv = n;
    double ll = 0.0;
    int32_t inf = 0;
    for (int64_t j = 0; j < npiv; ++j) {
        double d = AT(A, lda, j, j);
        if (predec) predec[j] = d;
        double dp = decide(d, u[j], &mask[j]);
        AT(A, lda, j, j) = dp;
        pivots[j] = dp;
        ll += log(fabs(dp));
        if (inf == 0 && (dp == 0.0 || isnan(dp))) inf = (int32_t)(j + 1);
        /* row_j[k] = A[j,k] = A[k,j] (unscaled), then A[j+1:n, j] /= A[j,j] */
        for (int64_t k = j + 1; k < n; ++k) {
            row_j[k] = AT(A, lda, k, j);
            AT(A, lda, k, j) /= dp;
        }
        /* lower triangle of A[j+1:n, j+1:n] -= A[j+1:n, j] * A[j, j+1:n] */
#pragma omp parallel for schedule(static)
        for (int64_t k = j + 1; k < n; ++k) {
            const double ajk = row_j[k];
            double* colk = &AT(A, lda, 0, k);
            const double* colj = &AT(A, lda, 0, j);
            for (int64_t i = k; i < n; ++i) colk[i] -= colj[i] * ajk;
        }
    }
    *loglik = ll;
    *info = inf;
    return 0;
}

/* Number of OpenMP threads the rank-one updates run on. */
int dpp_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Complex kernels (Sec. 1 examples built on complex kernels; Sec. 3, the
 * dense complex LU experiment). Same listing, complex arithmetic. Storage is
 * interleaved (real, imaginary) doubles, column-major, leading dimension lda
 * counted in complex entries.
 *
 * Readings of points the paper leaves open for complex kernels:
 *   - a conditional inclusion probability is real, so the imaginary part of
 *     a computed diagonal entry is rounding residue: the Bernoulli decision,
 *     the returned pivots and predec and the likelihood use the real part;
 *     d'_j = Re(A[j,j]) on keeping, Re(A[j,j]) - 1 on rejecting;
 *   - LU scales the column by the whole complex pivot (A[j,j], or A[j,j] - 1),
 *     so L U is exactly the computed factorization of K - 1_{Y^c};
 *   - LDL^H (Hermitian K, lower triangle): D is real, the diagonal entries'
 *     imaginary parts are never read, and the stored diagonal is d'_j + 0i;
 *     the update subtracts l_i d'_j conj(l_k), i.e. the scaled column times
 *     the conjugate of the unscaled one;
 *   - info: the first j with Re(d'_j) == 0 or a NaN part.
 */
#include <complex.h>

#define ZAT(A, lda, i, k) ((A)[(size_t)(i) + (size_t)(k) * (size_t)(lda)])

static int zbad(double complex p) { return creal(p) == 0.0 || isnan(creal(p)) || isnan(cimag(p)); }

int dpp_oracle_zlu(double* Araw, int64_t n, int64_t lda, const double* u, int64_t npiv,
                   uint8_t* mask, double* pivots, double* predec, double* loglik, int32_t* info)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || !Araw || !u || !mask || !pivots || !loglik || !info)
        return 1;
    double complex* A = (double complex*)Araw;
    if (npiv <= 0 || npiv > n) npiv = n;
    double ll = 0.0;
    int32_t inf = 0;
    for (int64_t j = 0; j < npiv; ++j) {
        const double complex a = ZAT(A, lda, j, j);
        const double d = creal(a);
        if (predec) predec[j] = d;
        uint8_t keep;
        const double dp = decide(d, u[j], &keep);
        mask[j] = keep;
        const double complex p = keep ? a : a - 1.0;
        ZAT(A, lda, j, j) = p;
        pivots[j] = dp;
        ll += log(fabs(dp));
        if (inf == 0 && zbad(p)) inf = (int32_t)(j + 1);
        for (int64_t i = j + 1; i < n; ++i) ZAT(A, lda, i, j) /= p;
#pragma omp parallel for schedule(static)
        for (int64_t k = j + 1; k < n; ++k) {
            const double complex ujk = ZAT(A, lda, j, k);
            double complex* colk = &ZAT(A, lda, 0, k);
            const double complex* colj = &ZAT(A, lda, 0, j);
            for (int64_t i = j + 1; i < n; ++i) colk[i] -= colj[i] * ujk;
        }
    }
    *loglik = ll;
    *info = inf;
    return 0;
}

/* Hermitian complex kernel, lower triangle; row_j: 2n doubles of scratch. */
int dpp_oracle_zldlh(double* Araw, int64_t n, int64_t lda, const double* u, int64_t npiv,
                     uint8_t* mask, double* pivots, double* predec, double* loglik,
                     int32_t* info, double* row_raw)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || !Araw || !u || !mask || !pivots || !loglik || !info ||
        !row_raw)
        return 1;
    double complex* A = (double complex*)Araw;
    double complex* row_j = (double complex*)row_raw;
    if (npiv <= 0 || npiv > n) npiv = n;
    double ll = 0.0;
    int32_t inf = 0;
    for (int64_t j = 0; j < npiv; ++j) {
        const double d = creal(ZAT(A, lda, j, j));
        if (predec) predec[j] = d;
        const double dp = decide(d, u[j], &mask[j]);
        ZAT(A, lda, j, j) = dp;
        pivots[j] = dp;
        ll += log(fabs(dp));
        if (inf == 0 && (dp == 0.0 || isnan(dp))) inf = (int32_t)(j + 1);
        /* row_j[k] = A[j,k] = conj(A[k,j]) (unscaled), then A[j+1:n, j] /= d'_j */
        for (int64_t k = j + 1; k < n; ++k) {
            row_j[k] = conj(ZAT(A, lda, k, j));
            ZAT(A, lda, k, j) /= dp;
        }
#pragma omp parallel for schedule(static)
        for (int64_t k = j + 1; k < n; ++k) {
            const double complex ajk = row_j[k];
            double complex* colk = &ZAT(A, lda, 0, k);
            const double complex* colj = &ZAT(A, lda, 0, j);
            for (int64_t i = k; i < n; ++i) colk[i] -= colj[i] * ajk;
        }
    }
    *loglik = ll;
    *info = inf;
    return 0;
}
