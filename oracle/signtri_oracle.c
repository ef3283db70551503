/*
 * TEST INFRASTRUCTURE ONLY -- the CPU oracle for U = sign(T).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  The product library (HIP kernels behind the C ABI in
 * include/signtri.h) shares nothing with it: no header, helper, table or
 * constant.  It is deliberately plain and slow: element by element, FP64 or
 * complex128, ascending summation order, compiled without floating-point
 * contraction so that every result is reproducible bit for bit.
 *
 * What it computes (Stotland, Schwartz, Toledo, "High-Performance Algorithms
 * for Computing the Sign Function of Triangular Matrices"):
 *
 *   - the scalar sign takes the sign of the real part (Section 1); it is
 *     undefined when the real part is zero (Section 1, last paragraph of the
 *     definition), and we also reject non-finite diagonal entries;
 *   - u_ii = sign(t_ii) (Algorithm 3, first loop);
 *   - for every i < j, visited by column j ascending and row i descending
 *     (Algorithm 3), either
 *       Eq. (1), the element Parlett equation from TU = UT, when
 *                u_ii + u_jj = 0 (the two signs differ):
 *         u_ij = t_ij (u_ii - u_jj) / (t_ii - t_jj)
 *                + [sum_{k=i+1}^{j-1} (u_ik t_kj - t_ik u_kj)] / (t_ii - t_jj)
 *       Eq. (2), Higham's involution equation from U^2 = I, otherwise:
 *         u_ij = - [sum_{k=i+1}^{j-1} u_ik u_kj] / (u_ii + u_jj)
 *   - u_ij = 0 below the diagonal.
 *
 * The superdiagonal d = j - i of U depends only on superdiagonals < d, so the
 * entries of one superdiagonal are computed in parallel (OpenMP).  Each entry
 * uses the same expression and the same k order as the column-wise loop of
 * Algorithm 3, so the result is bitwise identical to the serial order.
 *
 * The Sylvester oracle solves A X - X B = C for upper-triangular A (m x m)
 * and B (p x p) by element substitution.  With F_ii = I and F_jj = -I (or the
 * reverse) the block equation of Algorithm 2 for a sign-split T reduces to
 * exactly this equation with C = +-2 T_12 (Section 2, the paragraph on the
 * trivial diagonal blocks of the sign function).
 *
 * The Parlett oracle computes F = phi(T) for a general function phi given
 * its values on the diagonal, f_ii = phi(t_ii) (Algorithm 1): for every i < j,
 * by column j ascending and row i descending,
 *   f_ij = [t_ij (f_ii - f_jj) + sum_{k=i+1}^{j-1} (f_ik t_kj - t_ik f_kj)]
 *          / (t_ii - t_jj),
 * the element equation of TF = FT (Section 2); it needs distinct diagonal
 * entries.
 *
 * Storage: column-major with a leading dimension; complex numbers are
 * interleaved (re, im) pairs of doubles.  Only the upper triangle of the
 * inputs is read.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Sign of the real part: +1, -1, or 0 when undefined (zero or not finite). */
static int real_part_sign(double re, double im)
{
    if (!isfinite(re) || !isfinite(im)) return 0;
    if (re > 0.0) return 1;
    if (re < 0.0) return -1;
    return 0;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Real case.  Returns 0 on success, or the 1-based index of the first
 * diagonal entry whose sign is undefined (U is then left untouched), or -1 if
 * memory could not be allocated.
 */
int64_t oracle_sign_tri_d(int64_t n, const double *T, int64_t ldt,
                          double *U, int64_t ldu, int nthreads)
{
    if (n <= 0) return 0;
    int *s = (int *)malloc(sizeof(int) * (size_t)n);
    if (!s) return -1;
    for (int64_t i = 0; i < n; ++i) {
        s[i] = real_part_sign(T[i + i * ldt], 0.0);
        if (s[i] == 0) { free(s); return i + 1; }
    }
    size_t nn = (size_t)n * (size_t)n;
    /* Row-major copies give unit stride for u_ik, t_ik; column-major copies
     * give unit stride for u_kj, t_kj. */
    double *Tr = (double *)calloc(nn, sizeof(double));
    double *Tc = (double *)calloc(nn, sizeof(double));
    double *Ur = (double *)calloc(nn, sizeof(double));
    double *Uc = (double *)calloc(nn, sizeof(double));
    if (!Tr || !Tc || !Ur || !Uc) {
        free(Tr); free(Tc); free(Ur); free(Uc); free(s);
        return -1;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i <= j; ++i) {
            double t = T[i + j * ldt];
            Tr[i * n + j] = t;
            Tc[j * n + i] = t;
        }
    for (int64_t i = 0; i < n; ++i) {
        Ur[i * n + i] = (double)s[i];
        Uc[i * n + i] = (double)s[i];
    }
    set_threads(nthreads);
#pragma omp parallel
    for (int64_t d = 1; d < n; ++d) {
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n - d; ++i) {
            int64_t j = i + d;
            const double *uri = Ur + i * n; /* u_i* */
            const double *tri = Tr + i * n; /* t_i* */
            const double *ucj = Uc + j * n; /* u_*j */
            const double *tcj = Tc + j * n; /* t_*j */
            double uii = (double)s[i], ujj = (double)s[j];
            double u;
            if (uii + ujj == 0.0) {
                /* Eq. (1) */
                double sum = 0.0;
                for (int64_t k = i + 1; k < j; ++k)
                    sum = sum + (uri[k] * tcj[k] - tri[k] * ucj[k]);
                double den = tri[i] - Tr[j * n + j];
                u = tri[j] * (uii - ujj) / den + sum / den;
            } else {
                /* Eq. (2) */
                double sum = 0.0;
                for (int64_t k = i + 1; k < j; ++k)
                    sum = sum + uri[k] * ucj[k];
                u = -sum / (uii + ujj);
            }
            Ur[i * n + j] = u;
            Uc[j * n + i] = u;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            U[i + j * ldu] = (i <= j) ? Ur[i * n + j] : 0.0;
    free(Tr); free(Tc); free(Ur); free(Uc); free(s);
    return 0;
}

/* Complex helpers, written out in real arithmetic. */
typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b)
{
    cplx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}

static inline cplx csub(cplx a, cplx b)
{
    cplx r;
    r.re = a.re - b.re;
    r.im = a.im - b.im;
    return r;
}

static inline cplx cadd(cplx a, cplx b)
{
    cplx r;
    r.re = a.re + b.re;
    r.im = a.im + b.im;
    return r;
}

/* a / b by the textbook formula (a * conj(b)) / |b|^2. */
static inline cplx cdiv(cplx a, cplx b)
{
    double den = b.re * b.re + b.im * b.im;
    cplx r;
    r.re = (a.re * b.re + a.im * b.im) / den;
    r.im = (a.im * b.re - a.re * b.im) / den;
    return r;
}

static inline cplx cscale(cplx a, double x)
{
    cplx r;
    r.re = a.re * x;
    r.im = a.im * x;
    return r;
}

/*
 * Complex case, same algorithm and return convention as the real case.
 * T and U hold interleaved (re, im) doubles; ldt, ldu count complex elements.
 */
int64_t oracle_sign_tri_z(int64_t n, const double *T, int64_t ldt,
                          double *U, int64_t ldu, int nthreads)
{
    if (n <= 0) return 0;
    int *s = (int *)malloc(sizeof(int) * (size_t)n);
    if (!s) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const double *t = T + 2 * (i + i * ldt);
        s[i] = real_part_sign(t[0], t[1]);
        if (s[i] == 0) { free(s); return i + 1; }
    }
    size_t nn = (size_t)n * (size_t)n;
    cplx *Tr = (cplx *)calloc(nn, sizeof(cplx));
    cplx *Tc = (cplx *)calloc(nn, sizeof(cplx));
    cplx *Ur = (cplx *)calloc(nn, sizeof(cplx));
    cplx *Uc = (cplx *)calloc(nn, sizeof(cplx));
    if (!Tr || !Tc || !Ur || !Uc) {
        free(Tr); free(Tc); free(Ur); free(Uc); free(s);
        return -1;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i <= j; ++i) {
            const double *t = T + 2 * (i + j * ldt);
            cplx v;
            v.re = t[0];
            v.im = t[1];
            Tr[i * n + j] = v;
            Tc[j * n + i] = v;
        }
    for (int64_t i = 0; i < n; ++i) {
        cplx v;
        v.re = (double)s[i];
        v.im = 0.0;
        Ur[i * n + i] = v;
        Uc[i * n + i] = v;
    }
    set_threads(nthreads);
#pragma omp parallel
    for (int64_t d = 1; d < n; ++d) {
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n - d; ++i) {
            int64_t j = i + d;
            const cplx *uri = Ur + i * n;
            const cplx *tri = Tr + i * n;
            const cplx *ucj = Uc + j * n;
            const cplx *tcj = Tc + j * n;
            double uii = (double)s[i], ujj = (double)s[j];
            cplx u;
            if (uii + ujj == 0.0) {
                /* Eq. (1) */
                cplx sum = {0.0, 0.0};
                for (int64_t k = i + 1; k < j; ++k)
                    sum = cadd(sum, csub(cmul(uri[k], tcj[k]), cmul(tri[k], ucj[k])));
                cplx den = csub(tri[i], Tr[j * n + j]);
                u = cadd(cdiv(cscale(tri[j], uii - ujj), den), cdiv(sum, den));
            } else {
                /* Eq. (2) */
                cplx sum = {0.0, 0.0};
                for (int64_t k = i + 1; k < j; ++k)
                    sum = cadd(sum, cmul(uri[k], ucj[k]));
                u = cscale(sum, -1.0 / (uii + ujj));
            }
            Ur[i * n + j] = u;
            Uc[j * n + i] = u;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            double *o = U + 2 * (i + j * ldu);
            if (i <= j) {
                o[0] = Ur[i * n + j].re;
                o[1] = Ur[i * n + j].im;
            } else {
                o[0] = 0.0;
                o[1] = 0.0;
            }
        }
    free(Tr); free(Tc); free(Ur); free(Uc); free(s);
    return 0;
}

/*
 * Triangular Sylvester equation A X - X B = C (real), A m x m and B p x p
 * upper triangular, X and C m x p.  Element (i, j) of the equation reads
 *   (a_ii - b_jj) x_ij = c_ij - sum_{k>i} a_ik x_kj + sum_{k<j} x_ik b_kj,
 * so rows are taken bottom-up and columns left to right.  Returns 0, or the
 * 1-based linear index (i + j*m + 1) of the first zero pivot a_ii - b_jj.
 */
int64_t oracle_trsyl_d(int64_t m, int64_t p, const double *A, int64_t lda,
                       const double *B, int64_t ldb, const double *C,
                       int64_t ldc, double *X, int64_t ldx)
{
    for (int64_t j = 0; j < p; ++j)
        for (int64_t i = m - 1; i >= 0; --i) {
            double sum = C[i + j * ldc];
            for (int64_t k = i + 1; k < m; ++k)
                sum = sum - A[i + k * lda] * X[k + j * ldx];
            for (int64_t k = 0; k < j; ++k)
                sum = sum + X[i + k * ldx] * B[k + j * ldb];
            double den = A[i + i * lda] - B[j + j * ldb];
            if (den == 0.0) return i + j * m + 1;
            X[i + j * ldx] = sum / den;
        }
    return 0;
}

/* Complex version of oracle_trsyl_d (interleaved storage). */
int64_t oracle_trsyl_z(int64_t m, int64_t p, const double *A, int64_t lda,
                       const double *B, int64_t ldb, const double *C,
                       int64_t ldc, double *X, int64_t ldx)
{
#define CZ(M, ld, r, c) (*(const cplx *)((M) + 2 * ((r) + (c) * (ld))))
    for (int64_t j = 0; j < p; ++j)
        for (int64_t i = m - 1; i >= 0; --i) {
            cplx sum = CZ(C, ldc, i, j);
            for (int64_t k = i + 1; k < m; ++k)
                sum = csub(sum, cmul(CZ(A, lda, i, k), CZ(X, ldx, k, j)));
            for (int64_t k = 0; k < j; ++k)
                sum = cadd(sum, cmul(CZ(X, ldx, i, k), CZ(B, ldb, k, j)));
            cplx den = csub(CZ(A, lda, i, i), CZ(B, ldb, j, j));
            if (den.re == 0.0 && den.im == 0.0) return i + j * m + 1;
            cplx x = cdiv(sum, den);
            X[2 * (i + j * ldx)] = x.re;
            X[2 * (i + j * ldx) + 1] = x.im;
        }
#undef CZ
    return 0;
}

/*
 * F = phi(T) by Algorithm 1 (real): fd[i] = phi(t_ii) given; F n x n, zero
 * below the diagonal.  Returns 0, or the 1-based linear index (i + j*n + 1) of
 * the first pair with t_ii == t_jj (the recurrence is undefined there).
 */
int64_t oracle_parlett_d(int64_t n, const double *T, int64_t ldt, const double *fd,
                         double *F, int64_t ldf)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) F[i + j * ldf] = i == j ? fd[i] : 0.0;
    for (int64_t j = 1; j < n; ++j)
        for (int64_t i = j - 1; i >= 0; --i) {
            double sum = T[i + j * ldt] * (fd[i] - fd[j]);
            for (int64_t k = i + 1; k < j; ++k)
                sum = sum + (F[i + k * ldf] * T[k + j * ldt] - T[i + k * ldt] * F[k + j * ldf]);
            const double den = T[i + i * ldt] - T[j + j * ldt];
            if (den == 0.0) return i + j * n + 1;
            F[i + j * ldf] = sum / den;
        }
    return 0;
}

/* Complex version of oracle_parlett_d (interleaved storage, fd interleaved too). */
int64_t oracle_parlett_z(int64_t n, const double *T, int64_t ldt, const double *fd,
                         double *F, int64_t ldf)
{
#define CZ(M, ld, r, c) (*(const cplx *)((M) + 2 * ((r) + (c) * (ld))))
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            F[2 * (i + j * ldf)] = i == j ? fd[2 * i] : 0.0;
            F[2 * (i + j * ldf) + 1] = i == j ? fd[2 * i + 1] : 0.0;
        }
    for (int64_t j = 1; j < n; ++j)
        for (int64_t i = j - 1; i >= 0; --i) {
            const cplx fi = {fd[2 * i], fd[2 * i + 1]}, fj = {fd[2 * j], fd[2 * j + 1]};
            cplx sum = cmul(CZ(T, ldt, i, j), csub(fi, fj));
            for (int64_t k = i + 1; k < j; ++k)
                sum = cadd(sum, csub(cmul(CZ(F, ldf, i, k), CZ(T, ldt, k, j)),
                                     cmul(CZ(T, ldt, i, k), CZ(F, ldf, k, j))));
            const cplx den = csub(CZ(T, ldt, i, i), CZ(T, ldt, j, j));
            if (den.re == 0.0 && den.im == 0.0) return i + j * n + 1;
            const cplx x = cdiv(sum, den);
            F[2 * (i + j * ldf)] = x.re;
            F[2 * (i + j * ldf) + 1] = x.im;
        }
#undef CZ
    return 0;
}
