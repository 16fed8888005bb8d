/*
 * CPU oracle helpers in plain C.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product library links, loads or calls this file; only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg use it, through oracle/.
 *
 * Two things here need arithmetic that NumPy does not offer:
 *
 *  1. the alpha/beta step of the emulated GEMM, which the recombination
 *     reading fixes as one fused multiply-add per element
 *        C <- fma(alpha, X, beta*C)      (beta != 0)
 *        C <- fma(alpha, X, 0.0)         (beta == 0, C not read);
 *     C99 fma() is the correctly rounded IEEE 754 fusedMultiplyAdd.
 *
 *  2. the double-double reference products that stand in for the true FP64
 *     product the emulation approximates (the paper's emulation section
 *     measures the split scheme against FP64): each dot product is evaluated
 *     with the compensated algorithm Dot2 of Ogita, Rump and Oishi,
 *     "Accurate sum and dot product", SIAM J. Sci. Comput. 26(6), 2005:
 *        TwoProduct(a, b) -> (p, e): p = fl(a*b), e = fma(a, b, -p)
 *        TwoSum(s, p)     -> (s', q): s' = fl(s+p), exact error q (Knuth)
 *        result = fl(s + sum of all errors)
 *     Its error is at most u|x'y| + gamma_{n}^2 |x|'|y|, i.e. the value is the
 *     correctly rounded dot product unless cancellation exceeds ~1e16.
 *
 * Matrices are column-major with leading dimensions, as in the library ABI.
 */
#include <math.h>
#include <stdint.h>

static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* C[i] <- fma(alpha, X[i], beta*C[i]) (beta != 0) or fma(alpha, X[i], 0). */
void orc_axpby_fma(int64_t count, double alpha, const double *X, double beta,
                   double *C)
{
    if (beta == 0.0) {
        for (int64_t i = 0; i < count; ++i) C[i] = fma(alpha, X[i], 0.0);
    } else {
        for (int64_t i = 0; i < count; ++i) C[i] = fma(alpha, X[i], beta * C[i]);
    }
}

/* C (m x n) <- Dot2 evaluation of A (m x k) * B (k x n). */
void orc_dot2_gemm(int m, int n, int k, const double *A, int lda,
                   const double *B, int ldb, double *C, int ldc)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < m; ++i) {
            double s = 0.0, c = 0.0;
            for (int l = 0; l < k; ++l) {
                double p, ep, q;
                two_prod(A[i + (int64_t)l * lda], B[l + (int64_t)j * ldb], &p, &ep);
                two_sum(s, p, &s, &q);
                c += q + ep;
            }
            C[i + (int64_t)j * ldc] = s + c;
        }
    }
}

/* R (n x nrhs) <- Dot2 evaluation of B - A X, A n x n. */
void orc_dot2_residual(int n, int nrhs, const double *A, int lda,
                       const double *X, int ldx, const double *B, int ldb,
                       double *R, int ldr)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int j = 0; j < nrhs; ++j) {
        for (int i = 0; i < n; ++i) {
            double s = B[i + (int64_t)j * ldb], c = 0.0;
            for (int l = 0; l < n; ++l) {
                double p, ep, q;
                two_prod(-A[i + (int64_t)l * lda], X[l + (int64_t)j * ldx], &p, &ep);
                two_sum(s, p, &s, &q);
                c += q + ep;
            }
            R[i + (int64_t)j * ldr] = s + c;
        }
    }
}

/* Number of OpenMP threads the parallel loops above use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
