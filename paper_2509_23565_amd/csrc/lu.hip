// FP64 parts of the blocked LU with partial pivoting and of the solve
// (paper: section "Dense Numerical Solvers Using FP64 Emulation", eqns
// (5)-(8): the panel, where the pivots are chosen and U11^-1 reaches A21,
// stays in FP64 "custom code"; only the Schur update is emulated).
//
// Every FP64 update here is one rounded product followed by one rounded
// subtraction (this file is compiled with -ffp-contract=off), applied to each
// element in increasing elimination order, so the factors and solutions are
// identical bit for bit to a column-by-column right-looking elimination with
// the same pivots.
#include "common.h"

#include <float.h>

namespace emu {

// ---------------------------------------------------------------- panel
// Pivot order: NaN ranks above every number; otherwise larger magnitude
// wins; ties go to the smaller row index.
__device__ __forceinline__ bool better(double va, int ia, double vb, int ib) {
    bool na = va != va, nb = vb != vb;
    if (na || nb) {
        if (na && nb) return ia < ib;
        return na;
    }
    if (va != vb) return va > vb;
    return ia < ib;
}

constexpr int PANEL_THREADS = 1024;
constexpr int PANEL_MAX_NB = 1024;

// One workgroup factors the panel A[0:rows, 0:jb] (global row offset row0)
// column by column.  Data stay in global memory (the panel is re-read from
// L2); all waves of the workgroup share one L1, so barriers order them.
__global__ __launch_bounds__(PANEL_THREADS) void k_panel(double *__restrict__ A,
                                                         long long lda, int rows,
                                                         int jb, int *ipiv,
                                                         int row0, int *info) {
    __shared__ double prow[PANEL_MAX_NB];
    __shared__ double red_v[PANEL_THREADS / 64];
    __shared__ int red_i[PANEL_THREADS / 64];
    __shared__ int s_p;
    __shared__ double s_piv;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int ncol = rows < jb ? rows : jb;

    for (int c = 0; c < ncol; ++c) {
        double *colc = A + (long long)c * lda;
        // 1. pivot search over rows c..rows-1
        double bv = -1.0;
        int bi = INT_MAX;
        for (int i = c + tid; i < rows; i += PANEL_THREADS) {
            double v = fabs(colc[i]);
            if (better(v, i, bv, bi)) { bv = v; bi = i; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            double ov = __shfl_xor(bv, off, 64);
            int oi = __shfl_xor(bi, off, 64);
            if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { red_v[wid] = bv; red_i[wid] = bi; }
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < PANEL_THREADS / 64; ++q)
                if (better(red_v[q], red_i[q], bv, bi)) { bv = red_v[q]; bi = red_i[q]; }
            double piv = colc[bi];
            ipiv[c] = row0 + bi + 1;
            if (piv == 0.0 && *info == 0) *info = row0 + c + 1;
            s_p = bi;
            s_piv = piv;
        }
        __syncthreads();
        const int p = s_p;
        const double piv = s_piv;
        if (piv != 0.0) {
            // 2. interchange rows c and p across the panel
            if (p != c) {
                for (int j = tid; j < jb; j += PANEL_THREADS) {
                    double *a = A + (long long)j * lda;
                    double t0 = a[c];
                    a[c] = a[p];
                    a[p] = t0;
                }
            }
            __syncthreads();
            // 3. scale the column below the pivot
            if (fabs(piv) >= DBL_MIN) {
                const double rp = 1.0 / piv;
                for (int i = c + 1 + tid; i < rows; i += PANEL_THREADS) colc[i] = colc[i] * rp;
            } else {
                for (int i = c + 1 + tid; i < rows; i += PANEL_THREADS) colc[i] = colc[i] / piv;
            }
        }
        // 4. rank-1 update of the trailing panel columns
        for (int j = c + 1 + tid; j < jb; j += PANEL_THREADS) prow[j] = A[c + (long long)j * lda];
        __syncthreads();
        for (int i = c + 1 + tid; i < rows; i += PANEL_THREADS) {
            const double l = colc[i];
            for (int j = c + 1; j < jb; ++j) {
                double *a = A + i + (long long)j * lda;
                *a = *a - l * prow[j];
            }
        }
        __syncthreads();
    }
}

int launch_panel(double *A, long long lda, int rows, int jb, int *ipiv, int row0,
                 int *info, hipStream_t stream) {
    if (jb > PANEL_MAX_NB) {
        set_error("panel width %d above %d", jb, PANEL_MAX_NB);
        return EMU_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL(k_panel, dim3(1), dim3(PANEL_THREADS), 0, stream, A, lda, rows,
                       jb, ipiv, row0, info);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------- laswp
// Thread per column: columns [0, ncols_left) and [col_right, col_right +
// ncols_right); interchanges ipiv[k1..k2) applied in order.
__global__ void k_laswp(double *__restrict__ A, long long lda, int nrows,
                        int ncols_left, int col_right, int ncols_right,
                        const int *__restrict__ ipiv, int k1, int k2) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncols_left + ncols_right) return;
    int col = t < ncols_left ? t : col_right + (t - ncols_left);
    double *a = A + (long long)col * lda;
    for (int c = k1; c < k2; ++c) {
        int p = ipiv[c] - 1;
        if (p > c && p < nrows) {
            double t0 = a[c];
            a[c] = a[p];
            a[p] = t0;
        }
    }
}

int launch_laswp(double *A, long long lda, int nrows, int ncols_left, int col_right,
                 int ncols_right, const int *ipiv, int k1, int k2,
                 hipStream_t stream) {
    int total = ncols_left + ncols_right;
    if (total <= 0 || k2 <= k1) return 0;
    hipLaunchKernelGGL(k_laswp, dim3((total + 255) / 256), dim3(256), 0, stream, A,
                       lda, nrows, ncols_left, col_right, ncols_right, ipiv, k1, k2);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ----------------------------------------------------------------- trsm
// B (jb x ncols) <- L^-1 B, L unit lower (jb x jb).  Thread per column;
// for k increasing, b_i = b_i - l_ik b_k (i > k).  NB >= jb: the column
// lives in registers and L in LDS.
template <int NB>
__global__ __launch_bounds__(256) void k_trsm_reg(const double *__restrict__ L,
                                                  long long ldl, int jb,
                                                  double *__restrict__ B,
                                                  long long ldb, int ncols) {
    __shared__ double Ls[NB * NB];
    for (int idx = threadIdx.x; idx < jb * jb; idx += blockDim.x) {
        int i = idx % jb, k = idx / jb;
        Ls[k * NB + i] = L[i + (long long)k * ldl];
    }
    __syncthreads();
    int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    double *bcol = B + (long long)col * ldb;
    double b[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i] = i < jb ? bcol[i] : 0.0;
#pragma unroll
    for (int k = 0; k < NB - 1; ++k) {
        if (k < jb - 1) {
            const double bk = b[k];
#pragma unroll
            for (int i = k + 1; i < NB; ++i)
                if (i < jb) b[i] = b[i] - Ls[k * NB + i] * bk;
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
        if (i < jb) bcol[i] = b[i];
}

__global__ __launch_bounds__(256) void k_trsm_gen(const double *__restrict__ L,
                                                  long long ldl, int jb,
                                                  double *__restrict__ B,
                                                  long long ldb, int ncols) {
    int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    double *bcol = B + (long long)col * ldb;
    for (int k = 0; k < jb - 1; ++k) {
        const double bk = bcol[k];
        const double *lk = L + (long long)k * ldl;
        for (int i = k + 1; i < jb; ++i) bcol[i] = bcol[i] - lk[i] * bk;
    }
}

int launch_trsm_llnu(const double *L, long long ldl, int jb, double *B, long long ldb,
                     int ncols, hipStream_t stream) {
    if (ncols <= 0 || jb <= 1) return 0;
    dim3 grid((ncols + 255) / 256);
    if (jb <= 32)
        hipLaunchKernelGGL(k_trsm_reg<32>, grid, dim3(256), 0, stream, L, ldl, jb, B,
                           ldb, ncols);
    else if (jb <= 64)
        hipLaunchKernelGGL(k_trsm_reg<64>, grid, dim3(256), 0, stream, L, ldl, jb, B,
                           ldb, ncols);
    else
        hipLaunchKernelGGL(k_trsm_gen, grid, dim3(256), 0, stream, L, ldl, jb, B, ldb,
                           ncols);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------- getrs
// The row interchanges of the whole factorization are composed into one
// gather permutation by a single thread (they are sequential by definition),
// then each right-hand side is gathered.
__global__ void k_perm_from_ipiv(const int *__restrict__ ipiv, int n, int *perm) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int c = 0; c < n; ++c) {
        int p = ipiv[c] - 1;
        if (p > c && p < n) {       // valid interchanges satisfy c <= p < n
            int t = perm[c];
            perm[c] = perm[p];
            perm[p] = t;
        }
    }
}

// X (n x nrhs, scratch, leading dimension n) <- P B
__global__ void k_gather_rows(const double *__restrict__ B, long long ldb, int n,
                              const int *__restrict__ perm, double *__restrict__ X) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i < n) X[i + (long long)j * n] = B[perm[i] + (long long)j * ldb];
}

__global__ void k_copy_cols(const double *__restrict__ X, int n, double *__restrict__ B,
                            long long ldb) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i < n) B[i + (long long)j * ldb] = X[i + (long long)j * n];
}

constexpr int TRSV_NB = 64;

// Forward substitution, diagonal block [k0, k0+kb): one wave per rhs; lane
// i holds x_{k0+i}; for k increasing, lanes i > k subtract l_ik x_k.
__global__ __launch_bounds__(64) void k_fwd_diag(const double *__restrict__ LU,
                                                 long long lda, int n, int k0, int kb,
                                                 double *__restrict__ X) {
    const int lane = threadIdx.x;
    double *x = X + (long long)blockIdx.x * n;
    const int i = k0 + lane;
    double b = lane < kb ? x[i] : 0.0;
    for (int k = 0; k < kb - 1; ++k) {
        const double xk = __shfl(b, k, 64);
        if (lane > k && lane < kb) b = b - LU[i + (long long)(k0 + k) * lda] * xk;
    }
    if (lane < kb) x[i] = b;
}

// Rows [r0, r1) after the diagonal block: x_i -= l_ik x_k, k increasing.
__global__ __launch_bounds__(256) void k_fwd_update(const double *__restrict__ LU,
                                                    long long lda, int n, int k0,
                                                    int kb, int r0,
                                                    double *__restrict__ X) {
    __shared__ double xs[TRSV_NB];
    double *x = X + (long long)blockIdx.y * n;
    if (threadIdx.x < kb) xs[threadIdx.x] = x[k0 + threadIdx.x];
    __syncthreads();
    const int i = r0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double b = x[i];
    for (int k = 0; k < kb; ++k) b = b - LU[i + (long long)(k0 + k) * lda] * xs[k];
    x[i] = b;
}

// Back substitution, diagonal block [k0, k0+kb): for k decreasing,
// x_k = b_k / u_kk, then lanes i < k subtract u_ik x_k.
__global__ __launch_bounds__(64) void k_bwd_diag(const double *__restrict__ LU,
                                                 long long lda, int n, int k0, int kb,
                                                 double *__restrict__ X) {
    const int lane = threadIdx.x;
    double *x = X + (long long)blockIdx.x * n;
    const int i = k0 + lane;
    double b = lane < kb ? x[i] : 0.0;
    for (int k = kb - 1; k >= 0; --k) {
        if (lane == k) b = b / LU[i + (long long)i * lda];
        const double xk = __shfl(b, k, 64);
        if (lane < k) b = b - LU[i + (long long)(k0 + k) * lda] * xk;
    }
    if (lane < kb) x[i] = b;
}

// Rows [0, k0) above the diagonal block: x_i -= u_ik x_k, k decreasing.
__global__ __launch_bounds__(256) void k_bwd_update(const double *__restrict__ LU,
                                                    long long lda, int n, int k0,
                                                    int kb, double *__restrict__ X) {
    __shared__ double xs[TRSV_NB];
    double *x = X + (long long)blockIdx.y * n;
    if (threadIdx.x < kb) xs[threadIdx.x] = x[k0 + threadIdx.x];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k0) return;
    double b = x[i];
    for (int k = kb - 1; k >= 0; --k) b = b - LU[i + (long long)(k0 + k) * lda] * xs[k];
    x[i] = b;
}

int launch_getrs(int n, int nrhs, const double *LU, long long lda, const int *ipiv,
                 double *B, long long ldb, int *perm_ws, hipStream_t stream) {
    if (n <= 0 || nrhs <= 0) return 0;
    int *perm = perm_ws;
    double *X = reinterpret_cast<double *>(
        reinterpret_cast<char *>(perm_ws) + align256((size_t)n * sizeof(int)));
    hipLaunchKernelGGL(k_perm_from_ipiv, dim3(1), dim3(64), 0, stream, ipiv, n, perm);
    dim3 gcol((n + 255) / 256, nrhs);
    hipLaunchKernelGGL(k_gather_rows, gcol, dim3(256), 0, stream, B, ldb, n, perm, X);
    for (int k0 = 0; k0 < n; k0 += TRSV_NB) {
        int kb = n - k0 < TRSV_NB ? n - k0 : TRSV_NB;
        hipLaunchKernelGGL(k_fwd_diag, dim3(nrhs), dim3(64), 0, stream, LU, lda, n, k0,
                           kb, X);
        int r0 = k0 + kb;
        if (r0 < n) {
            dim3 g((n - r0 + 255) / 256, nrhs);
            hipLaunchKernelGGL(k_fwd_update, g, dim3(256), 0, stream, LU, lda, n, k0, kb,
                               r0, X);
        }
    }
    int last0 = (n - 1) / TRSV_NB * TRSV_NB;
    for (int k0 = last0; k0 >= 0; k0 -= TRSV_NB) {
        int kb = n - k0 < TRSV_NB ? n - k0 : TRSV_NB;
        hipLaunchKernelGGL(k_bwd_diag, dim3(nrhs), dim3(64), 0, stream, LU, lda, n, k0,
                           kb, X);
        if (k0 > 0) {
            dim3 g((k0 + 255) / 256, nrhs);
            hipLaunchKernelGGL(k_bwd_update, g, dim3(256), 0, stream, LU, lda, n, k0, kb,
                               X);
        }
    }
    hipLaunchKernelGGL(k_copy_cols, gcol, dim3(256), 0, stream, X, n, B, ldb);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

}  // namespace emu
