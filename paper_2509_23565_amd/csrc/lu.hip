// Row interchanges and the triangular solves of getrs (paper: eqn (5), the
// solve that follows the factorization; the panel and the trailing TRSM are
// in panel.hip).
//
// Every FP64 update here is one rounded product followed by one rounded
// subtraction (this library is compiled with -ffp-contract=off), applied to
// each element in increasing elimination order, so the solutions are
// identical bit for bit to plain column-oriented substitution.
#include "common.h"

namespace emu {

// ---------------------------------------------------------------- laswp
// The interchanges ipiv[k1..k2) (1-based global rows; A's first row is global
// row row0) are composed into one permutation of the rows they touch (at
// most 2 (k2 - k1) rows), then applied to columns [0, ncols_left) and
// [col_right, col_right + ncols_right): every workgroup reads its columns'
// touched rows into LDS and writes them back permuted, so the sequential
// chain of swaps costs no memory round trips.  Consecutive threads take
// consecutive touched rows of one column (the panel's rows are contiguous
// there), not consecutive columns of one row, which lie a leading dimension
// apart.
constexpr int SW_MAX = 1024;          // interchanges per call
constexpr int SW_TILE = 8192;         // doubles of LDS for the row tile

__global__ __launch_bounds__(256) void k_laswp_perm(double *__restrict__ A, long long lda,
                                                    int nrows, int ncols_left, int col_right,
                                                    int ncols_right,
                                                    const int *__restrict__ ipiv, int k1,
                                                    int k2, int row0) {
    __shared__ int pr[SW_MAX];            // target row of interchange c (local)
    __shared__ int pslot[SW_MAX];         // slot of that row
    __shared__ int first[SW_MAX];         // 1 if the row first appears here (outside [k1,k2))
    __shared__ int srow[2 * SW_MAX];      // row of each slot
    __shared__ int content[2 * SW_MAX];   // source row of each slot after all swaps
    __shared__ double tile[SW_TILE];
    __shared__ int s_nslot;
    const int t = threadIdx.x;
    const int J = k2 - k1;
    for (int c = t; c < J; c += blockDim.x) {
        int pv = ipiv[k1 + c] - 1 - row0;
        if (pv < k1 + c || pv >= nrows) pv = k1 + c;       // invalid: no interchange
        pr[c] = pv;
    }
    __syncthreads();
    // first appearance of each target row outside [k1, k2)
    for (int c = t; c < J; c += blockDim.x) {
        const int pv = pr[c];
        int f = (pv >= k2) ? 1 : 0;
        if (f)
            for (int c2 = 0; c2 < c; ++c2)
                if (pr[c2] == pv) {
                    f = 0;
                    break;
                }
        first[c] = f;
    }
    __syncthreads();
    if (t == 0) {
        int nx = 0;
        for (int c = 0; c < J; ++c) {
            srow[c] = k1 + c;
            content[c] = k1 + c;
        }
        for (int c = 0; c < J; ++c) {
            const int pv = pr[c];
            if (pv < k2) {
                pslot[c] = pv - k1;
            } else if (first[c]) {
                pslot[c] = J + nx;
                srow[J + nx] = pv;
                content[J + nx] = pv;
                ++nx;
            } else {
                for (int c2 = 0; c2 < c; ++c2)
                    if (pr[c2] == pv) {
                        pslot[c] = pslot[c2];
                        break;
                    }
            }
        }
        for (int c = 0; c < J; ++c) {        // the interchanges, in order
            const int a = c, b = pslot[c];
            const int x = content[a];
            content[a] = content[b];
            content[b] = x;
        }
        s_nslot = J + nx;
    }
    __syncthreads();
    const int nslot = s_nslot;
    const int CW = max(1, SW_TILE / nslot);                   // columns per pass
    const int ncols = ncols_left + ncols_right;
    for (int cb = blockIdx.x * CW; cb < ncols; cb += gridDim.x * CW) {
        const int cw = min(CW, ncols - cb);
        for (int e = t; e < nslot * cw; e += blockDim.x) {
            const int sl = e % nslot, jj = e / nslot;   // down a column
            const int cidx = cb + jj;
            const int col = cidx < ncols_left ? cidx : col_right + (cidx - ncols_left);
            tile[e] = A[content[sl] + (long long)col * lda];
        }
        __syncthreads();
        for (int e = t; e < nslot * cw; e += blockDim.x) {
            const int sl = e % nslot, jj = e / nslot;   // down a column
            if (content[sl] == srow[sl]) continue;
            const int cidx = cb + jj;
            const int col = cidx < ncols_left ? cidx : col_right + (cidx - ncols_left);
            A[srow[sl] + (long long)col * lda] = tile[e];
        }
        __syncthreads();
    }
}

int launch_laswp(double *A, long long lda, int nrows, int ncols_left, int col_right,
                 int ncols_right, const int *ipiv, int k1, int k2, int row0,
                 hipStream_t stream) {
    const int total = ncols_left + ncols_right;
    if (total <= 0 || k2 <= k1) return 0;
    if (k2 - k1 > SW_MAX) {
        set_error("more than %d interchanges in one call", SW_MAX);
        return EMU_ERR_UNSUPPORTED;
    }
    const int nslot_max = 2 * (k2 - k1);
    const int cw = nslot_max < SW_TILE ? SW_TILE / nslot_max : 1;
    int blocks = (total + cw - 1) / cw;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_laswp_perm, dim3(blocks), dim3(256), 0, stream, A, lda, nrows,
                       ncols_left, col_right, ncols_right, ipiv, k1, k2, row0);
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
