// FP64 kernels of the precision form: residual r = b - A x, infinity norms
// and the backward error used by iterative refinement.
//
// Paper: eqn (9) defines the scaled residual ||Ax - b|| / ((||A|| ||x|| +
// ||b||) n eps); refinement is not part of the paper (the precision form is
// this library's own), but its stopping test is that quantity without the
// n eps factor: eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf).
//
// Matrix-vector products read A once per call, coalesced along columns:
// threads own rows, a workgroup walks one chunk of columns and writes its
// partial sums; a second pass adds the chunks in a fixed order (so results
// are reproducible) and forms the residual and the per-column maxima.
// Maxima of non-negative doubles are combined with integer atomicMax on
// their bit patterns, which order the same way.
#include "common.h"

namespace emu {

constexpr int RES_ROWS = 256;      // rows per workgroup
constexpr int RES_COLS = 256;      // columns per chunk
constexpr int RES_MAX_RHS = 8;     // right-hand sides per pass

__device__ __forceinline__ void atomic_max_nonneg(double *p, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(p),
              (unsigned long long)__double_as_longlong(v));
}

// partial[(c*nr + r)*n + i] = sum over columns j of chunk c of A(i,j) X(j,r)
// (absolute values when ABS, with X = ones).
template <bool ABS>
__global__ __launch_bounds__(RES_ROWS) void k_matvec_partial(
    const double *__restrict__ A, long long lda, int n, const double *__restrict__ X,
    long long ldx, int nr, double *__restrict__ partial) {
    __shared__ double xs[RES_COLS * RES_MAX_RHS];
    const int c = blockIdx.y;
    const int j0 = c * RES_COLS;
    const int j1 = min(n, j0 + RES_COLS);
    if (!ABS) {
        for (int t = threadIdx.x; t < RES_COLS * nr; t += blockDim.x) {
            const int jj = t % RES_COLS, r = t / RES_COLS;
            xs[r * RES_COLS + jj] = (j0 + jj < n) ? X[(j0 + jj) + (long long)r * ldx] : 0.0;
        }
        __syncthreads();
    }
    const int i = blockIdx.x * RES_ROWS + threadIdx.x;
    if (i >= n) return;
    double acc[RES_MAX_RHS];
#pragma unroll
    for (int r = 0; r < RES_MAX_RHS; ++r) acc[r] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double a = A[i + (long long)j * lda];
        if (ABS) {
            acc[0] += fabs(a);
        } else {
#pragma unroll
            for (int r = 0; r < RES_MAX_RHS; ++r)
                if (r < nr) acc[r] = fma(a, xs[r * RES_COLS + (j - j0)], acc[r]);
        }
    }
    const int rr = ABS ? 1 : nr;
    for (int r = 0; r < rr; ++r) partial[((long long)c * rr + r) * n + i] = acc[r];
}

// ||A||_inf: out[0] = max_i sum_c partial[c][i]   (out[0] preset to 0)
__global__ __launch_bounds__(256) void k_rowsum_max(const double *__restrict__ partial,
                                                    int n, int nchunks, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < n)
        for (int c = 0; c < nchunks; ++c) s += partial[(long long)c * n + i];
    for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off, 64));
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, s);
}

// R = B - sum_c partial[c]; stats[3*r + {0,1,2}] = max |R|, max |X|, max |B|
// for right-hand side r (stats preset to 0).
__global__ __launch_bounds__(256) void k_resid_reduce(
    const double *__restrict__ partial, int n, int nr, int nchunks,
    const double *__restrict__ B, long long ldb, const double *__restrict__ X,
    long long ldx, double *__restrict__ R, long long ldr, double *stats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    double ar = 0.0, ax = 0.0, ab = 0.0;
    if (i < n) {
        double s = 0.0;
        for (int c = 0; c < nchunks; ++c) s += partial[((long long)c * nr + r) * n + i];
        const double b = B[i + (long long)r * ldb];
        const double res = b - s;
        R[i + (long long)r * ldr] = res;
        ar = fabs(res);
        ax = fabs(X[i + (long long)r * ldx]);
        ab = fabs(b);
    }
    for (int off = 32; off > 0; off >>= 1) {
        ar = fmax(ar, __shfl_xor(ar, off, 64));
        ax = fmax(ax, __shfl_xor(ax, off, 64));
        ab = fmax(ab, __shfl_xor(ab, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomic_max_nonneg(stats + 3 * r + 0, ar);
        atomic_max_nonneg(stats + 3 * r + 1, ax);
        atomic_max_nonneg(stats + 3 * r + 2, ab);
    }
}

__global__ void k_fill_double(double *p, double v, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// X(:, r) += D(:, r)
__global__ void k_add_cols(double *__restrict__ X, long long ldx,
                           const double *__restrict__ D, long long ldd, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i < n) X[i + (long long)r * ldx] += D[i + (long long)r * ldd];
}

// dst(:, 0:cols) = src(:, 0:cols), both column-major with n rows
__global__ void k_copy_mat(const double *__restrict__ src, long long lds_, double *__restrict__ dst,
                           long long ldd, int n, int cols) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * cols) return;
    const int i = (int)(idx % n), j = (int)(idx / n);
    dst[i + (long long)j * ldd] = src[i + (long long)j * lds_];
}

int refine_chunks(int n) { return (n + RES_COLS - 1) / RES_COLS; }

size_t refine_partial_bytes(int n, int nrhs) {
    const int nr = nrhs < RES_MAX_RHS ? nrhs : RES_MAX_RHS;
    return (size_t)refine_chunks(n) * (nr > 1 ? nr : 1) * n * sizeof(double);
}

int launch_norm_inf(const double *A, long long lda, int n, double *partial, double *out,
                    hipStream_t stream) {
    hipLaunchKernelGGL(k_fill_double, dim3(1), dim3(64), 0, stream, out, 0.0, 1);
    dim3 g((n + RES_ROWS - 1) / RES_ROWS, refine_chunks(n));
    hipLaunchKernelGGL((k_matvec_partial<true>), g, dim3(RES_ROWS), 0, stream, A, lda, n,
                       (const double *)nullptr, 0LL, 1, partial);
    hipLaunchKernelGGL(k_rowsum_max, dim3((n + 255) / 256), dim3(256), 0, stream, partial,
                       n, refine_chunks(n), out);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// R = B - A X for nrhs right-hand sides (in passes of RES_MAX_RHS), and
// stats[3r..3r+2] = (max|R|, max|X|, max|B|) per right-hand side.
int launch_residual(const double *A, long long lda, int n, const double *X, long long ldx,
                    const double *B, long long ldb, int nrhs, double *R, long long ldr,
                    double *partial, double *stats, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill_double, dim3((3 * nrhs + 255) / 256), dim3(256), 0, stream,
                       stats, 0.0, 3 * nrhs);
    const int nch = refine_chunks(n);
    for (int r0 = 0; r0 < nrhs; r0 += RES_MAX_RHS) {
        const int nr = nrhs - r0 < RES_MAX_RHS ? nrhs - r0 : RES_MAX_RHS;
        dim3 g((n + RES_ROWS - 1) / RES_ROWS, nch);
        hipLaunchKernelGGL((k_matvec_partial<false>), g, dim3(RES_ROWS), 0, stream, A, lda,
                           n, X + (long long)r0 * ldx, ldx, nr, partial);
        dim3 g2((n + 255) / 256, nr);
        hipLaunchKernelGGL(k_resid_reduce, g2, dim3(256), 0, stream, partial, n, nr, nch,
                           B + (long long)r0 * ldb, ldb, X + (long long)r0 * ldx, ldx,
                           R + (long long)r0 * ldr, ldr, stats + 3 * r0);
    }
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_add_cols(double *X, long long ldx, const double *D, long long ldd, int n,
                    int nrhs, hipStream_t stream) {
    dim3 g((n + 255) / 256, nrhs);
    hipLaunchKernelGGL(k_add_cols, g, dim3(256), 0, stream, X, ldx, D, ldd, n);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_copy_mat(const double *src, long long lds_, double *dst, long long ldd, int n,
                    int cols, hipStream_t stream) {
    const long long total = (long long)n * cols;
    if (total == 0) return 0;
    hipLaunchKernelGGL(k_copy_mat, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       stream, src, lds_, dst, ldd, n, cols);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

}  // namespace emu
