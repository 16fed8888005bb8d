// FP64 panel factorization and triangular solves of the blocked LU
// (paper: section "Dense Numerical Solvers Using FP64 Emulation": the panel,
// where partial pivoting picks the pivots and U11^-1 reaches A21, stays in
// FP64 custom code; eqn (8)'s Schur update is the only emulated step).
//
// Every update is one rounded product and one rounded subtraction (this
// library is compiled with -ffp-contract=off), and every element receives
// its updates in increasing elimination order, with whole-row interchanges.
// The results are therefore bit-identical to a plain column-by-column
// right-looking elimination of the panel, while the work is organised for
// the GPU:
//
//   * recursion: a panel of width w factors its left part, applies the left
//     part's interchanges to its right part, solves the top of the right part
//     (unit lower triangle), updates the rest of the right part with an
//     order-preserving FP64 tile kernel (k_gemm_seq: for each k in order,
//     c = c - a_ik b_kj), factors the right part, and moves the left part's
//     rows by the right part's interchanges;
//   * leaves of at most 16 columns: up to 2048 rows in one workgroup with
//     the block in registers (2 rows x 16 columns per thread); taller leaves
//     one launch per column over 1024-row workgroups, each launch finishing
//     column c (interchange, scaling, rank-1 update) and publishing the
//     workgroup's pivot candidate for column c + 1 together with a copy of
//     that candidate row, so the next launch needs no other synchronisation.
#include "common.h"
#include "devutil.h"

#include <float.h>

namespace emu {

constexpr int LEAF_W = 16;
constexpr int L1_THREADS = 1024;
constexpr int L1_R = 2;                      // rows per thread
constexpr int L1_ROWS = L1_THREADS * L1_R;   // 2048
constexpr int LC_THREADS = 256;
constexpr int LC_ROWS = 1024;                // rows per workgroup (4 per thread)
constexpr int LC_MAX_G = 64;                 // workgroups of one tall leaf (65536 rows)

// ------------------------------------------------- register-resident leaf
// P: top-left of the leaf block (global row grow0), rows x w, w <= 16.  The
// column loop is not unrolled (runtime column index, register selects) to
// keep the code small enough for the instruction cache.
__global__ __launch_bounds__(L1_THREADS) void k_leaf1(double *__restrict__ P, long long lda,
                                                      int rows, int w, int *ipiv, int grow0,
                                                      int *info) {
    __shared__ double urow[LEAF_W], xrow[LEAF_W];
    __shared__ double red_v[L1_THREADS / 64 + 1];
    __shared__ int red_i[L1_THREADS / 64 + 1];
    const int t = threadIdx.x;
    double v[L1_R][LEAF_W];
#pragma unroll
    for (int q = 0; q < L1_R; ++q) {
        const int i = t + q * L1_THREADS;
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j)
            v[q][j] = (i < rows && j < w) ? P[i + (long long)j * lda] : 0.0;
    }
#pragma unroll 1
    for (int c = 0; c < w; ++c) {
        double bv = -1.0;
        int bi = INT_MAX;
#pragma unroll
        for (int q = 0; q < L1_R; ++q) {
            const int i = t + q * L1_THREADS;
            double vc = 0.0;
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j)
                if (j == c) vc = v[q][j];
            if (i >= c && i < rows && better(fabs(vc), i, bv, bi)) {
                bv = fabs(vc);
                bi = i;
            }
        }
        block_best<L1_THREADS / 64>(bv, bi, red_v, red_i);
        const int p = bi;
#pragma unroll
        for (int q = 0; q < L1_R; ++q) {
            const int i = t + q * L1_THREADS;
            if (i == p)
#pragma unroll
                for (int j = 0; j < LEAF_W; ++j) urow[j] = v[q][j];
            if (i == c)
#pragma unroll
                for (int j = 0; j < LEAF_W; ++j) xrow[j] = v[q][j];
        }
        __syncthreads();
        const double piv = urow[c];
        if (t == 0) {
            ipiv[c] = grow0 + p + 1;
            if (piv == 0.0 && *info == 0) *info = grow0 + c + 1;
        }
        const bool swap = piv != 0.0 && p != c;
        // row c after the interchange (the old row c when there is none),
        // read from LDS where it is used
        const double *ur = (piv != 0.0) ? urow : xrow;
        const bool recip = fabs(piv) >= DBL_MIN;
        const double rp = 1.0 / piv;
#pragma unroll
        for (int q = 0; q < L1_R; ++q) {
            const int i = t + q * L1_THREADS;
            if (swap && i == c) {
#pragma unroll
                for (int j = 0; j < LEAF_W; ++j) v[q][j] = urow[j];
            } else if (swap && i == p) {
#pragma unroll
                for (int j = 0; j < LEAF_W; ++j) v[q][j] = xrow[j];
            }
            if (i > c && i < rows) {
                double l = 0.0;
#pragma unroll
                for (int j = 0; j < LEAF_W; ++j)
                    if (j == c) l = v[q][j];
                if (piv != 0.0) l = recip ? l * rp : l / piv;
#pragma unroll
                for (int j = 0; j < LEAF_W; ++j) {
                    if (j == c) v[q][j] = l;
                    if (j > c) v[q][j] = v[q][j] - l * ur[j];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < L1_R; ++q) {
        const int i = t + q * L1_THREADS;
        if (i < rows)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j)
                if (j < w) P[i + (long long)j * lda] = v[q][j];
    }
}

// ------------------------------------------------- per-column tall leaf
// Buffers of one column step: per workgroup its best candidate (value,
// row) and a copy of that row; plus a copy of row c itself.
struct LeafBuf {
    double *cval;   // [G]
    int *cidx;      // [G]
    double *crow;   // [G][16]
    double *rowc;   // [16]
};

__device__ __forceinline__ void publish_candidate(const double *__restrict__ P, long long lda,
                                                  int w, double bv, int bi, LeafBuf out,
                                                  double *red_v, int *red_i) {
    const int t = threadIdx.x;
    block_best<LC_THREADS / 64>(bv, bi, red_v, red_i);
    if (t == 0) {
        out.cval[blockIdx.x] = bv;
        out.cidx[blockIdx.x] = bi;
    }
    if (bi != INT_MAX && t < LEAF_W)
        out.crow[blockIdx.x * LEAF_W + t] = (t < w) ? P[bi + (long long)t * lda] : 0.0;
}

// Candidates for column 0 and a copy of row 0.
__global__ __launch_bounds__(LC_THREADS) void k_leafc_init(const double *__restrict__ P,
                                                           long long lda, int rows, int w,
                                                           LeafBuf out) {
    __shared__ double red_v[LC_THREADS / 64 + 1];
    __shared__ int red_i[LC_THREADS / 64 + 1];
    const int t = threadIdx.x;
    const int r0 = blockIdx.x * LC_ROWS;
    const int r1 = min(rows, r0 + LC_ROWS);
    double bv = -1.0;
    int bi = INT_MAX;
    for (int i = r0 + t; i < r1; i += LC_THREADS) {
        const double a = fabs(P[i]);
        if (better(a, i, bv, bi)) {
            bv = a;
            bi = i;
        }
    }
    if (blockIdx.x == 0 && t < LEAF_W) out.rowc[t] = (t < w) ? P[(long long)t * lda] : 0.0;
    publish_candidate(P, lda, w, bv, bi, out, red_v, red_i);
}

// Finish column c of the leaf; publish candidates for column c + 1.
// Each thread owns rows r0 + t + 256 q (q < 4) of its workgroup's 1024.
// All inputs (own rows, the G candidates with their rows, row c) are
// loaded up front, so a launch costs one memory round trip.
__global__ __launch_bounds__(LC_THREADS) void k_leafc(double *__restrict__ P, long long lda,
                                                      int rows, int w, int c, int *ipiv,
                                                      int grow0, int *info, int G,
                                                      LeafBuf in, LeafBuf out) {
    constexpr int Q = LC_ROWS / LC_THREADS;
    __shared__ double crow[LC_MAX_G * LEAF_W];
    __shared__ double xr[LEAF_W];
    __shared__ double red_v[LC_THREADS / 64 + 1];
    __shared__ int red_i[LC_THREADS / 64 + 1];
    __shared__ int s_g;
    const int t = threadIdx.x;
    const int r0 = blockIdx.x * LC_ROWS;
    double v[Q][LEAF_W];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = r0 + t + LC_THREADS * q;
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j)
            v[q][j] = (i >= c && i < rows && j < w) ? P[i + (long long)j * lda] : 0.0;
    }
    for (int e = t; e < G * LEAF_W; e += LC_THREADS) crow[e] = in.crow[e];
    if (t < LEAF_W) xr[t] = in.rowc[t];
    double bv = -1.0;
    int bi = INT_MAX;
    if (t < G) {
        bv = in.cval[t];
        bi = in.cidx[t];
    }
    if (t == 0) s_g = 0;
    block_best<LC_THREADS / 64>(bv, bi, red_v, red_i);   // includes barriers
    const int p = bi;
    if (t < G && in.cidx[t] == p) s_g = t;
    __syncthreads();
    const double *urp = crow + s_g * LEAF_W;
    const double piv = urp[c];
    if (piv == 0.0) urp = xr;                            // no interchange: row c stays
    if (blockIdx.x == 0 && t == 0) {
        ipiv[c] = grow0 + p + 1;
        if (piv == 0.0 && *info == 0) *info = grow0 + c + 1;
    }
    double ur[LEAF_W];
#pragma unroll
    for (int j = 0; j < LEAF_W; ++j) ur[j] = urp[j];
    const bool swap = piv != 0.0 && p != c;
    const bool recip = fabs(piv) >= DBL_MIN;
    const double rp = 1.0 / piv;
    double nbv = -1.0;
    int nbi = INT_MAX;
    double best[LEAF_W];
#pragma unroll
    for (int j = 0; j < LEAF_W; ++j) best[j] = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int i = r0 + t + LC_THREADS * q;
        if (i < c || i >= rows) continue;
        if (swap && i == c) {
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) v[q][j] = ur[j];
        } else if (swap && i == p) {
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) v[q][j] = xr[j];
        }
        if (i > c) {
            double l = 0.0;
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j)
                if (j == c) l = v[q][j];
            if (piv != 0.0) l = recip ? l * rp : l / piv;
            double nx = 0.0;
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) {
                if (j == c) v[q][j] = l;
                if (j > c) v[q][j] = v[q][j] - l * ur[j];
                if (j == c + 1) nx = v[q][j];
            }
            if (c + 1 < w && better(fabs(nx), i, nbv, nbi)) {
                nbv = fabs(nx);
                nbi = i;
#pragma unroll
                for (int j = 0; j < LEAF_W; ++j) best[j] = v[q][j];
            }
        }
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j)
            if (j < w) P[i + (long long)j * lda] = v[q][j];
        if (i == c + 1 && c + 1 < w)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) out.rowc[j] = v[q][j];
    }
    if (c + 1 < w) {
        const int mine = nbi;
        block_best<LC_THREADS / 64>(nbv, nbi, red_v, red_i);
        if (t == 0) {
            out.cval[blockIdx.x] = nbv;
            out.cidx[blockIdx.x] = nbi;
        }
        if (nbi != INT_MAX && mine == nbi)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) out.crow[blockIdx.x * LEAF_W + j] = best[j];
    }
}

// --------------------------------------------- order-preserving FP64 tiles
// C (m x n) -= A (m x k) B (k x n): every element c_ij is updated for k in
// increasing order as c = c - a_ik b_kj (two roundings), as in elimination.
constexpr int GS_T = 64, GS_K = 16;
__global__ __launch_bounds__(256) void k_gemm_seq(const double *__restrict__ A, long long lda,
                                                  const double *__restrict__ B, long long ldb,
                                                  double *__restrict__ C, long long ldc, int m,
                                                  int n, int k) {
    __shared__ double As[GS_K][GS_T + 1];
    __shared__ double Bs[GS_K][GS_T + 1];
    const int t = threadIdx.x;
    const int tr = t % 16, tc = t / 16;          // 16 x 16 threads, 4 x 4 each
    const int m0 = blockIdx.x * GS_T, n0 = blockIdx.y * GS_T;
    double c[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = m0 + tr + 16 * r, j = n0 + tc + 16 * s;
            c[r][s] = (i < m && j < n) ? C[i + (long long)j * ldc] : 0.0;
        }
    for (int k0 = 0; k0 < k; k0 += GS_K) {
        for (int e = t; e < GS_T * GS_K; e += 256) {
            const int ii = e % GS_T, kk = e / GS_T;
            const int i = m0 + ii, kx = k0 + kk;
            As[kk][ii] = (i < m && kx < k) ? A[i + (long long)kx * lda] : 0.0;
        }
        for (int e = t; e < GS_T * GS_K; e += 256) {
            const int kk = e % GS_K, jj = e / GS_K;
            const int j = n0 + jj, kx = k0 + kk;
            Bs[kk][jj] = (j < n && kx < k) ? B[kx + (long long)j * ldb] : 0.0;
        }
        __syncthreads();
        const int kend = min(GS_K, k - k0);
        for (int kk = 0; kk < kend; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][tr + 16 * r];
#pragma unroll
            for (int s = 0; s < 4; ++s) b[s] = Bs[kk][tc + 16 * s];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int s = 0; s < 4; ++s) c[r][s] = c[r][s] - a[r] * b[s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = m0 + tr + 16 * r, j = n0 + tc + 16 * s;
            if (i < m && j < n) C[i + (long long)j * ldc] = c[r][s];
        }
}

static int gemm_seq(const double *A, long long lda, const double *B, long long ldb, double *C,
                    long long ldc, int m, int n, int k, hipStream_t st) {
    if (m <= 0 || n <= 0 || k <= 0) return 0;
    dim3 g((m + GS_T - 1) / GS_T, (n + GS_T - 1) / GS_T);
    hipLaunchKernelGGL(k_gemm_seq, g, dim3(256), 0, st, A, lda, B, ldb, C, ldc, m, n, k);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------- unit-lower TRSM
// B (jb x ncols) <- L^-1 B for jb <= 64: thread per column, the column in
// registers, L in LDS; for k increasing, b_i = b_i - l_ik b_k (i > k).
template <int NB>
__global__ __launch_bounds__(256) void k_trsm_reg(const double *__restrict__ L, long long ldl,
                                                  int jb, double *__restrict__ B, long long ldb,
                                                  int ncols) {
    __shared__ double Ls[NB * NB];
    for (int idx = threadIdx.x; idx < jb * jb; idx += blockDim.x) {
        const int i = idx % jb, k = idx / jb;
        Ls[k * NB + i] = L[i + (long long)k * ldl];
    }
    __syncthreads();
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
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

// Blocked: 64-row diagonal solves, order-preserving tile updates between.
int launch_trsm_llnu(const double *L, long long ldl, int jb, double *B, long long ldb,
                     int ncols, hipStream_t stream) {
    if (ncols <= 0 || jb <= 1) return 0;
    constexpr int D = 64;
    for (int k0 = 0; k0 < jb; k0 += D) {
        const int kb = jb - k0 < D ? jb - k0 : D;
        dim3 grid((ncols + 255) / 256);
        const double *Lkk = L + k0 + (long long)k0 * ldl;
        double *Bk = B + k0;
        if (kb > 1) {
            if (kb <= 32)
                hipLaunchKernelGGL(k_trsm_reg<32>, grid, dim3(256), 0, stream, Lkk, ldl, kb,
                                   Bk, ldb, ncols);
            else
                hipLaunchKernelGGL(k_trsm_reg<64>, grid, dim3(256), 0, stream, Lkk, ldl, kb,
                                   Bk, ldb, ncols);
            EMU_TRY_HIP(hipGetLastError());
        }
        const int below = jb - (k0 + kb);
        if (below > 0)
            EMU_TRY(gemm_seq(L + (k0 + kb) + (long long)k0 * ldl, ldl, Bk, ldb,
                             B + k0 + kb, ldb, below, ncols, kb, stream));
    }
    return 0;
}

// ------------------------------------------------------------ recursion
size_t panel_scratch_bytes(int rows) {
    const int G = (rows + LC_ROWS - 1) / LC_ROWS;
    return 2 * (align256((size_t)G * sizeof(double)) + align256((size_t)G * sizeof(int)) +
                align256((size_t)G * LEAF_W * sizeof(double)) +
                align256(LEAF_W * sizeof(double)));
}

static LeafBuf leaf_buf(char *ws, int G, int which) {
    const size_t one = align256((size_t)G * sizeof(double)) + align256((size_t)G * sizeof(int)) +
                       align256((size_t)G * LEAF_W * sizeof(double)) +
                       align256(LEAF_W * sizeof(double));
    char *p = ws + which * one;
    LeafBuf b;
    b.cval = reinterpret_cast<double *>(p);
    p += align256((size_t)G * sizeof(double));
    b.cidx = reinterpret_cast<int *>(p);
    p += align256((size_t)G * sizeof(int));
    b.crow = reinterpret_cast<double *>(p);
    p += align256((size_t)G * LEAF_W * sizeof(double));
    b.rowc = reinterpret_cast<double *>(p);
    return b;
}

static int leaf(double *P, long long lda, int rows, int w, int *ipiv, int grow0, int *info,
                char *ws, hipStream_t st) {
    if (rows <= L1_ROWS) {
        hipLaunchKernelGGL(k_leaf1, dim3(1), dim3(L1_THREADS), 0, st, P, lda, rows, w, ipiv,
                           grow0, info);
        EMU_TRY_HIP(hipGetLastError());
        return 0;
    }
    const int G = (rows + LC_ROWS - 1) / LC_ROWS;
    if (G > LC_MAX_G) {
        set_error("panel of %d rows above %d", rows, LC_MAX_G * LC_ROWS);
        return EMU_ERR_UNSUPPORTED;
    }
    LeafBuf b0 = leaf_buf(ws, G, 0), b1 = leaf_buf(ws, G, 1);
    hipLaunchKernelGGL(k_leafc_init, dim3(G), dim3(LC_THREADS), 0, st, P, lda, rows, w, b0);
    for (int c = 0; c < w; ++c) {
        const LeafBuf &in = (c & 1) ? b1 : b0;
        const LeafBuf &out = (c & 1) ? b0 : b1;
        hipLaunchKernelGGL(k_leafc, dim3(G), dim3(LC_THREADS), 0, st, P, lda, rows, w, c, ipiv,
                           grow0, info, G, in, out);
    }
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// Factor columns [c0, c0 + w) of the panel whose top-left is A (global row
// and column row0), rows [c0, m_rows) of it; ipiv/info as in getrf.
static int panel_rec(double *A, long long lda, int m_rows, int c0, int w, int *ipiv, int row0,
                     int *info, char *ws, hipStream_t st) {
    double *P = A + c0 + (long long)c0 * lda;
    if (w <= LEAF_W)
        return leaf(P, lda, m_rows - c0, w, ipiv + c0, row0 + c0, info, ws, st);
    int w1 = (w / 2) / LEAF_W * LEAF_W;
    if (w1 < LEAF_W) w1 = LEAF_W;
    const int w2 = w - w1;
    EMU_TRY(panel_rec(A, lda, m_rows, c0, w1, ipiv, row0, info, ws, st));
    // interchanges of the left part on the right part's rows
    EMU_TRY(launch_laswp(A, lda, m_rows, 0, c0 + w1, w2, ipiv, c0, c0 + w1, row0, st));
    // U of the right part's top, then the rest of the right part
    EMU_TRY(launch_trsm_llnu(P, lda, w1, P + (long long)w1 * lda, lda, w2, st));
    EMU_TRY(gemm_seq(P + w1, lda, P + (long long)w1 * lda, lda, P + w1 + (long long)w1 * lda,
                     lda, m_rows - c0 - w1, w2, w1, st));
    EMU_TRY(panel_rec(A, lda, m_rows, c0 + w1, w2, ipiv, row0, info, ws, st));
    // interchanges of the right part on the left part's rows
    EMU_TRY(launch_laswp(A, lda, m_rows, 0, c0, w1, ipiv, c0 + w1, c0 + w, row0, st));
    return 0;
}

int launch_panel(double *A, long long lda, int rows, int jb, int *ipiv, int row0, int *info,
                 char *ws, hipStream_t stream) {
    return panel_rec(A, lda, rows, 0, jb, ipiv, row0, info, ws, stream);
}

}  // namespace emu
