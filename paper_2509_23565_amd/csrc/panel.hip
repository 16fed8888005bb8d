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
//   * leaves of at most 16 columns, the block in registers (2 rows x 16
//     columns per thread, 2048 rows per 1024-thread workgroup).  Each column
//     costs one workgroup barrier: every wave publishes its pivot candidate
//     together with a copy of the candidate row (and the owner of row c a
//     copy of row c) into a double-buffered LDS slot, so after the barrier
//     every wave picks the winner and reads both rows without a second
//     round.  Leaves taller than 2048 rows run as one cooperative launch of
//     up to 32 workgroups that exchange their candidates the same way
//     through global memory, with one grid-wide wait per column (bounded:
//     a wait that exceeds its bound aborts the leaf and raises
//     EMU_STATUS_PANEL_WAIT).
#include "common.h"
#include "devutil.h"

#include <float.h>

namespace emu {

constexpr int LEAF_W = 16;
constexpr int LF_THREADS = 1024;
constexpr int LF_WAVES = LF_THREADS / 64;
constexpr int LF_R = 2;                        // rows per thread
constexpr int LF_ROWS = LF_THREADS * LF_R;     // rows per workgroup
constexpr int LF_MAX_G = 32;                   // workgroups of one leaf (65536 rows)
constexpr int LF_SPIN_LIMIT = 1 << 20;         // polls of one grid-wide wait

// Cross-workgroup exchange of a multi-workgroup leaf (global scratch).
struct LeafX {
    double *val;        // [2][LF_MAX_G] best |value| per workgroup
    int *idx;           // [2][LF_MAX_G] its row
    double *row;        // [2][LF_MAX_G][LEAF_W] a copy of that row
    double *rowc;       // [2][LEAF_W] a copy of row c
    unsigned *count;    // arrivals; zero before the launch
    int *abort;         // set by a workgroup whose wait exceeded the bound
    int *status;        // device status word (EMU_STATUS_PANEL_WAIT)
};

// Best (value, row) over aligned groups of W lanes (xor butterfly).
template <int W>
__device__ __forceinline__ void lanes_best(double &v, int &i) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
}

__device__ __forceinline__ void st_relaxed(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                       (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_relaxed(const double *p) {
    return __longlong_as_double((long long)__hip_atomic_load(
        reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
        __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_relaxed(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct LeafLds {
    double val[2][LF_WAVES];
    int idx[2][LF_WAVES];
    double row[2][LF_WAVES][LEAF_W];
    double xrow[2][LEAF_W];
    double ur[2][LEAF_W];
    double xr[2][LEAF_W];
    int p[2];
    int abort;
};

// Column c of a leaf: pivot search, interchange, scaling, rank-1 update of
// this thread's rows.  Returns false when a multi-workgroup wait aborted.
template <bool MULTI, int c>
__device__ __forceinline__ bool leaf_col(double (&v)[LF_R][LEAF_W], LeafLds &L, int rows,
                                         int base_row, int g, int *ipiv, int grow0, int *info,
                                         const LeafX &x, unsigned base) {
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    constexpr int buf = c & 1;
    // this thread's and this wave's candidate for column c
    double bv = -1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * LF_THREADS;
        if (i >= c && i < rows && better(fabs(v[q][c]), i, bv, bi)) {
            bv = fabs(v[q][c]);
            bi = i;
        }
    }
    lanes_best<64>(bv, bi);
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * LF_THREADS;
        if (i == bi)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) L.row[buf][wid][j] = v[q][j];
        if (i == c)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) L.xrow[buf][j] = v[q][j];
    }
    if (lane == 0) {
        L.val[buf][wid] = bv;
        L.idx[buf][wid] = bi;
    }
    __syncthreads();
    // the workgroup's winner (every wave computes it)
    double wv = L.val[buf][lane & (LF_WAVES - 1)];
    int wi = L.idx[buf][lane & (LF_WAVES - 1)];
    lanes_best<LF_WAVES>(wv, wi);
    int p;
    const double *ur, *xr;
    if constexpr (!MULTI) {
        p = wi;
        ur = L.row[buf][((p - base_row) % LF_THREADS) / 64];
        xr = L.xrow[buf];
    } else {
        const int G = (int)gridDim.x;
        if (wid == 0) {
            if (lane < LEAF_W) {
                const double *src = L.row[buf][((wi - base_row) % LF_THREADS) / 64];
                st_relaxed(x.row + ((long long)buf * LF_MAX_G + g) * LEAF_W + lane, src[lane]);
                if (g == 0) st_relaxed(x.rowc + buf * LEAF_W + lane, L.xrow[buf][lane]);
            }
            if (lane == 0) {
                st_relaxed(x.val + buf * LF_MAX_G + g, wv);
                st_relaxed(x.idx + buf * LF_MAX_G + g, wi);
                // arrive, then wait for every workgroup of this column
                __hip_atomic_fetch_add(x.count, 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                const unsigned target = base + (unsigned)G * (unsigned)(c + 1);
                int spins = 0;
                while (__hip_atomic_load(x.count, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (ld_relaxed(x.abort) != 0) {
                        L.abort = 1;
                        break;
                    }
                    if (++spins > LF_SPIN_LIMIT) {
                        st_relaxed(x.abort, 1);
                        __hip_atomic_fetch_or(x.status, EMU_STATUS_PANEL_WAIT,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        L.abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            // the grid's winner, its row and row c
            const int l = lane & (LF_MAX_G - 1);
            double gv = -1.0;
            int gi = INT_MAX;
            if (l < G) {
                gv = ld_relaxed(x.val + buf * LF_MAX_G + l);
                gi = ld_relaxed(x.idx + buf * LF_MAX_G + l);
            }
            lanes_best<LF_MAX_G>(gv, gi);
            const int gp = (gi >= 0 && gi < G * LF_ROWS) ? gi / LF_ROWS : 0;
            if (lane < LEAF_W) {
                L.ur[buf][lane] = ld_relaxed(x.row + ((long long)buf * LF_MAX_G + gp) * LEAF_W + lane);
                L.xr[buf][lane] = ld_relaxed(x.rowc + buf * LEAF_W + lane);
            }
            if (lane == 0) L.p[buf] = gi;
        }
        __syncthreads();
        if (L.abort) return false;
        p = L.p[buf];
        ur = L.ur[buf];
        xr = L.xr[buf];
    }
    const double piv = ur[c];
    if (g == 0 && t == 0) {
        ipiv[c] = grow0 + p + 1;
        if (piv == 0.0 && *info == 0) *info = grow0 + c + 1;
    }
    const bool swap = piv != 0.0 && p != c;
    // row c after the interchange (the old row c when the pivot is zero)
    const double *u = (piv != 0.0) ? ur : xr;
    const bool recip = fabs(piv) >= DBL_MIN;
    const double rp = 1.0 / piv;
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * LF_THREADS;
        if (i < c || i >= rows) continue;
        if (swap && i == c) {
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) v[q][j] = ur[j];
        } else if (swap && i == p) {
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) v[q][j] = xr[j];
        }
        if (i > c) {
            double l = v[q][c];
            if (piv != 0.0) l = recip ? l * rp : l / piv;
            v[q][c] = l;
#pragma unroll
            for (int j = c + 1; j < LEAF_W; ++j) v[q][j] = v[q][j] - l * u[j];
        }
    }
    return true;
}

template <bool MULTI, int c>
__device__ __forceinline__ bool leaf_cols(double (&v)[LF_R][LEAF_W], LeafLds &L, int rows,
                                          int w, int base_row, int g, int *ipiv, int grow0,
                                          int *info, const LeafX &x, unsigned base) {
    if constexpr (c < LEAF_W) {
        if (c >= w) return true;
        if (!leaf_col<MULTI, c>(v, L, rows, base_row, g, ipiv, grow0, info, x, base))
            return false;
        return leaf_cols<MULTI, c + 1>(v, L, rows, w, base_row, g, ipiv, grow0, info, x, base);
    } else {
        return true;
    }
}

// P: top-left of the leaf (global row grow0), rows x w, w <= 16, rows >= w.
// Workgroup g owns rows [2048 g, 2048 g + 2048): thread t rows
// 2048 g + t and 2048 g + t + 1024.  MULTI: launched cooperatively; the
// arrival counter holds `base` at the launch (it only grows within a panel).
template <bool MULTI>
__global__ __launch_bounds__(LF_THREADS) void k_leaf(double *__restrict__ P, long long lda,
                                                     int rows, int w, int *ipiv, int grow0,
                                                     int *info, LeafX x, unsigned base) {
    __shared__ LeafLds L;
    const int t = threadIdx.x;
    const int g = MULTI ? (int)blockIdx.x : 0;
    const int base_row = g * LF_ROWS;
    if (t == 0) L.abort = 0;
    double v[LF_R][LEAF_W];
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * LF_THREADS;
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j)
            v[q][j] = (i < rows && j < w) ? P[i + (long long)j * lda] : 0.0;
    }
    if (!leaf_cols<MULTI, 0>(v, L, rows, w, base_row, g, ipiv, grow0, info, x, base)) return;
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * LF_THREADS;
        if (i < rows)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j)
                if (j < w) P[i + (long long)j * lda] = v[q][j];
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
// B (jb x ncols) <- L^-1 B for jb <= NB: one wave per 64 columns, a thread
// per column with the column in registers, L in LDS; for k increasing,
// b_i = b_i - l_ik b_k (i > k).  The column tile is staged through LDS so
// that global reads and writes run down the columns (contiguous), not
// across them (64 lanes a leading dimension apart).
constexpr int TR_COLS = 64;
template <int NB>
__global__ __launch_bounds__(TR_COLS) void k_trsm_reg(const double *__restrict__ L,
                                                      long long ldl, int jb,
                                                      double *__restrict__ B, long long ldb,
                                                      int ncols) {
    __shared__ double Ls[NB * NB];
    __shared__ double Bt[NB][TR_COLS + 1];
    const int t = threadIdx.x;
    const int col0 = blockIdx.x * TR_COLS;
    const int nc = min(TR_COLS, ncols - col0);
    for (int idx = t; idx < jb * jb; idx += TR_COLS) {
        const int i = idx % jb, k = idx / jb;
        Ls[k * NB + i] = L[i + (long long)k * ldl];
    }
    for (int e = t; e < jb * nc; e += TR_COLS) {
        const int i = e % jb, c = e / jb;
        Bt[i][c] = B[i + (long long)(col0 + c) * ldb];
    }
    __syncthreads();
    double b[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i] = i < jb ? Bt[i][t] : 0.0;
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
        if (i < jb) Bt[i][t] = b[i];
    __syncthreads();
    for (int e = t; e < jb * nc; e += TR_COLS) {
        const int i = e % jb, c = e / jb;
        B[i + (long long)(col0 + c) * ldb] = Bt[i][c];
    }
}

// Blocked: 64-row diagonal solves, order-preserving tile updates between.
int launch_trsm_llnu(const double *L, long long ldl, int jb, double *B, long long ldb,
                     int ncols, hipStream_t stream) {
    if (ncols <= 0 || jb <= 1) return 0;
    constexpr int D = 64;
    for (int k0 = 0; k0 < jb; k0 += D) {
        const int kb = jb - k0 < D ? jb - k0 : D;
        dim3 grid((ncols + TR_COLS - 1) / TR_COLS);
        const double *Lkk = L + k0 + (long long)k0 * ldl;
        double *Bk = B + k0;
        if (kb > 1) {
            if (kb <= 32)
                hipLaunchKernelGGL(k_trsm_reg<32>, grid, dim3(TR_COLS), 0, stream, Lkk, ldl, kb,
                                   Bk, ldb, ncols);
            else
                hipLaunchKernelGGL(k_trsm_reg<64>, grid, dim3(TR_COLS), 0, stream, Lkk, ldl, kb,
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
static size_t leafx_bytes() {
    return align256(2 * LF_MAX_G * sizeof(double)) + align256(2 * LF_MAX_G * sizeof(int)) +
           align256(2 * LF_MAX_G * LEAF_W * sizeof(double)) +
           align256(2 * LEAF_W * sizeof(double)) + align256(2 * sizeof(int));
}

size_t panel_scratch_bytes(int rows) {
    (void)rows;
    return leafx_bytes();
}

static LeafX leaf_x(char *ws, int *status) {
    LeafX x;
    char *p = ws;
    x.val = reinterpret_cast<double *>(p);
    p += align256(2 * LF_MAX_G * sizeof(double));
    x.idx = reinterpret_cast<int *>(p);
    p += align256(2 * LF_MAX_G * sizeof(int));
    x.row = reinterpret_cast<double *>(p);
    p += align256(2 * LF_MAX_G * LEAF_W * sizeof(double));
    x.rowc = reinterpret_cast<double *>(p);
    p += align256(2 * LEAF_W * sizeof(double));
    x.count = reinterpret_cast<unsigned *>(p);
    x.abort = reinterpret_cast<int *>(p) + 1;
    x.status = status;
    return x;
}

// One panel factorization: scratch, status word, and the arrivals the
// multi-workgroup leaves of this panel have made so far (the counter is
// zeroed once per panel).
struct PanelRun {
    char *ws;
    int *status;
    unsigned arrivals;
};

static int leaf(double *P, long long lda, int rows, int w, int *ipiv, int grow0, int *info,
                PanelRun &pr, hipStream_t st) {
    LeafX x = leaf_x(pr.ws, pr.status);
    if (rows <= LF_ROWS) {
        hipLaunchKernelGGL(k_leaf<false>, dim3(1), dim3(LF_THREADS), 0, st, P, lda, rows, w,
                           ipiv, grow0, info, x, 0u);
        EMU_TRY_HIP(hipGetLastError());
        return 0;
    }
    const int G = (rows + LF_ROWS - 1) / LF_ROWS;
    if (G > LF_MAX_G) {
        set_error("panel of %d rows above %d", rows, LF_MAX_G * LF_ROWS);
        return EMU_ERR_UNSUPPORTED;
    }
    unsigned base = pr.arrivals;
    void *args[] = {&P, &lda, &rows, &w, &ipiv, &grow0, &info, &x, &base};
    EMU_TRY_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_leaf<true>),
                                           dim3(G), dim3(LF_THREADS), args, 0, st));
    pr.arrivals += (unsigned)G * (unsigned)w;
    return 0;
}

// Factor columns [c0, c0 + w) of the panel whose top-left is A (global row
// and column row0), rows [c0, m_rows) of it; ipiv/info as in getrf.
static int panel_rec(double *A, long long lda, int m_rows, int c0, int w, int *ipiv, int row0,
                     int *info, PanelRun &pr, hipStream_t st) {
    double *P = A + c0 + (long long)c0 * lda;
    if (w <= LEAF_W)
        return leaf(P, lda, m_rows - c0, w, ipiv + c0, row0 + c0, info, pr, st);
    int w1 = (w / 2) / LEAF_W * LEAF_W;
    if (w1 < LEAF_W) w1 = LEAF_W;
    const int w2 = w - w1;
    EMU_TRY(panel_rec(A, lda, m_rows, c0, w1, ipiv, row0, info, pr, st));
    // interchanges of the left part on the right part's rows
    EMU_TRY(launch_laswp(A, lda, m_rows, 0, c0 + w1, w2, ipiv, c0, c0 + w1, row0, st));
    // U of the right part's top, then the rest of the right part
    EMU_TRY(launch_trsm_llnu(P, lda, w1, P + (long long)w1 * lda, lda, w2, st));
    EMU_TRY(gemm_seq(P + w1, lda, P + (long long)w1 * lda, lda, P + w1 + (long long)w1 * lda,
                     lda, m_rows - c0 - w1, w2, w1, st));
    EMU_TRY(panel_rec(A, lda, m_rows, c0 + w1, w2, ipiv, row0, info, pr, st));
    // interchanges of the right part on the left part's rows
    EMU_TRY(launch_laswp(A, lda, m_rows, 0, c0, w1, ipiv, c0 + w1, c0 + w, row0, st));
    return 0;
}

int launch_panel(double *A, long long lda, int rows, int jb, int *ipiv, int row0, int *info,
                 char *ws, int *status, hipStream_t stream) {
    PanelRun pr{ws, status, 0u};
    if (rows > LF_ROWS) {
        // arrival counter and abort flag start at zero (a fill kernel, not a memset)
        LeafX x = leaf_x(ws, status);
        EMU_TRY(launch_fill_int(reinterpret_cast<int *>(x.count), 0, 2, stream));
    }
    return panel_rec(A, lda, rows, 0, jb, ipiv, row0, info, pr, stream);
}

}  // namespace emu
