// Row interchanges and the triangular solves of getrs (paper: eqn (5), the
// solve that follows the factorization; the panel and the trailing TRSM are
// in panel.hip).
//
// Every FP64 update here is one rounded product followed by one rounded
// subtraction (this library is compiled with -ffp-contract=off), applied to
// each element in increasing elimination order, so the solutions are
// identical bit for bit to plain column-oriented substitution.
#include "common.h"
#include "devutil.h"

namespace emu {

// ------------------------------------------------- composed interchanges
// A run of row interchanges (step c swaps rows c and p_c, c increasing,
// p_c >= c) is sequential by definition, but its result has a closed form
// that a workgroup evaluates in parallel.  Step c only touches rows c and
// p_c >= c, so row c is final after step c and receives what row p_c held
// just before it.  Let g(j) be what row j holds just before step j: the
// content that the last earlier step i < j with p_i = j moved there, which
// is g(i), or j itself if there is no such step.  Then
//   row c (in the run)     ends with g(i) for the last i < c with p_i = p_c,
//                          or p_c if there is none;
//   row y below the run    ends with g(i) for the last i with p_i = y.
// The steps are sorted by (p_c, c) (bitonic, in LDS), which lines up each
// step with the previous one of the same target; g follows chains of
// strictly decreasing rows and is resolved by pointer jumping.  Rows are
// relative to the run's first; pivot c is piv[c] - 1 - base relative to it,
// and a value outside [c, R) means no interchange.
constexpr int CW = 1024;                     // steps per composition (threads)

struct ComposeLds {
    unsigned long long key[CW];              // (target << 32) | step, sorted
    int pred[CW];                            // last earlier step of the same target
    int g[CW];                               // chain links, then g(row)
};

// Thread c gets in blk the row whose old contents end in row c (c < min(J,
// R); c itself if unchanged), and, if it holds the last step into a row y
// below the run (y >= min(J, R)), ty = y and tsrc = the row whose old
// contents end there (else ty = -1).  All CW threads call it.
__device__ void wg_compose(const int *__restrict__ piv, int J, int R, int base, ComposeLds &L,
                           int &blk, int &ty, int &tsrc) {
    const int c = threadIdx.x;
    const int Jr = J < R ? J : R;
    int p = c;
    if (c < Jr) {
        p = piv[c] - 1 - base;
        if (p < c || p >= R) p = c;
    }
    L.key[c] = c < Jr ? ((unsigned long long)(unsigned)p << 32) | (unsigned)c : ~0ull;
    L.g[c] = c;
    __syncthreads();
    for (int size = 2; size <= CW; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int o = c ^ stride;
            if (o > c) {
                const unsigned long long x = L.key[c], y = L.key[o];
                if ((x > y) == ((c & size) == 0)) {
                    L.key[c] = y;
                    L.key[o] = x;
                }
            }
            __syncthreads();
        }
    // sorted position c: step i into target t
    int t = -1, i = -1, prev = -1;
    bool last = false;
    if (c < Jr) {
        const unsigned long long kc = L.key[c];
        t = (int)(kc >> 32);
        i = (int)(kc & 0xffffffffull);
        if (c > 0 && (int)(L.key[c - 1] >> 32) == t) prev = (int)(L.key[c - 1] & 0xffffffffull);
        last = c == Jr - 1 || (int)(L.key[c + 1] >> 32) != t;
        L.pred[i] = prev;
        // the last step before step t into row t (steps into t are <= t)
        if (last && t < Jr) L.g[t] = i < t ? i : (prev >= 0 ? prev : t);
    }
    __syncthreads();
    // chains are at most CW rows long: ten rounds of pointer jumping
    for (int r = 0; (1 << r) < CW; ++r) {
        const int nn = c < Jr ? L.g[L.g[c]] : c;
        __syncthreads();
        if (c < Jr) L.g[c] = nn;
        __syncthreads();
    }
    blk = c;
    if (c < Jr) {
        const int pr = L.pred[c];
        blk = pr >= 0 ? L.g[pr] : p;
    }
    ty = -1;
    tsrc = 0;
    if (last && t >= Jr) {
        ty = t;
        tsrc = L.g[i];
    }
}

constexpr int PERM_LDS_MAX = 32768;

// ---------------------------------------------------------------- laswp
// The interchanges ipiv[k1..k2) (1-based global rows; A's first row is
// global row row0) are applied to columns [0, ncols_left) and
// [col_right, col_right + ncols_right) of rows [k1, nrows).  A one-workgroup
// kernel composes them (above) and lists the rows that change as a plan:
// plan[0] = count, then each row (relative to A) and the row whose old
// values it receives.  The apply kernel reads the plan and moves, for its
// columns, every listed row's old value into place (all reads of a
// workgroup's tile before any write; consecutive threads walk down a
// column).
constexpr int SW_MAX = 1024;                 // interchanges per call
constexpr int SW_SLOTS = 2 * SW_MAX;         // rows a call can change
constexpr int SW_TILE = 4096;                // elements per workgroup pass

size_t laswp_plan_bytes(int nrows) {
    (void)nrows;
    return align256((size_t)(1 + 2 * SW_SLOTS) * sizeof(int));
}

// The plan: the run's rows that change, in order, then the rows below it
// that change, in increasing order.
__global__ __launch_bounds__(CW) void k_swap_plan(const int *__restrict__ ipiv, int k1, int k2,
                                                  int nrows, int row0, int *__restrict__ plan) {
    static_assert(SW_MAX <= CW, "one call's interchanges fit one composition");
    __shared__ ComposeLds L;
    __shared__ int wsum[2][CW / 64];
    const int R = nrows - k1;
    const int J = k2 - k1;
    const int Jr = J < R ? J : R;
    int blk, ty, tsrc;
    wg_compose(ipiv + k1, J, R, row0 + k1, L, blk, ty, tsrc);
    const int c = threadIdx.x, lane = c & 63, w = c >> 6;
    const bool f1 = c < Jr && blk != c, f2 = ty >= 0;
    const unsigned long long m1 = __ballot(f1), m2 = __ballot(f2);
    if (lane == 0) {
        wsum[0][w] = __popcll(m1);
        wsum[1][w] = __popcll(m2);
    }
    __syncthreads();
    int o1 = 0, o2 = 0, n1 = 0, n2 = 0;
    for (int x = 0; x < CW / 64; ++x) {
        const int a = wsum[0][x], b = wsum[1][x];
        if (x < w) {
            o1 += a;
            o2 += b;
        }
        n1 += a;
        n2 += b;
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    if (f1) {
        const int pos = o1 + __popcll(m1 & below);
        plan[1 + pos] = k1 + c;
        plan[1 + SW_SLOTS + pos] = k1 + blk;
    }
    if (f2) {
        const int pos = n1 + o2 + __popcll(m2 & below);
        plan[1 + pos] = k1 + ty;
        plan[1 + SW_SLOTS + pos] = k1 + tsrc;
    }
    if (c == 0) plan[0] = n1 + n2;
}

__global__ __launch_bounds__(256) void k_swap_apply(double *__restrict__ A, long long lda,
                                                    int ncols_left, int col_right,
                                                    int ncols_right, int cw,
                                                    const int *__restrict__ plan) {
    constexpr int PER = SW_TILE / 256;
    __shared__ int srow[SW_SLOTS], ssrc[SW_SLOTS];
    const int t = threadIdx.x;
    const int nslot = plan[0];
    for (int e = t; e < nslot; e += 256) {
        srow[e] = plan[1 + e];
        ssrc[e] = plan[1 + SW_SLOTS + e];
    }
    __syncthreads();
    if (nslot == 0) return;
    const int ncols = ncols_left + ncols_right;
    // columns of this workgroup, in passes of at most SW_TILE elements
    const int cpp = nslot < SW_TILE ? SW_TILE / nslot : 1;      // columns per pass
    const int c_begin = blockIdx.x * cw;
    const int c_end = min(ncols, c_begin + cw);
    for (int cb = c_begin; cb < c_end; cb += cpp) {
        const int cn = min(cpp, c_end - cb);
        const int total = nslot * cn;
        double vals[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = t + 256 * k;
            vals[k] = 0.0;
            if (e < total) {
                const int sl = e % nslot, jj = e / nslot;
                const int cidx = cb + jj;
                const int col = cidx < ncols_left ? cidx : col_right + (cidx - ncols_left);
                vals[k] = A[ssrc[sl] + (long long)col * lda];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = t + 256 * k;
            if (e < total) {
                const int sl = e % nslot, jj = e / nslot;
                const int cidx = cb + jj;
                const int col = cidx < ncols_left ? cidx : col_right + (cidx - ncols_left);
                A[srow[sl] + (long long)col * lda] = vals[k];
            }
        }
        __syncthreads();
    }
}

// perm[r] <- perm[source of r] for the rows a plan lists (all reads first):
// the row permutation of a factorization, kept up to date panel by panel.
__global__ __launch_bounds__(1024) void k_perm_apply(int *__restrict__ perm,
                                                     const int *__restrict__ plan) {
    const int nslot = plan[0];
    int v[SW_SLOTS / 1024];
#pragma unroll
    for (int r = 0; r < SW_SLOTS / 1024; ++r) {
        const int e = threadIdx.x + 1024 * r;
        v[r] = e < nslot ? perm[plan[1 + SW_SLOTS + e]] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SW_SLOTS / 1024; ++r) {
        const int e = threadIdx.x + 1024 * r;
        if (e < nslot) perm[plan[1 + e]] = v[r];
    }
}

__global__ void k_perm_init(int *__restrict__ perm, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = i;
}

int launch_perm_init(int *perm, int n, hipStream_t stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_perm_init, dim3((n + 255) / 256), dim3(256), 0, stream, perm, n);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_laswp(double *A, long long lda, int nrows, int ncols_left, int col_right,
                 int ncols_right, const int *ipiv, int k1, int k2, int row0, int *plan,
                 hipStream_t stream, int *perm) {
    const int total = ncols_left + ncols_right;
    if (k2 <= k1 || nrows <= k1) return 0;
    if (total <= 0 && !perm) return 0;
    if (k2 - k1 > SW_MAX) {
        set_error("more than %d interchanges in one call", SW_MAX);
        return EMU_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL(k_swap_plan, dim3(1), dim3(CW), 0, stream, ipiv, k1, k2, nrows, row0,
                       plan);
    if (perm) hipLaunchKernelGGL(k_perm_apply, dim3(1), dim3(1024), 0, stream, perm, plan);
    return launch_laswp_apply(A, lda, nrows, ncols_left, col_right, ncols_right, k1, k2, plan,
                              stream);
}

int launch_laswp_apply(double *A, long long lda, int nrows, int ncols_left, int col_right,
                       int ncols_right, int k1, int k2, const int *plan, hipStream_t stream) {
    const int total = ncols_left + ncols_right;
    if (total <= 0 || k2 <= k1 || nrows <= k1) return 0;
    // columns per workgroup from the largest possible plan (2 per interchange)
    const int nslot_max = 2 * (k2 - k1);
    const int cw = nslot_max < SW_TILE ? SW_TILE / nslot_max : 1;
    const int blocks = (total + cw - 1) / cw;
    hipLaunchKernelGGL(k_swap_apply, dim3(blocks), dim3(256), 0, stream, A, lda, ncols_left,
                       col_right, ncols_right, cw, plan);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------- getrs
// The row interchanges of the whole factorization composed into one gather
// permutation (in LDS when it fits), CW interchanges at a time.
__global__ __launch_bounds__(CW) void k_perm_from_ipiv(const int *__restrict__ ipiv, int n,
                                                       int *__restrict__ perm) {
    __shared__ int lp[PERM_LDS_MAX];
    __shared__ ComposeLds L;
    const int c = threadIdx.x;
    const bool in_lds = n <= PERM_LDS_MAX;
    int *pm = in_lds ? lp : perm;
    for (int i = c; i < n; i += CW) pm[i] = i;
    __syncthreads();
    // pivots kb .. kb + J act on rows kb.. (relative rows of pm + kb)
    for (int kb = 0; kb < n; kb += CW) {
        const int J = n - kb < CW ? n - kb : CW;
        int blk, ty, tsrc;
        wg_compose(ipiv + kb, J, n - kb, kb, L, blk, ty, tsrc);
        const bool f1 = c < J && blk != c;
        const int v1 = f1 ? pm[kb + blk] : 0;
        const int v2 = ty >= 0 ? pm[kb + tsrc] : 0;
        __syncthreads();
        if (f1) pm[kb + c] = v1;
        if (ty >= 0) pm[kb + ty] = v2;
        __syncthreads();
    }
    if (in_lds)
        for (int i = c; i < n; i += CW) perm[i] = lp[i];
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

// Value of lane k (k uniform) broadcast to the wave.
__device__ __forceinline__ double lane_bcast(double v, int k) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, k);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// The kb x kb diagonal block at (k0, k0) into LDS, column-major (lane i
// reads row i of every column: contiguous in global memory, conflict-free
// in LDS).
__device__ __forceinline__ void load_diag_block(const double *__restrict__ LU, long long lda,
                                                int k0, int kb, double *Ds) {
    const int lane = threadIdx.x & 63;
    // all loads issued before the first store (no serialized round trips)
    double col[TRSV_NB];
#pragma unroll
    for (int k = 0; k < TRSV_NB; ++k)
        col[k] = (k < kb && lane < kb) ? LU[(k0 + lane) + (long long)(k0 + k) * lda] : 0.0;
#pragma unroll
    for (int k = 0; k < TRSV_NB; ++k) Ds[k * TRSV_NB + lane] = col[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Forward substitution, diagonal block [k0, k0+kb): one wave per rhs; lane
// i holds x_{k0+i}; for k increasing, lanes i > k subtract l_ik x_k.
__global__ __launch_bounds__(64) void k_fwd_diag(const double *__restrict__ LU,
                                                 long long lda, int n, int k0, int kb,
                                                 double *__restrict__ X) {
    __shared__ double Ds[TRSV_NB * TRSV_NB];
    const int lane = threadIdx.x;
    load_diag_block(LU, lda, k0, kb, Ds);
    double *x = X + (long long)blockIdx.x * n;
    const int i = k0 + lane;
    double b = lane < kb ? x[i] : 0.0;
    for (int k = 0; k < kb - 1; ++k) {
        const double xk = lane_bcast(b, k);
        if (lane > k && lane < kb) b = b - Ds[k * TRSV_NB + lane] * xk;
    }
    if (lane < kb) x[i] = b;
}

// Rows [r0, n) after the diagonal block [k0, k0+kb): x_i -= l_ik x_k, k
// increasing.  Workgroup 0's first wave holds rows r0 .. r0+63, the next
// diagonal block (kb2 rows): once they are updated it solves that block in
// registers as k_fwd_diag does, so the sweep needs no diagonal launch of
// its own after the first.
__global__ __launch_bounds__(256) void k_fwd_update(const double *__restrict__ LU,
                                                    long long lda, int n, int k0,
                                                    int kb, int r0, int kb2,
                                                    double *__restrict__ X) {
    __shared__ double xs[TRSV_NB];
    __shared__ double Ds[TRSV_NB * TRSV_NB];
    double *x = X + (long long)blockIdx.y * n;
    const bool diag = blockIdx.x == 0 && kb2 > 0 && threadIdx.x < 64;
    if (threadIdx.x < kb) xs[threadIdx.x] = x[k0 + threadIdx.x];
    if (diag) load_diag_block(LU, lda, r0, kb2, Ds);
    __syncthreads();
    const int i = r0 + blockIdx.x * blockDim.x + threadIdx.x;
    double b = 0.0;
    if (i < n) {
        double l[TRSV_NB];
#pragma unroll
        for (int k = 0; k < TRSV_NB; ++k)
            l[k] = k < kb ? LU[i + (long long)(k0 + k) * lda] : 0.0;
        b = x[i];
#pragma unroll
        for (int k = 0; k < TRSV_NB; ++k)
            if (k < kb) b = b - l[k] * xs[k];
    }
    if (diag) {
        const int lane = threadIdx.x;
        for (int k = 0; k < kb2 - 1; ++k) {
            const double xk = lane_bcast(b, k);
            if (lane > k && lane < kb2) b = b - Ds[k * TRSV_NB + lane] * xk;
        }
    }
    if (i < n) x[i] = b;
}

// Back substitution, diagonal block [k0, k0+kb): for k decreasing,
// x_k = b_k / u_kk, then lanes i < k subtract u_ik x_k.
__global__ __launch_bounds__(64) void k_bwd_diag(const double *__restrict__ LU,
                                                 long long lda, int n, int k0, int kb,
                                                 double *__restrict__ X) {
    __shared__ double Ds[TRSV_NB * TRSV_NB];
    const int lane = threadIdx.x;
    load_diag_block(LU, lda, k0, kb, Ds);
    double *x = X + (long long)blockIdx.x * n;
    const int i = k0 + lane;
    double b = lane < kb ? x[i] : 0.0;
    for (int k = kb - 1; k >= 0; --k) {
        if (lane == k) b = b / Ds[k * TRSV_NB + k];
        const double xk = lane_bcast(b, k);
        if (lane < k) b = b - Ds[k * TRSV_NB + lane] * xk;
    }
    if (lane < kb) x[i] = b;
}

// Rows [0, k0) above the diagonal block [k0, k0+kb): x_i -= u_ik x_k, k
// decreasing.  k0 is a multiple of 64, so rows k0-64 .. k0-1, the previous
// diagonal block, are one whole wave of the last workgroup: once they are
// updated that wave solves the block in registers as k_bwd_diag does.
__global__ __launch_bounds__(256) void k_bwd_update(const double *__restrict__ LU,
                                                    long long lda, int n, int k0,
                                                    int kb, double *__restrict__ X) {
    __shared__ double xs[TRSV_NB];
    __shared__ double Ds[TRSV_NB * TRSV_NB];
    double *x = X + (long long)blockIdx.y * n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // the wave holding rows [k0 - 64, k0) (uniform per wave)
    const bool diag = i >= k0 - TRSV_NB && i - (int)(threadIdx.x & 63) + TRSV_NB <= k0;
    if (threadIdx.x < kb) xs[threadIdx.x] = x[k0 + threadIdx.x];
    if (diag) load_diag_block(LU, lda, k0 - TRSV_NB, TRSV_NB, Ds);
    __syncthreads();
    if (i >= k0) return;
    double u[TRSV_NB];
#pragma unroll
    for (int k = 0; k < TRSV_NB; ++k) u[k] = k < kb ? LU[i + (long long)(k0 + k) * lda] : 0.0;
    double b = x[i];
#pragma unroll
    for (int k = TRSV_NB - 1; k >= 0; --k)
        if (k < kb) b = b - u[k] * xs[k];
    if (diag) {
        const int lane = threadIdx.x & 63;
        for (int k = TRSV_NB - 1; k >= 0; --k) {
            if (lane == k) b = b / Ds[k * TRSV_NB + k];
            const double xk = lane_bcast(b, k);
            if (lane < k) b = b - Ds[k * TRSV_NB + lane] * xk;
        }
    }
    x[i] = b;
}

// ------------------------------------------ inverted diagonal blocks
// For block b of the precision form's solves: L_bb^-1 (unit lower) at
// inv + 2 b 64^2 and U_bb^-1 at inv + (2 b + 1) 64^2, column-major 64 x 64,
// zero outside the block's nb x nb part.  One wave per block; lane j
// computes column j of each inverse by substitution on the unit vector
// (its entries in LDS, column j only read and written by lane j).
size_t tri_inv_bytes(int n) {
    return align256((size_t)((n + TRSV_NB - 1) / TRSV_NB) * 2 * TRSV_NB * TRSV_NB *
                    sizeof(double));
}

__global__ __launch_bounds__(64) void k_tri_inv(const double *__restrict__ LU, long long lda,
                                                int n, double *__restrict__ inv) {
    __shared__ double Ds[TRSV_NB * TRSV_NB];        // the block, column-major
    __shared__ double Xs[TRSV_NB * TRSV_NB];        // entry i of column j at i 64 + j
    const int j = threadIdx.x;
    const int b = blockIdx.x;
    const int r0 = b * TRSV_NB;
    const int nb = n - r0 < TRSV_NB ? n - r0 : TRSV_NB;
    for (int k = 0; k < TRSV_NB; ++k)
        Ds[k * TRSV_NB + j] =
            (k < nb && j < nb) ? LU[r0 + j + (long long)(r0 + k) * lda] : 0.0;
    __syncthreads();
    double *Li = inv + (size_t)(2 * b) * TRSV_NB * TRSV_NB;
    double *Ui = Li + TRSV_NB * TRSV_NB;
    // L^-1 e_j: x_i = 0 (i < j), 1 (i = j), -sum_{k = j}^{i - 1} l_ik x_k
    for (int i = 0; i < TRSV_NB; ++i) {
        double x = 0.0;
        if (j < nb && i < nb && i >= j) {
            if (i == j) {
                x = 1.0;
            } else {
                double sum = 0.0;
#pragma unroll 8
                for (int k = j; k < i; ++k) sum = sum + Ds[k * TRSV_NB + i] * Xs[k * TRSV_NB + j];
                x = -sum;
            }
        }
        Xs[i * TRSV_NB + j] = x;
    }
    for (int i = 0; i < TRSV_NB; ++i) Li[j * TRSV_NB + i] = Xs[i * TRSV_NB + j];
    // U^-1 e_j: x_i = 0 (i > j), 1 / u_jj (i = j),
    // -(sum_{k = i + 1}^{j} u_ik x_k) / u_ii (i < j)
    for (int i = TRSV_NB - 1; i >= 0; --i) {
        double x = 0.0;
        if (j < nb && i < nb && i <= j) {
            if (i == j) {
                x = 1.0 / Ds[j * TRSV_NB + j];
            } else {
                double sum = 0.0;
#pragma unroll 8
                for (int k = i + 1; k <= j; ++k)
                    sum = sum + Ds[k * TRSV_NB + i] * Xs[k * TRSV_NB + j];
                x = -sum / Ds[i * TRSV_NB + i];
            }
        }
        Xs[i * TRSV_NB + j] = x;
    }
    for (int i = 0; i < TRSV_NB; ++i) Ui[j * TRSV_NB + i] = Xs[i * TRSV_NB + j];
}

int launch_tri_inv(const double *LU, long long lda, int n, double *inv, hipStream_t stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_tri_inv, dim3((n + TRSV_NB - 1) / TRSV_NB), dim3(64), 0, stream, LU,
                       lda, n, inv);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ------------------------------------------- persistent triangular solves
// One launch per sweep for up to PT_RHS right-hand sides: one workgroup per
// 64-row block, one wave per right-hand side.  A workgroup takes its place
// in the sweep from a ticket (in the order workgroups start, so it waits
// only on blocks held by workgroups already running: no deadlock whatever
// the occupancy).  Each lane owns a row: it subtracts the earlier blocks'
// contributions in sweep order as their solutions appear, 64 columns at a
// time (the block's columns loaded before its solution is awaited), then the
// wave resolves its own diagonal block in registers, with the block in LDS,
// as the blocked kernels do, and publishes its 64 solutions as tagged
// 64-bit words (32-bit payload, the sweep's tag in the high half, written by
// relaxed stores and validated one by one, so one read follows the last
// write).  Every element receives the same operations in the same order as
// in the column-by-column substitution.  The wait is bounded: a wave that
// exceeds PT_SPIN_LIMIT polls raises EMU_STATUS_SOLVE_WAIT and the abort
// flag, and the waves still waiting leave; the solution is then invalid.
// INV (the precision form): the diagonal block is not resolved by its
// 64-step chain but multiplied by its inverse (k_tri_inv), 64 independent
// products per lane; the solution then differs from substitution in
// rounding, which the refinement corrects.
constexpr int PT_RHS = 4;
constexpr int PT_SPIN_LIMIT = 1 << 21;
constexpr int PT_WORDS = 2 * TRSV_NB;                 // words per block and rhs

__device__ __forceinline__ unsigned long long pt_load(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool FWD, bool INV>
__global__ __launch_bounds__(64 * PT_RHS) void k_trsv_persist(
    const double *__restrict__ LU, long long lda, int n, int nrhs, double *__restrict__ X,
    unsigned long long *__restrict__ words, int *__restrict__ ctr, int *__restrict__ status,
    unsigned tag, const double *__restrict__ inv) {
    extern __shared__ double Dsh[];                   // TRSV_NB^2 doubles per wave
    __shared__ int s_q;
    const int t = threadIdx.x, lane = t & 63;
    const int r = __builtin_amdgcn_readfirstlane(t >> 6);   // right-hand side of this wave
    if (t == 0) s_q = atomicAdd(&ctr[0], 1);
    __syncthreads();
    const int nblk = (n + TRSV_NB - 1) / TRSV_NB;
    const int q = s_q;                                // place of this block in the sweep
    if (q >= nblk || r >= nrhs) return;               // whole waves
    const int blk = FWD ? q : nblk - 1 - q;
    const int r0 = blk * TRSV_NB;
    const int nb = n - r0 < TRSV_NB ? n - r0 : TRSV_NB;
    const int i = r0 + lane;
    double *x = X + (long long)r * n;
    double *Ds = Dsh + (size_t)r * TRSV_NB * TRSV_NB;
    // the diagonal block (INV: its inverse) into LDS (lane i reads row i of
    // every column)
    {
        double col[TRSV_NB];
        if constexpr (INV) {
            const double *iv = inv + ((size_t)2 * blk + (FWD ? 0 : 1)) * TRSV_NB * TRSV_NB;
#pragma unroll
            for (int k = 0; k < TRSV_NB; ++k) col[k] = iv[k * TRSV_NB + lane];
        } else {
#pragma unroll
            for (int k = 0; k < TRSV_NB; ++k)
                col[k] = (k < nb && lane < nb) ? LU[i + (long long)(r0 + k) * lda] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < TRSV_NB; ++k) Ds[k * TRSV_NB + lane] = col[k];
    }
    double acc = lane < nb ? x[i] : 0.0;
    const unsigned long long tg = (unsigned long long)tag << 32;
    for (int p = 0; p < q; ++p) {
        const int bj = FWD ? p : nblk - 1 - p;        // earlier block of the sweep
        const int c0 = bj * TRSV_NB;
        const int cb = n - c0 < TRSV_NB ? n - c0 : TRSV_NB;
        double l[TRSV_NB];
#pragma unroll
        for (int k = 0; k < TRSV_NB; ++k)
            l[k] = (lane < nb && k < cb) ? LU[i + (long long)(c0 + k) * lda] : 0.0;
        const unsigned long long *wj = words + ((long long)bj * PT_RHS + r) * PT_WORDS;
        unsigned long long w0 = 0ull, w1 = 0ull;
        int spins = 0;
        for (;;) {
            if (lane < cb) {
                w0 = pt_load(wj + 2 * lane);
                w1 = pt_load(wj + 2 * lane + 1);
            }
            const bool ok = lane >= cb || ((w0 >> 32) == (tg >> 32) && (w1 >> 32) == (tg >> 32));
            if (__ballot(!ok) == 0ull) break;
            if ((++spins & 63) == 0) {
                if (__hip_atomic_load(&ctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                    return;
                if (spins > PT_SPIN_LIMIT) {
                    if (lane == 0) {
                        __hip_atomic_store(&ctr[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_or(status, EMU_STATUS_SOLVE_WAIT, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    }
                    return;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        const double xv = __longlong_as_double(
            (long long)(((w1 & 0xFFFFFFFFull) << 32) | (w0 & 0xFFFFFFFFull)));
        if constexpr (FWD) {
#pragma unroll
            for (int k = 0; k < TRSV_NB; ++k) {
                if (k < cb) {
                    const double xk = lane_bcast(xv, k);
                    acc = acc - l[k] * xk;
                }
            }
        } else {
#pragma unroll
            for (int k = TRSV_NB - 1; k >= 0; --k) {
                if (k < cb) {
                    const double xk = lane_bcast(xv, k);
                    acc = acc - l[k] * xk;
                }
            }
        }
    }
    if constexpr (INV) {
        // entries outside the block's nb x nb part are zero, and so is acc
        // in the lanes past nb
        double y = 0.0;
#pragma unroll 16
        for (int k = 0; k < TRSV_NB; ++k) {
            const double ak = lane_bcast(acc, k);
            y = y + Ds[k * TRSV_NB + lane] * ak;
        }
        acc = y;
    } else if constexpr (FWD) {
        for (int k = 0; k < nb - 1; ++k) {
            const double xk = lane_bcast(acc, k);
            if (lane > k && lane < nb) acc = acc - Ds[k * TRSV_NB + lane] * xk;
        }
    } else {
        for (int k = nb - 1; k >= 0; --k) {
            if (lane == k) acc = acc / Ds[k * TRSV_NB + k];
            const double xk = lane_bcast(acc, k);
            if (lane < k) acc = acc - Ds[k * TRSV_NB + lane] * xk;
        }
    }
    if (lane < nb) {
        x[i] = acc;
        unsigned long long *wb = words + ((long long)blk * PT_RHS + r) * PT_WORDS;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(acc);
        __hip_atomic_store(wb + 2 * lane, tg | (bits & 0xFFFFFFFFull), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(wb + 2 * lane + 1, tg | (bits >> 32), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Scratch of launch_getrs: the permutation, X, and the persistent solves'
// records and counters.
static size_t getrs_words_bytes(int n) {
    const size_t nblk = (size_t)(n + TRSV_NB - 1) / TRSV_NB;
    return align256(nblk * PT_RHS * PT_WORDS * sizeof(unsigned long long));
}

size_t getrs_ws_bytes(int n, int nrhs) {
    return align256((size_t)n * sizeof(int)) + align256((size_t)n * nrhs * sizeof(double)) +
           getrs_words_bytes(n) + 256;
}

int launch_getrs(int n, int nrhs, const double *LU, long long lda, const int *ipiv,
                 double *B, long long ldb, int *perm_ws, hipStream_t stream, bool perm_ready,
                 int *status, const int *perm_ext, const double *inv) {
    if (n <= 0 || nrhs <= 0) return 0;
    const int *perm = perm_ext ? perm_ext : perm_ws;
    char *base = reinterpret_cast<char *>(perm_ws);
    double *X = reinterpret_cast<double *>(base + align256((size_t)n * sizeof(int)));
    if (!perm_ready && !perm_ext)
        hipLaunchKernelGGL(k_perm_from_ipiv, dim3(1), dim3(CW), 0, stream, ipiv, n, perm_ws);
    dim3 gcol((n + 255) / 256, nrhs);
    hipLaunchKernelGGL(k_gather_rows, gcol, dim3(256), 0, stream, B, ldb, n, perm, X);
    if (nrhs <= PT_RHS && status) {
        char *wbase = base + align256((size_t)n * sizeof(int)) +
                      align256((size_t)n * nrhs * sizeof(double));
        unsigned long long *words = reinterpret_cast<unsigned long long *>(wbase);
        int *ctr = reinterpret_cast<int *>(wbase + getrs_words_bytes(n));
        const int nblk = (n + TRSV_NB - 1) / TRSV_NB;
        // records (tag 0: not written) and both sweeps' tickets and abort flags
        EMU_TRY(launch_fill_int(reinterpret_cast<int *>(words), 0,
                                (int)(getrs_words_bytes(n) / sizeof(int)), stream));
        EMU_TRY(launch_fill_int(ctr, 0, 4, stream));
        const size_t lds = (size_t)nrhs * TRSV_NB * TRSV_NB * sizeof(double);
        // up to PT_RHS diagonal blocks of dynamic LDS (128 KB): allowed once
        static const hipError_t attr = [] {
            const int mx = PT_RHS * TRSV_NB * TRSV_NB * (int)sizeof(double);
            const void *fns[4] = {reinterpret_cast<const void *>(&k_trsv_persist<true, false>),
                                  reinterpret_cast<const void *>(&k_trsv_persist<false, false>),
                                  reinterpret_cast<const void *>(&k_trsv_persist<true, true>),
                                  reinterpret_cast<const void *>(&k_trsv_persist<false, true>)};
            hipError_t e = hipSuccess;
            for (int f = 0; f < 4 && e == hipSuccess; ++f)
                e = hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize, mx);
            return e;
        }();
        if (attr != hipSuccess) return fail_hip(attr, "hipFuncSetAttribute");
        if (inv) {
            hipLaunchKernelGGL((k_trsv_persist<true, true>), dim3(nblk), dim3(64 * nrhs), lds,
                               stream, LU, lda, n, nrhs, X, words, ctr, status, 1u, inv);
            hipLaunchKernelGGL((k_trsv_persist<false, true>), dim3(nblk), dim3(64 * nrhs), lds,
                               stream, LU, lda, n, nrhs, X, words, ctr + 2, status, 2u, inv);
        } else {
            hipLaunchKernelGGL((k_trsv_persist<true, false>), dim3(nblk), dim3(64 * nrhs), lds,
                               stream, LU, lda, n, nrhs, X, words, ctr, status, 1u, inv);
            hipLaunchKernelGGL((k_trsv_persist<false, false>), dim3(nblk), dim3(64 * nrhs), lds,
                               stream, LU, lda, n, nrhs, X, words, ctr + 2, status, 2u, inv);
        }
        hipLaunchKernelGGL(k_copy_cols, gcol, dim3(256), 0, stream, X, n, B, ldb);
        EMU_TRY_HIP(hipGetLastError());
        return 0;
    }
    // forward: the first diagonal block, then per block the update of the
    // rows below it together with the next diagonal block
    hipLaunchKernelGGL(k_fwd_diag, dim3(nrhs), dim3(64), 0, stream, LU, lda, n, 0,
                       n < TRSV_NB ? n : TRSV_NB, X);
    for (int k0 = 0; k0 < n; k0 += TRSV_NB) {
        const int kb = n - k0 < TRSV_NB ? n - k0 : TRSV_NB;
        const int r0 = k0 + kb;
        if (r0 < n) {
            const int kb2 = n - r0 < TRSV_NB ? n - r0 : TRSV_NB;
            dim3 g((n - r0 + 255) / 256, nrhs);
            hipLaunchKernelGGL(k_fwd_update, g, dim3(256), 0, stream, LU, lda, n, k0, kb,
                               r0, kb2, X);
        }
    }
    // backward: the last diagonal block, then per block the update of the
    // rows above it together with the previous diagonal block
    const int last0 = (n - 1) / TRSV_NB * TRSV_NB;
    hipLaunchKernelGGL(k_bwd_diag, dim3(nrhs), dim3(64), 0, stream, LU, lda, n, last0,
                       n - last0, X);
    for (int k0 = last0; k0 > 0; k0 -= TRSV_NB) {
        const int kb = n - k0 < TRSV_NB ? n - k0 : TRSV_NB;
        dim3 g((k0 + 255) / 256, nrhs);
        hipLaunchKernelGGL(k_bwd_update, g, dim3(256), 0, stream, LU, lda, n, k0, kb, X);
    }
    hipLaunchKernelGGL(k_copy_cols, gcol, dim3(256), 0, stream, X, n, B, ldb);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

}  // namespace emu
