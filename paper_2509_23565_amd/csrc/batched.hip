// Batched grouped form: many independent LU systems of uneven size solved
// together (this form is not in the paper; each system is the paper's LU with
// the emulated Schur update of eqn (8)).
//
// Systems are sorted by size, so the systems still active at block step j
// (n_i > j nb) are a prefix of the list.  Each step issues one launch per
// phase for all active systems: panel (one workgroup per system, the panel in
// registers), interchanges right of the panel with the triangular solve
// (interchanges left of the panels: once, after the last step), slicing of
// every L21 and U12
// (one pass each: K = nb <= 32 is a single fragment block), and one
// persistent grouped slice-product GEMM over the concatenated tile lists of
// all systems.  The whole sequence (and the solves) is captured once per
// batch shape into a hipGraph and replayed; per call only the descriptor
// tables are refreshed.  Every FP64 step follows the single-system order, so
// each system's factors are bit-identical to emu_dgetrf with the same nb.
//
// An autotuner times the candidate block sizes and grouped-GEMM grid sizes
// on a copy of a batch and records the fastest per batch shape.
#include "common.h"
#include "devutil.h"

#include <float.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

namespace emu {

constexpr int BMAX_N = 1024;       // grouped path: systems up to this size
constexpr int BMAX_NB = 32;        // panel width held in registers
constexpr int BMAX_RHS = 8;

struct BSys {
    double *A;
    long long lda;
    int n;
    int nrhs;
    int *ipiv;
    int *info;
    double *B;
    long long ldb;
};

// ------------------------------------------------------------------ panel
// One workgroup per active system: column-by-column over the rows x jb
// panel at (j0, j0), one row per thread, the row's jb <= 32 values in
// registers (same operations and order as the single-system panel).  The
// column loop is unrolled at compile time, so every register index is fixed.
struct BPanelLds {
    double urow[BMAX_NB], xrow[BMAX_NB];
    long long red_k[16];
    int red_i[16];
};

template <int c>
__device__ __forceinline__ void bpanel_cols(double (&v)[BMAX_NB], BPanelLds &L, int t, int rows,
                                            int w, const BSys &S, int j0) {
    if constexpr (c < BMAX_NB) {
        if (c >= w) return;
        long long bk = -1;
        int bi = INT_MAX;
        if (t >= c && t < rows) {
            bk = pivot_key(v[c]);
            bi = t;
        }
        block_key_best<16>(bk, bi, L.red_k, L.red_i);
        const int p = bi;
        if (t == p)
#pragma unroll
            for (int j = 0; j < BMAX_NB; ++j) L.urow[j] = v[j];
        if (t == c)
#pragma unroll
            for (int j = 0; j < BMAX_NB; ++j) L.xrow[j] = v[j];
        __syncthreads();
        const double piv = L.urow[c];
        if (t == 0) {
            S.ipiv[j0 + c] = j0 + p + 1;
            if (piv == 0.0 && *S.info == 0) *S.info = j0 + c + 1;
        }
        const bool swap = piv != 0.0 && p != c;
        const double *ur = (piv != 0.0) ? L.urow : L.xrow;
        if (swap && t == c) {
#pragma unroll
            for (int j = 0; j < BMAX_NB; ++j) v[j] = L.urow[j];
        } else if (swap && t == p) {
#pragma unroll
            for (int j = 0; j < BMAX_NB; ++j) v[j] = L.xrow[j];
        }
        if (t > c && t < rows) {
            double l = v[c];
            if (piv != 0.0) l = (fabs(piv) >= DBL_MIN) ? l * (1.0 / piv) : l / piv;
            v[c] = l;
#pragma unroll
            for (int j = c + 1; j < BMAX_NB; ++j) v[j] = v[j] - l * ur[j];
        }
        __syncthreads();
        bpanel_cols<c + 1>(v, L, t, rows, w, S, j0);
    }
}

__global__ __launch_bounds__(1024) void k_bpanel(const BSys *__restrict__ sys, int j0, int nb) {
    __shared__ BPanelLds L;
    const BSys S = sys[blockIdx.x];
    const int rows = S.n - j0;
    if (rows <= 0) return;
    const int w = nb < rows ? nb : rows;
    double *P = S.A + j0 + (long long)j0 * S.lda;
    const int t = threadIdx.x;
    double v[BMAX_NB];
#pragma unroll
    for (int j = 0; j < BMAX_NB; ++j)
        v[j] = (t < rows && j < w) ? P[t + (long long)j * S.lda] : 0.0;
    bpanel_cols<0>(v, L, t, rows, w, S, j0);
    if (t < rows)
#pragma unroll
        for (int j = 0; j < BMAX_NB; ++j)
            if (j < w) P[t + (long long)j * S.lda] = v[j];
}

// Interchanges of step j0 on the columns right of the panel, fused with
// U12 = L11^-1 A12 on them (the columns left of the panel receive their
// interchanges at the end, k_blaswp_left).  Per 64 columns: wave 0 composes
// the jb <= 32 interchanges into the rows they move (at most 64); the top jb
// rows after the interchanges are gathered into an LDS tile (a row that
// comes from below reads its source row) and the moved rows below the top
// are read, all before any write; then those are written, one wave solves
// the tile (a lane per column, L11 in LDS, same order as the single-system
// TRSM) and the top rows are written back down the columns.
constexpr int BST_COLS = 64;
__global__ __launch_bounds__(256) void k_bswap_trsm(const BSys *__restrict__ sys, int j0, int nb) {
    __shared__ double Ls[BMAX_NB * BMAX_NB];
    __shared__ double Bt[BMAX_NB][BST_COLS + 1];
    __shared__ int srow_s[2 * BMAX_NB], ssrc_s[2 * BMAX_NB], topsrc[BMAX_NB];
    __shared__ int nslot_s;
    const BSys S = sys[blockIdx.y];
    const int rows = S.n - j0;
    if (rows <= 0) return;
    const int w = nb < rows ? nb : rows;
    const int ncols = S.n - j0 - w;                  // columns [j0 + w, n)
    const int c0 = blockIdx.x * BST_COLS;
    if (ncols <= 0 || c0 >= ncols) return;           // uniform per workgroup
    const int t = threadIdx.x;
    const int nc = ncols - c0 < BST_COLS ? ncols - c0 : BST_COLS;
    double *Ac = S.A + j0 + (long long)(j0 + w + c0) * S.lda;   // row j0 of the first column
    if (t < 64) {
        int pk = -1;
        if (t < w) {
            pk = S.ipiv[j0 + t] - 1 - j0;
            if (pk < t || pk >= rows) pk = t;        // no interchange
        }
        int srow, src;
        const int ns = wave_compose32(pk, w, srow, src);
        srow_s[t] = srow;
        ssrc_s[t] = src;
        if (t == 0) nslot_s = ns;
        // source row of every top row (the wave's LDS writes stay in order)
        if (t < BMAX_NB) topsrc[t] = t;
        if (t < ns && srow < w) topsrc[srow] = src;
    }
    {
        const double *L = S.A + j0 + (long long)j0 * S.lda;
        const int i = t & 31;
#pragma unroll
        for (int r = 0; r < BMAX_NB * BMAX_NB / 256; ++r) {
            const int k = (t >> 5) + 8 * r;
            Ls[k * BMAX_NB + i] = (i < w && k < w) ? L[i + (long long)k * S.lda] : 0.0;
        }
    }
    __syncthreads();
    const int ns = nslot_s;
    // the top tile after the interchanges (row i = t % 32, 8 columns apart)
    double tv[BMAX_NB * BST_COLS / 256];
    {
        const int i = t & 31;
        const int src = topsrc[i];
#pragma unroll
        for (int r = 0; r < BMAX_NB * BST_COLS / 256; ++r) {
            const int c = (t >> 5) + 8 * r;
            tv[r] = (i < w && c < nc) ? Ac[src + (long long)c * S.lda] : 0.0;
        }
    }
    // moved rows below the top (slot x = t % 64, 4 columns apart)
    const int x = t & 63;
    const int to = srow_s[x], from = ssrc_s[x];
    const bool below = x < ns && to >= w && to != from;
    double bv[BST_COLS / 4];
#pragma unroll
    for (int r = 0; r < BST_COLS / 4; ++r) {
        const int c = (t >> 6) + 4 * r;
        bv[r] = (below && c < nc) ? Ac[from + (long long)c * S.lda] : 0.0;
    }
    {
        const int i = t & 31;
#pragma unroll
        for (int r = 0; r < BMAX_NB * BST_COLS / 256; ++r) Bt[i][(t >> 5) + 8 * r] = tv[r];
    }
    __syncthreads();                                 // every read precedes any write
#pragma unroll
    for (int r = 0; r < BST_COLS / 4; ++r) {
        const int c = (t >> 6) + 4 * r;
        if (below && c < nc) Ac[to + (long long)c * S.lda] = bv[r];
    }
    if (t < 64) {
        const int lane = t;
        double b[BMAX_NB];
#pragma unroll
        for (int i = 0; i < BMAX_NB; ++i) b[i] = Bt[i][lane];
#pragma unroll
        for (int k = 0; k < BMAX_NB - 1; ++k) {
            if (k < w - 1) {
                const double bk = b[k];
#pragma unroll
                for (int i = k + 1; i < BMAX_NB; ++i)
                    if (i < w) b[i] = b[i] - Ls[k * BMAX_NB + i] * bk;
            }
        }
#pragma unroll
        for (int i = 0; i < BMAX_NB; ++i) Bt[i][lane] = b[i];
    }
    __syncthreads();
    {
        const int i = t & 31;
#pragma unroll
        for (int r = 0; r < BMAX_NB * BST_COLS / 256; ++r) {
            const int c = (t >> 5) + 8 * r;
            if (i < w && c < nc) Ac[i + (long long)c * S.lda] = Bt[i][c];
        }
    }
}

// The interchanges of every step applied to the columns left of its panel,
// once, after the factorization: block b (columns [b nb, b nb + nb)) must
// receive those of steps b + 1, b + 2, ... in that order, i.e. column
// out[i] = in[pi_b(i)] with pi_b = sigma_{b+1} o pi_{b+1} (sigma_s: the
// row map of step s's interchanges).  One workgroup per system keeps
// Q = pi_b^-1 over the rows in LDS, walking b downwards (each step's
// interchanges composed by one wave into at most 64 moved rows update Q in
// one parallel round), and moves each row v of block b's columns to Q[v]:
// reads run down the columns, all reads of a pass before its writes.  The
// factors are those of applying the interchanges step by step.
constexpr int BSL_COLS = 8;        // columns per read/write pass
__global__ __launch_bounds__(256) void k_blaswp_left(const BSys *__restrict__ sys, int nb) {
    __shared__ int Q[BMAX_N];
    __shared__ int srow_s[2 * BMAX_NB], ssrc_s[2 * BMAX_NB];
    __shared__ int nslot_s;
    const BSys S = sys[blockIdx.x];
    const int n = S.n, t = threadIdx.x;
    const int steps = (n + nb - 1) / nb;
    if (steps < 2) return;                           // uniform per workgroup
    for (int v = t; v < n; v += 256) Q[v] = v;
    constexpr int RPT = BMAX_N / 256;                // rows per thread and column
    for (int b = steps - 2; b >= 0; --b) {
        const int j0 = (b + 1) * nb;                 // step b + 1
        const int rows = n - j0;
        const int w = nb < rows ? nb : rows;
        __syncthreads();                             // Q and the slots are free
        if (t < 64) {
            int pk = -1;
            if (t < w) {
                pk = S.ipiv[j0 + t] - 1 - j0;
                if (pk < t || pk >= rows) pk = t;    // no interchange
            }
            int srow, src;
            const int ns = wave_compose32(pk, w, srow, src);
            srow_s[t] = srow;
            ssrc_s[t] = src;
            if (t == 0) nslot_s = ns;
        }
        __syncthreads();
        // Q_b[src] = Q_{b+1}[srow] for the moved rows (reads before writes)
        const int ns = nslot_s;
        int qv = 0;
        const bool mv = t < ns && srow_s[t] != ssrc_s[t];
        if (mv) qv = Q[j0 + srow_s[t]];
        __syncthreads();
        if (mv) Q[j0 + ssrc_s[t]] = qv;
        __syncthreads();
        // block b's columns: row v (v >= j0) moves to row Q[v]
        const int cb = b * nb, ce = cb + nb;         // ce <= j0 < n
        for (int c0 = cb; c0 < ce; c0 += BSL_COLS) {
            double val[BSL_COLS][RPT];
#pragma unroll
            for (int cc = 0; cc < BSL_COLS; ++cc)
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const int v = j0 + t + 256 * k;
                    val[cc][k] = (c0 + cc < ce && v < n)
                                     ? S.A[v + (long long)(c0 + cc) * S.lda] : 0.0;
                }
            __syncthreads();                         // all reads of the pass first
#pragma unroll
            for (int cc = 0; cc < BSL_COLS; ++cc)
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const int v = j0 + t + 256 * k;
                    if (c0 + cc < ce && v < n && Q[v] != v)
                        S.A[Q[v] + (long long)(c0 + cc) * S.lda] = val[cc][k];
                }
            __syncthreads();
        }
    }
}


// ------------------------------------------------------------------ solve
// One workgroup per system: interchanges (one thread per right-hand side),
// then forward and back substitution in 64-row blocks (a wave resolves the
// diagonal block with shuffles, all threads update the other rows), in the
// same per-element order as the single-system solve.  B lives in LDS.
__global__ __launch_bounds__(1024) void k_bgetrs(const BSys *__restrict__ sys) {
    __shared__ double X[BMAX_N * BMAX_RHS];
    __shared__ int piv[BMAX_N];
    const BSys S = sys[blockIdx.x];
    const int n = S.n, nr = S.nrhs;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    for (int e = t; e < n * nr; e += blockDim.x) {
        const int i = e % n, r = e / n;
        X[r * BMAX_N + i] = S.B[i + (long long)r * S.ldb];
    }
    for (int c = t; c < n; c += blockDim.x) piv[c] = S.ipiv[c];
    __syncthreads();
    if (t < nr) {
        double *x = X + t * BMAX_N;
        for (int c = 0; c < n; ++c) {
            const int p = piv[c] - 1;
            if (p > c && p < n) {
                const double q = x[c];
                x[c] = x[p];
                x[p] = q;
            }
        }
    }
    __syncthreads();
    const double *LU = S.A;
    const long long lda = S.lda;
    for (int k0 = 0; k0 < n; k0 += 64) {
        const int kb = n - k0 < 64 ? n - k0 : 64;
        if (wid < nr) {                               // diagonal block, wave per rhs
            double *x = X + wid * BMAX_N;
            const int i = k0 + lane;
            double b = lane < kb ? x[i] : 0.0;
            // row i of the block in chunks of 16, each chunk's loads up front
#pragma unroll
            for (int kc = 0; kc < 64; kc += 16) {
                double lrow[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    lrow[u] = (kc + u < kb && lane < kb)
                                  ? LU[i + (long long)(k0 + kc + u) * lda] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int k = kc + u;
                    if (k < kb - 1) {
                        const double xk = lane_read_f64(b, k);
                        if (lane > k && lane < kb) b = b - lrow[u] * xk;
                    }
                }
            }
            if (lane < kb) x[i] = b;
        }
        __syncthreads();
        for (int e = t; e < (n - k0 - kb) * nr; e += blockDim.x) {
            const int i = k0 + kb + e % (n - k0 - kb), r = e / (n - k0 - kb);
            double *x = X + r * BMAX_N;
            double b = x[i];
#pragma unroll
            for (int kc = 0; kc < 64; kc += 16) {
                double l[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    l[u] = kc + u < kb ? LU[i + (long long)(k0 + kc + u) * lda] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (kc + u < kb) b = b - l[u] * x[k0 + kc + u];
            }
            x[i] = b;
        }
        __syncthreads();
    }
    const int last0 = (n - 1) / 64 * 64;
    for (int k0 = last0; k0 >= 0; k0 -= 64) {
        const int kb = n - k0 < 64 ? n - k0 : 64;
        if (wid < nr) {
            double *x = X + wid * BMAX_N;
            const int i = k0 + lane;
            double b = lane < kb ? x[i] : 0.0;
#pragma unroll
            for (int kc = 48; kc >= 0; kc -= 16) {
                double urow[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    urow[u] = (kc + u < kb && lane < kb)
                                  ? LU[i + (long long)(k0 + kc + u) * lda] : 0.0;
#pragma unroll
                for (int u = 15; u >= 0; --u) {
                    const int k = kc + u;
                    if (k < kb) {
                        if (lane == k) b = b / urow[u];
                        const double xk = lane_read_f64(b, k);
                        if (lane < k) b = b - urow[u] * xk;
                    }
                }
            }
            if (lane < kb) x[i] = b;
        }
        __syncthreads();
        for (int e = t; e < k0 * nr; e += blockDim.x) {
            const int i = e % k0, r = e / k0;
            double *x = X + r * BMAX_N;
            double b = x[i];
#pragma unroll
            for (int kc = 48; kc >= 0; kc -= 16) {
                double u[16];
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    u[v] = kc + v < kb ? LU[i + (long long)(k0 + kc + v) * lda] : 0.0;
#pragma unroll
                for (int v = 15; v >= 0; --v)
                    if (kc + v < kb) b = b - u[v] * x[k0 + kc + v];
            }
            x[i] = b;
        }
        __syncthreads();
    }
    for (int e = t; e < n * nr; e += blockDim.x) {
        const int i = e % n, r = e / n;
        S.B[i + (long long)r * S.ldb] = X[r * BMAX_N + i];
    }
}

__global__ void k_binfo_clear(const BSys *__restrict__ sys, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) *sys[i].info = 0;
}

// ------------------------------------------------------------------ plans
struct BatchPlan {
    int count = 0, nb = 0, s = 0, steps = 0, grid_mult = 1, nmax = 0;
    int shape = 0;                     // grouped GEMM tile (gemm_tile_counts)
    bool solve = false;
    std::vector<int> order;            // system index of sorted slot q
    std::vector<int> nact;             // active systems per step
    std::vector<int> g_off, g_cnt, g_tiles, j_off, j_cnt, j_waves;
    std::vector<GemmArgs> gemm;        // all steps
    std::vector<int> gprefix;          // per step: g_cnt + 1 entries, concatenated
    std::vector<int> gp_off;
    std::vector<SliceJob> jobs;
    std::vector<int> jprefix;
    std::vector<int> jp_off;
    std::vector<BSys> sys;             // sorted
    // scratch offsets
    size_t o_sys = 0, o_gemm = 0, o_gpre = 0, o_jobs = 0, o_jpre = 0, o_planes = 0, total = 0;
    std::vector<size_t> sys_planes;    // per sorted slot: offset of its plane region
};

static size_t region_bytes(int n, int nb, int s) {
    const int k = nb < n ? nb : n;
    const int lines = n - k > 0 ? n - k : 1;
    const Planes g = plane_geom(lines, k);
    return 2 * (align256((size_t)g.LB * 32 * sizeof(int)) + align256((size_t)s * g.plane_bytes));
}

// Shapes only: offsets, counts and scratch size.
static void plan_shape(BatchPlan &pl, int count, const int *n, const int *nrhs, int nb, int s,
                       bool solve) {
    pl.count = count;
    pl.nb = nb;
    pl.s = s;
    pl.solve = solve;
    pl.order.resize(count);
    std::iota(pl.order.begin(), pl.order.end(), 0);
    std::stable_sort(pl.order.begin(), pl.order.end(),
                     [&](int a, int b) { return n[a] > n[b]; });
    pl.nmax = count ? n[pl.order[0]] : 0;
    pl.steps = (pl.nmax + nb - 1) / nb;
    (void)nrhs;
    size_t off = 0;
    pl.o_sys = off;
    off += align256((size_t)count * sizeof(BSys));
    // count problems/jobs per step
    pl.nact.assign(pl.steps, 0);
    pl.g_off.assign(pl.steps, 0);
    pl.g_cnt.assign(pl.steps, 0);
    pl.g_tiles.assign(pl.steps, 0);
    pl.j_off.assign(pl.steps, 0);
    pl.j_cnt.assign(pl.steps, 0);
    pl.j_waves.assign(pl.steps, 0);
    pl.gp_off.assign(pl.steps, 0);
    pl.jp_off.assign(pl.steps, 0);
    int gsum = 0, jsum = 0, gps = 0, jps = 0;
    for (int st = 0; st < pl.steps; ++st) {
        const int j0 = st * nb;
        int act = 0, gc = 0;
        for (int q = 0; q < count; ++q) {
            const int ni = n[pl.order[q]];
            if (ni <= j0) break;
            ++act;
            const int jb = nb < ni - j0 ? nb : ni - j0;
            if (j0 + jb < ni) ++gc;
        }
        pl.nact[st] = act;
        pl.g_off[st] = gsum;
        pl.g_cnt[st] = gc;
        pl.j_off[st] = jsum;
        pl.j_cnt[st] = 2 * gc;
        pl.gp_off[st] = gps;
        pl.jp_off[st] = jps;
        gsum += gc;
        jsum += 2 * gc;
        gps += gc + 1;
        jps += 2 * gc + 1;
    }
    pl.o_gemm = off;
    off += align256((size_t)gsum * sizeof(GemmArgs));
    pl.o_gpre = off;
    off += align256((size_t)gps * sizeof(int));
    pl.o_jobs = off;
    off += align256((size_t)jsum * sizeof(SliceJob));
    pl.o_jpre = off;
    off += align256((size_t)jps * sizeof(int));
    pl.o_planes = off;
    pl.sys_planes.assign(count, 0);
    for (int q = 0; q < count; ++q) {
        pl.sys_planes[q] = off;
        off += region_bytes(n[pl.order[q]], nb, s);
    }
    pl.total = off;
}

// Descriptor contents for the given matrices and scratch base.
static void plan_fill(BatchPlan &pl, const int *n, const int *nrhs, double *const *A,
                      const int *lda, int *const *ipiv, int *info, double *const *B,
                      const int *ldb, char *base) {
    const int count = pl.count, nb = pl.nb, s = pl.s;
    pl.sys.resize(count);
    for (int q = 0; q < count; ++q) {
        const int i = pl.order[q];
        BSys &S = pl.sys[q];
        S.A = A[i];
        S.lda = lda[i];
        S.n = n[i];
        S.nrhs = nrhs ? nrhs[i] : 0;
        S.ipiv = ipiv[i];
        S.info = info + i;
        S.B = B ? B[i] : nullptr;
        S.ldb = ldb ? ldb[i] : 1;
    }
    pl.gemm.clear();
    pl.jobs.clear();
    pl.gprefix.clear();
    pl.jprefix.clear();
    for (int st = 0; st < pl.steps; ++st) {
        const int j0 = st * nb;
        int tiles = 0, waves = 0;
        pl.gprefix.push_back(0);
        pl.jprefix.push_back(0);
        for (int q = 0; q < pl.nact[st]; ++q) {
            const BSys &S = pl.sys[q];
            const int jb = nb < S.n - j0 ? nb : S.n - j0;
            const int j1 = j0 + jb;
            if (j1 >= S.n) continue;
            const int lines = S.n - j1;
            const Planes g = plane_geom(lines, jb);
            char *reg = base + pl.sys_planes[q];
            const size_t half = region_bytes(S.n, nb, s) / 2;
            int *codeA = reinterpret_cast<int *>(reg);
            int8_t *pa = reinterpret_cast<int8_t *>(reg + align256((size_t)g.LB * 32 * sizeof(int)));
            int *codeB = reinterpret_cast<int *>(reg + half);
            int8_t *pb = reinterpret_cast<int8_t *>(reg + half +
                                                    align256((size_t)g.LB * 32 * sizeof(int)));
            SliceJob ja{S.A + j1 + (long long)j0 * S.lda, S.lda, lines, jb, 1, g.LB, codeA, pa,
                        g.plane_bytes};
            SliceJob jbj{S.A + j0 + (long long)j1 * S.lda, S.lda, lines, jb, 0, g.LB, codeB, pb,
                         g.plane_bytes};
            pl.jobs.push_back(ja);
            waves += g.LB;
            pl.jprefix.push_back(waves);
            pl.jobs.push_back(jbj);
            waves += g.LB;
            pl.jprefix.push_back(waves);
            GemmArgs ga{};
            ga.Ap = pa;
            ga.Bp = pb;
            ga.a_plane = g.plane_bytes;
            ga.b_plane = g.plane_bytes;
            ga.codeA = codeA;
            ga.codeB = codeB;
            ga.M = lines;
            ga.N = lines;
            ga.KB = g.KB;
            ga.alpha = -1.0;
            ga.beta = 1.0;
            ga.C = S.A + j1 + (long long)j1 * S.lda;
            ga.ldc = S.lda;
            gemm_tile_counts(s, lines, lines, &ga.tiles_m, &ga.tiles_n, pl.shape);
            pl.gemm.push_back(ga);
            tiles += ga.tiles_m * ga.tiles_n;
            pl.gprefix.push_back(tiles);
        }
        pl.g_tiles[st] = tiles;
        pl.j_waves[st] = waves;
    }
}

// Host staging of the descriptor tables: one pinned buffer (grown on
// demand, guarded by g_bmu) mirroring the device layout [0, o_planes), so a
// call uploads all tables with a single DMA instead of many staged copies
// from pageable memory.
static void *g_pinned = nullptr;
static size_t g_pinned_bytes = 0;

static int pinned_reserve(size_t bytes) {
    if (bytes > g_pinned_bytes) {
        if (g_pinned) EMU_TRY_HIP(hipHostFree(g_pinned));
        g_pinned = nullptr;
        g_pinned_bytes = 0;
        EMU_TRY_HIP(hipHostMalloc(&g_pinned, bytes, hipHostMallocDefault));
        g_pinned_bytes = bytes;
    }
    return 0;
}

static int plan_upload(const BatchPlan &pl, char *base, hipStream_t st) {
    const size_t bytes = pl.o_planes;
    EMU_TRY(pinned_reserve(bytes));
    char *h = static_cast<char *>(g_pinned);
    std::memcpy(h + pl.o_sys, pl.sys.data(), pl.sys.size() * sizeof(BSys));
    if (!pl.gemm.empty()) {
        std::memcpy(h + pl.o_gemm, pl.gemm.data(), pl.gemm.size() * sizeof(GemmArgs));
        std::memcpy(h + pl.o_gpre, pl.gprefix.data(), pl.gprefix.size() * sizeof(int));
        std::memcpy(h + pl.o_jobs, pl.jobs.data(), pl.jobs.size() * sizeof(SliceJob));
        std::memcpy(h + pl.o_jpre, pl.jprefix.data(), pl.jprefix.size() * sizeof(int));
    }
    EMU_TRY_HIP(hipMemcpyAsync(base, h, bytes, hipMemcpyHostToDevice, st));
    // the staging buffer is refilled on the next call: wait for the copy
    EMU_TRY_HIP(hipStreamSynchronize(st));
    return 0;
}

static int plan_launch(const BatchPlan &pl, char *base, int *status, int cus, hipStream_t st) {
    const BSys *sys = reinterpret_cast<const BSys *>(base + pl.o_sys);
    hipLaunchKernelGGL(k_binfo_clear, dim3((pl.count + 255) / 256), dim3(256), 0, st, sys,
                       pl.count);
    const int ggrid = cus * gemm_grouped_blocks_per_cu(pl.s, pl.shape) * pl.grid_mult;
    for (int stp = 0; stp < pl.steps; ++stp) {
        const int j0 = stp * pl.nb;
        const int act = pl.nact[stp];
        hipLaunchKernelGGL(k_bpanel, dim3(act), dim3(1024), 0, st, sys, j0, pl.nb);
        hipLaunchKernelGGL(k_bswap_trsm, dim3((pl.nmax + BST_COLS - 1) / BST_COLS, act),
                           dim3(256), 0, st, sys, j0, pl.nb);
        EMU_TRY_HIP(hipGetLastError());
        if (pl.g_cnt[stp] > 0) {
            const SliceJob *jobs = reinterpret_cast<const SliceJob *>(base + pl.o_jobs) +
                                   pl.j_off[stp];
            const int *jpre = reinterpret_cast<const int *>(base + pl.o_jpre) + pl.jp_off[stp];
            EMU_TRY(launch_slice_small_grouped(jobs, jpre, pl.j_cnt[stp], pl.j_waves[stp], pl.s,
                                               status, st));
            const GemmArgs *probs = reinterpret_cast<const GemmArgs *>(base + pl.o_gemm) +
                                    pl.g_off[stp];
            const int *gpre = reinterpret_cast<const int *>(base + pl.o_gpre) + pl.gp_off[stp];
            EMU_TRY(launch_slicegemm_grouped(probs, gpre, pl.g_cnt[stp], pl.g_tiles[stp], ggrid,
                                             pl.s, st, /*one_kstep=*/true, pl.shape));
        }
    }
    hipLaunchKernelGGL(k_blaswp_left, dim3(pl.count), dim3(256), 0, st, sys, pl.nb);
    EMU_TRY_HIP(hipGetLastError());
    if (pl.solve) {
        hipLaunchKernelGGL(k_bgetrs, dim3(pl.count), dim3(1024), 0, st, sys);
        EMU_TRY_HIP(hipGetLastError());
    }
    return 0;
}


// --------------------------------------------------- batched refinement
// Precision form for a batch: every system is factored (grouped, as above)
// from a copy of A with s slices and solved; then, per system, the FP64
// residual r = b - A x and eta = max_r ||r||_inf / (||A||_inf ||x||_inf +
// ||b||_inf) (the single-system form's stopping quantity), a solve with the
// stored factors and x += d, until eta <= tol.  A system whose eta stops
// halving, exceeds the step budget or is NaN is refactored with two slices
// more (up to nine), the others keep their result.  All systems still
// refining take one grouped launch per phase.
struct BIr {
    const double *A;
    long long lda;
    const double *B;
    long long ldb;
    double *X;
    long long ldx;
    double *R;          // n x nrhs, leading dimension n
    int n, nrhs;
};

struct BCopy {
    const double *src;
    long long lds;
    double *dst;
    long long ldd;
    int rows, cols;
};

__global__ __launch_bounds__(256) void k_bcopy(const BCopy *__restrict__ jobs) {
    const BCopy J = jobs[blockIdx.x];
    // four columns per pass, all loads of a pass before its stores
    for (int j0 = 0; j0 < J.cols; j0 += 4) {
        for (int i = threadIdx.x; i < J.rows; i += 256) {
            double v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                v[c] = j0 + c < J.cols ? J.src[i + (long long)(j0 + c) * J.lds] : 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (j0 + c < J.cols) J.dst[i + (long long)(j0 + c) * J.ldd] = v[c];
        }
    }
}

// One workgroup per system: R = B - A X (each entry: the products a_ij x_j
// accumulated with fma in increasing j, then subtracted from b), and eta.
__global__ __launch_bounds__(256) void k_bresid(const BIr *__restrict__ sys,
                                                double *__restrict__ eta) {
    __shared__ double xs[BMAX_N * BMAX_RHS];
    __shared__ double red[4][1 + 3 * BMAX_RHS];
    const BIr S = sys[blockIdx.x];
    const int n = S.n, nr = S.nrhs, t = threadIdx.x, lane = t & 63, wid = t >> 6;
    for (int e = t; e < n * nr; e += blockDim.x)
        xs[(e / n) * BMAX_N + e % n] = S.X[e % n + (long long)(e / n) * S.ldx];
    __syncthreads();
    double mA = 0.0, mR[BMAX_RHS], mX[BMAX_RHS], mB[BMAX_RHS];
#pragma unroll
    for (int r = 0; r < BMAX_RHS; ++r) mR[r] = mX[r] = mB[r] = 0.0;
    // the thread's rows i = t + 256 q walk the columns together, so their
    // loads are in flight at once; each row's sums run over j in order
    constexpr int RPT = BMAX_N / 256;
    double ax[RPT][BMAX_RHS], ra[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        ra[q] = 0.0;
#pragma unroll
        for (int r = 0; r < BMAX_RHS; ++r) ax[q][r] = 0.0;
    }
#pragma unroll 4
    for (int j = 0; j < n; ++j) {
        double a[RPT], xv[BMAX_RHS];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = t + 256 * q;
            a[q] = i < n ? S.A[i + (long long)j * S.lda] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < BMAX_RHS; ++r) xv[r] = r < nr ? xs[r * BMAX_N + j] : 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            ra[q] += fabs(a[q]);
#pragma unroll
            for (int r = 0; r < BMAX_RHS; ++r)
                if (r < nr) ax[q][r] = fma(a[q], xv[r], ax[q][r]);
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = t + 256 * q;
        if (i >= n) continue;
        mA = fmax(mA, ra[q]);
#pragma unroll
        for (int r = 0; r < BMAX_RHS; ++r) {
            if (r < nr) {
                const double b = S.B[i + (long long)r * S.ldb];
                const double rv = b - ax[q][r];
                S.R[i + (long long)r * n] = rv;
                mR[r] = (rv != rv || mR[r] != mR[r]) ? __builtin_nan("") : fmax(mR[r], fabs(rv));
                mX[r] = fmax(mX[r], fabs(xs[r * BMAX_N + i]));
                mB[r] = fmax(mB[r], fabs(b));
            }
        }
    }
    // workgroup maxima (NaN in a residual is kept)
    auto wmax = [&](double v) {
        for (int o = 32; o > 0; o >>= 1) {
            const double w = __shfl_xor(v, o);
            v = (v != v || w != w) ? __builtin_nan("") : fmax(v, w);
        }
        return v;
    };
    mA = wmax(mA);
#pragma unroll
    for (int r = 0; r < BMAX_RHS; ++r) {
        mR[r] = wmax(mR[r]);
        mX[r] = wmax(mX[r]);
        mB[r] = wmax(mB[r]);
    }
    if (lane == 0) {
        red[wid][0] = mA;
#pragma unroll
        for (int r = 0; r < BMAX_RHS; ++r) {
            red[wid][1 + 3 * r] = mR[r];
            red[wid][2 + 3 * r] = mX[r];
            red[wid][3 + 3 * r] = mB[r];
        }
    }
    __syncthreads();
    if (t == 0) {
        double nA = 0.0, e = 0.0;
        for (int w = 0; w < 4; ++w) nA = fmax(nA, red[w][0]);
        for (int r = 0; r < nr; ++r) {
            double R = 0.0, X = 0.0, B = 0.0;
            bool nan = false;
            for (int w = 0; w < 4; ++w) {
                const double v = red[w][1 + 3 * r];
                nan = nan || v != v;
                R = fmax(R, v);
                X = fmax(X, red[w][2 + 3 * r]);
                B = fmax(B, red[w][3 + 3 * r]);
            }
            const double den = nA * X + B;
            const double er = nan ? __builtin_nan("") : (den > 0.0 ? R / den : R);
            if (!(er <= e)) e = er;
        }
        eta[blockIdx.x] = e;
    }
}

// X += R (the correction the solve left in R), one workgroup per system.
__global__ __launch_bounds__(256) void k_badd(const BIr *__restrict__ sys) {
    const BIr S = sys[blockIdx.x];
    for (int e = threadIdx.x; e < S.n * S.nrhs; e += blockDim.x) {
        const int i = e % S.n, r = e / S.n;
        double *x = S.X + i + (long long)r * S.ldx;
        *x = *x + S.R[i + (long long)r * S.n];
    }
}

// ------------------------------------------------------ graph cache, tuning
struct GraphEntry {
    BatchPlan plan;
    hipGraphExec_t exec = nullptr;
    void *ws = nullptr;
};
static std::mutex g_bmu;
static std::map<std::string, GraphEntry> g_graphs;
struct Tuned {
    int nb, mult, shape;
};
static std::map<std::string, Tuned> g_tuned;   // batch shape -> choice
static bool g_tuned_loaded = false;

static std::string shape_key(int count, const int *n, const int *nrhs, int nb, int s,
                             bool solve, int mult, int tile) {
    std::string k = std::to_string(count) + ":" + std::to_string(nb) + ":" + std::to_string(s) +
                    ":" + (solve ? "1" : "0") + ":" + std::to_string(mult) + ":" +
                    std::to_string(tile) + ":";
    unsigned long long h = 1469598103934665603ull;
    for (int i = 0; i < count; ++i) {
        h = (h ^ (unsigned long long)n[i]) * 1099511628211ull;
        h = (h ^ (unsigned long long)(nrhs ? nrhs[i] : 0)) * 1099511628211ull;
    }
    return k + std::to_string(h);
}

// Tuning key: the device architecture and HIP runtime version, then the
// batch's coarse shape (count, largest n, slice count).
// Key prefix of the tuning table: device architecture and HIP runtime
// version, so a table file written on other hardware or software is not used.
static std::string tune_prefix() {
    static thread_local std::string prefix;
    if (prefix.empty()) {
        int dev = 0, rt = 0;
        hipDeviceProp_t prop;
        std::string arch = "unknown";
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            arch = prop.gcnArchName;
            for (char &c : arch)
                if (c == ' ' || c == ':') c = '_';
        }
        if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
        prefix = arch + "/hip" + std::to_string(rt) + "/";
    }
    return prefix;
}

static std::string tune_key(int count, int nmax, int s) {
    return tune_prefix() + std::to_string(count) + "/" + std::to_string(nmax) + "/" +
           std::to_string(s);
}

static std::string getrf_key(int m, int n, int s) {
    return tune_prefix() + "getrf/" + std::to_string(m) + "/" + std::to_string(n) + "/" +
           std::to_string(s);
}

static const char *tune_file() { return std::getenv("EMU_AUTOTUNE_CACHE"); }

// tile shape of batched calls with an explicit block size (emu_set_param
// "batched_tile"); the autotuned choice applies when nb = 0
static thread_local int g_batched_tile = 0;

static void tune_load() {
    if (g_tuned_loaded) return;
    g_tuned_loaded = true;
    const char *f = tune_file();
    if (!f) return;
    FILE *fp = std::fopen(f, "r");
    if (!fp) return;
    // one entry per line: "key nb grid_mult tile_shape"
    char key[256];
    int nb, mult, tile;
    while (std::fscanf(fp, "%255s %d %d %d", key, &nb, &mult, &tile) == 4)
        g_tuned[key] = {nb, mult, tile};
    std::fclose(fp);
}

static void tune_save() {
    const char *f = tune_file();
    if (!f) return;
    FILE *fp = std::fopen(f, "w");
    if (!fp) return;
    for (auto &kv : g_tuned)
        std::fprintf(fp, "%s %d %d %d\n", kv.first.c_str(), kv.second.nb, kv.second.mult,
                     kv.second.shape);
    std::fclose(fp);
}

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

static int check_batch(int count, const int *n, const int *nrhs, double *const *A, const int *lda,
                       int *const *ipiv, int *info, double *const *B, const int *ldb, int nb,
                       int nslices, bool solve) {
    if (count < 0) return -1;
    if (count > 0 && !n) return -2;
    if (solve && count > 0 && !nrhs) return -3;
    if (count > 0 && !A) return -4;
    if (count > 0 && !lda) return -5;
    if (count > 0 && !ipiv) return -6;
    if (count > 0 && !info) return -7;
    if (solve && count > 0 && (!B || !ldb)) return -8;
    if (nb < 0 || nb > BMAX_NB) return -9;
    if (nslices < 1 || nslices > GROUPED_MAX_SLICES) return -10;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 1 || n[i] > BMAX_N) {
            set_error("batched: system %d has n = %d (supported 1..%d)", i, n[i], BMAX_N);
            return EMU_ERR_UNSUPPORTED;
        }
        if (!A[i] || lda[i] < n[i] || !ipiv[i]) return -4;
        if (solve) {
            if (nrhs[i] < 1 || nrhs[i] > BMAX_RHS) {
                set_error("batched: system %d has %d right-hand sides (1..%d)", i, nrhs[i],
                          BMAX_RHS);
                return EMU_ERR_UNSUPPORTED;
            }
            if (!B[i] || ldb[i] < n[i]) return -8;
        }
    }
    return 0;
}

// Factor (and solve) a batch through the cached graph of its shape.  A graph
// is tied to the scratch it was captured with (its descriptor tables and
// digit planes live there): a call whose scratch is elsewhere captures anew.
static int run_batch(int count, const int *n, const int *nrhs, double *const *A,
                     const int *lda, int *const *ipiv, int *info, double *const *B,
                     const int *ldb, int nb, int nslices, int mult, bool solve, int tile = 0) {
    std::lock_guard<std::mutex> lk(g_bmu);
    if (nslices < 6) tile = 0;          // one tile shape below six slices
    const std::string key = shape_key(count, n, nrhs, nb, nslices, solve, mult, tile);
    auto it = g_graphs.find(key);
    GraphEntry e;
    size_t need;
    if (it != g_graphs.end()) {
        need = it->second.plan.total;
    } else {
        plan_shape(e.plan, count, n, nrhs, nb, nslices, solve);
        e.plan.grid_mult = mult;
        e.plan.shape = tile;
        need = e.plan.total;
    }
    Call call;
    EMU_TRY(call.begin(need));
    hipStream_t st = call.st;
    char *base = call.ws;
    if (it != g_graphs.end() && it->second.ws != base) {
        e.plan = std::move(it->second.plan);
        if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
        g_graphs.erase(it);
        it = g_graphs.end();
    }
    if (it == g_graphs.end()) {
        plan_fill(e.plan, n, nrhs, A, lda, ipiv, info, B, ldb, base);
        EMU_TRY(plan_upload(e.plan, base, st));
        hipStream_t cap;
        EMU_TRY_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        EMU_TRY_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        int rc = plan_launch(e.plan, base, call.dev->status, device_cus(), cap);
        hipGraph_t graph = nullptr;
        hipError_t ec = hipStreamEndCapture(cap, &graph);
        (void)hipStreamDestroy(cap);
        if (rc != 0) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ec != hipSuccess) return fail_hip(ec, "hipStreamEndCapture");
        ec = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ec != hipSuccess) return fail_hip(ec, "hipGraphInstantiate");
        e.ws = base;
        it = g_graphs.emplace(key, std::move(e)).first;
    } else {
        plan_fill(it->second.plan, n, nrhs, A, lda, ipiv, info, B, ldb, base);
        EMU_TRY(plan_upload(it->second.plan, base, st));
    }
    EMU_TRY_HIP(hipGraphLaunch(it->second.exec, st));
    return 0;
}

void set_batched_tile(int tile) { g_batched_tile = tile; }

int tuned_getrf_nb(int m, int n, int s) {
    std::lock_guard<std::mutex> lk(g_bmu);
    tune_load();
    auto it = g_tuned.find(getrf_key(m, n, s));
    return it != g_tuned.end() ? it->second.nb : 0;
}

void record_getrf_nb(int m, int n, int s, int nb) {
    std::lock_guard<std::mutex> lk(g_bmu);
    tune_load();
    g_tuned[getrf_key(m, n, s)] = {nb, 0, 0};
    tune_save();
}

}  // namespace emu

using namespace emu;

extern "C" {

int emu_dgetrf_batched(int count, const int *n, double *const *A, const int *lda,
                       int *const *ipiv, int *info, int nb, int nslices) {
    int bad = check_batch(count, n, nullptr, A, lda, ipiv, info, nullptr, nullptr, nb, nslices,
                          false);
    if (bad) return bad;
    if (count == 0) return 0;
    int mult = 1, tile = g_batched_tile;
    if (nb == 0) {
        std::lock_guard<std::mutex> lk(g_bmu);
        tune_load();
        int nmax = *std::max_element(n, n + count);
        auto t = g_tuned.find(tune_key(count, nmax, nslices));
        nb = t != g_tuned.end() ? t->second.nb : BMAX_NB;
        mult = t != g_tuned.end() ? t->second.mult : 1;
        tile = t != g_tuned.end() ? t->second.shape : 0;
    }
    return run_batch(count, n, nullptr, A, lda, ipiv, info, nullptr, nullptr, nb, nslices, mult,
                     false, tile);
}

int emu_dgesv_batched(int count, const int *n, const int *nrhs, double *const *A,
                      const int *lda, int *const *ipiv, int *info, double *const *B,
                      const int *ldb, int nb, int nslices) {
    int bad = check_batch(count, n, nrhs, A, lda, ipiv, info, B, ldb, nb, nslices, true);
    if (bad) return bad;
    if (count == 0) return 0;
    int mult = 1, tile = g_batched_tile;
    if (nb == 0) {
        std::lock_guard<std::mutex> lk(g_bmu);
        tune_load();
        int nmax = *std::max_element(n, n + count);
        auto t = g_tuned.find(tune_key(count, nmax, nslices));
        nb = t != g_tuned.end() ? t->second.nb : BMAX_NB;
        mult = t != g_tuned.end() ? t->second.mult : 1;
        tile = t != g_tuned.end() ? t->second.shape : 0;
    }
    return run_batch(count, n, nrhs, A, lda, ipiv, info, B, ldb, nb, nslices, mult, true, tile);
}

int emu_dgetrs_batched(int count, const int *n, const int *nrhs, const double *const *LU,
                       const int *lda, const int *const *ipiv, double *const *B,
                       const int *ldb) {
    if (count < 0) return -1;
    if (count == 0) return 0;
    if (!n) return -2;
    if (!nrhs) return -3;
    if (!LU) return -4;
    if (!lda) return -5;
    if (!ipiv) return -6;
    if (!B) return -7;
    if (!ldb) return -8;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 1 || n[i] > BMAX_N) {
            set_error("batched solve: system %d has n = %d (supported 1..%d)", i, n[i], BMAX_N);
            return EMU_ERR_UNSUPPORTED;
        }
        if (nrhs[i] < 1 || nrhs[i] > BMAX_RHS) {
            set_error("batched solve: system %d has %d right-hand sides (1..%d)", i, nrhs[i],
                      BMAX_RHS);
            return EMU_ERR_UNSUPPORTED;
        }
        if (!LU[i]) return -4;
        if (lda[i] < n[i]) return -5;
        if (!ipiv[i]) return -6;
        if (!B[i]) return -7;
        if (ldb[i] < n[i]) return -8;
    }
    std::vector<BSys> sys(count);
    for (int i = 0; i < count; ++i) {
        BSys &S = sys[i];
        S.A = const_cast<double *>(LU[i]);        // read only by the solve
        S.lda = lda[i];
        S.n = n[i];
        S.nrhs = nrhs[i];
        S.ipiv = const_cast<int *>(ipiv[i]);
        S.info = nullptr;
        S.B = B[i];
        S.ldb = ldb[i];
    }
    const size_t bytes = (size_t)count * sizeof(BSys);
    std::lock_guard<std::mutex> lk(g_bmu);     // guards the pinned staging buffer
    Call call;
    EMU_TRY(call.begin(bytes));
    EMU_TRY(pinned_reserve(bytes));
    std::memcpy(g_pinned, sys.data(), bytes);
    EMU_TRY_HIP(hipMemcpyAsync(call.ws, g_pinned, bytes, hipMemcpyHostToDevice, call.st));
    // the staging buffer is refilled on the next call: wait for the copy
    EMU_TRY_HIP(hipStreamSynchronize(call.st));
    hipLaunchKernelGGL(k_bgetrs, dim3(count), dim3(1024), 0, call.st,
                       reinterpret_cast<const BSys *>(call.ws));
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int emu_dgesv_batched_ir(int count, const int *n, const int *nrhs, const double *const *A,
                         const int *lda, const double *const *B, const int *ldb,
                         double *const *X, const int *ldx, int nb, int nslices, double tol,
                         int maxiter, int *iters, double *berr, int *s_final, int *info) {
    if (count < 0) return -1;
    if (count > 0 && (!n || !nrhs)) return -2;
    if (count > 0 && (!A || !lda)) return -4;
    if (count > 0 && (!B || !ldb)) return -6;
    if (count > 0 && (!X || !ldx)) return -8;
    if (nb < 0 || nb > BMAX_NB) return -10;
    if (nslices < 1 || nslices > GROUPED_MAX_SLICES) return -11;
    if (!(tol > 0.0)) return -12;
    if (maxiter < 0) return -13;
    if (count > 0 && (!iters || !berr || !s_final || !info)) return -14;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 1 || n[i] > BMAX_N || nrhs[i] < 1 || nrhs[i] > BMAX_RHS) {
            set_error("batched refinement: system %d has n = %d, nrhs = %d (1..%d, 1..%d)", i,
                      n[i], nrhs[i], BMAX_N, BMAX_RHS);
            return EMU_ERR_UNSUPPORTED;
        }
        if (!A[i] || lda[i] < n[i]) return -4;
        if (!B[i] || ldb[i] < n[i]) return -6;
        if (!X[i] || ldx[i] < n[i]) return -8;
        iters[i] = 0;
        berr[i] = 0.0;
        s_final[i] = nslices;
        info[i] = 0;
    }
    if (count == 0) return 0;
    if (nb == 0) nb = BMAX_NB;
    Device *dev;
    hipStream_t st;
    EMU_TRY(current(&dev, &st));
    // private memory of this call: factors, pivots, info, residuals, eta,
    // descriptor tables
    std::vector<size_t> o_lu(count), o_piv(count), o_r(count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        o_lu[i] = off;
        off += align256((size_t)n[i] * n[i] * sizeof(double));
        o_piv[i] = off;
        off += align256((size_t)n[i] * sizeof(int));
        o_r[i] = off;
        off += align256((size_t)n[i] * nrhs[i] * sizeof(double));
    }
    const size_t o_info = off;
    off += align256((size_t)count * sizeof(int));
    const size_t o_eta = off;
    off += align256((size_t)count * sizeof(double));
    const size_t o_ir = off;
    off += align256((size_t)count * sizeof(BIr));
    const size_t o_cp = off;
    off += align256((size_t)2 * count * sizeof(BCopy));
    char *mem = nullptr;
    EMU_TRY_HIP(hipMalloc(&mem, off));
    struct Free {
        char *p;
        hipStream_t st;
        ~Free() {
            (void)hipStreamSynchronize(st);
            (void)hipFree(p);
        }
    } guard{mem, st};
    auto LUp = [&](int i) { return reinterpret_cast<double *>(mem + o_lu[i]); };
    auto PIVp = [&](int i) { return reinterpret_cast<int *>(mem + o_piv[i]); };
    auto Rp = [&](int i) { return reinterpret_cast<double *>(mem + o_r[i]); };
    int *dinfo = reinterpret_cast<int *>(mem + o_info);
    double *deta = reinterpret_cast<double *>(mem + o_eta);
    BIr *dir = reinterpret_cast<BIr *>(mem + o_ir);
    BCopy *dcp = reinterpret_cast<BCopy *>(mem + o_cp);

    std::vector<int> todo(count);             // systems to (re)factor
    std::iota(todo.begin(), todo.end(), 0);
    // host descriptor tables, alive for the whole call: each is rewritten
    // only after a stream synchronization that follows its last upload
    std::vector<BIr> ir, ir2;
    std::vector<BSys> sol;
    ir.reserve(count);
    ir2.reserve(count);
    sol.reserve(count);
    std::vector<double> prev(count), heta(count);
    int s = nslices;
    int rc_all = 0;
    while (!todo.empty()) {
        const int c = (int)todo.size();
        // copies A -> LU, B -> X of the systems to factor
        std::vector<BCopy> cp(2 * c);
        std::vector<int> sn(c), snr(c), sld(c), sldx(c);
        std::vector<double *> sA(c), sX(c);
        std::vector<int *> spiv(c);
        for (int q = 0; q < c; ++q) {
            const int i = todo[q];
            cp[2 * q] = {A[i], lda[i], LUp(i), n[i], n[i], n[i]};
            cp[2 * q + 1] = {B[i], ldb[i], X[i], ldx[i], n[i], nrhs[i]};
            sn[q] = n[i];
            snr[q] = nrhs[i];
            sld[q] = n[i];
            sldx[q] = ldx[i];
            sA[q] = LUp(i);
            sX[q] = X[i];
            spiv[q] = PIVp(i);
        }
        EMU_TRY_HIP(hipMemcpyAsync(dcp, cp.data(), cp.size() * sizeof(BCopy),
                                   hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_bcopy, dim3(2 * c), dim3(256), 0, st, dcp);
        EMU_TRY_HIP(hipGetLastError());
        EMU_TRY(run_batch(c, sn.data(), snr.data(), sA.data(), sld.data(), spiv.data(), dinfo,
                          sX.data(), sldx.data(), nb, s, 1, true));
        std::vector<int> hinfo(c);
        EMU_TRY_HIP(hipMemcpyAsync(hinfo.data(), dinfo, c * sizeof(int), hipMemcpyDeviceToHost,
                                   st));
        EMU_TRY_HIP(hipStreamSynchronize(st));
        std::vector<int> act;                 // systems refining
        for (int q = 0; q < c; ++q) {
            const int i = todo[q];
            info[i] = hinfo[q];
            s_final[i] = s;
            prev[i] = -1.0;
            if (hinfo[q] == 0) act.push_back(i);
        }
        std::vector<int> fall;                // systems to refactor with more slices
        for (int it = 0; !act.empty(); ++it) {
            const int a = (int)act.size();
            ir.resize(a);
            for (int q = 0; q < a; ++q) {
                const int i = act[q];
                ir[q] = {A[i], lda[i], B[i], ldb[i], X[i], ldx[i], Rp(i), n[i], nrhs[i]};
            }
            EMU_TRY_HIP(hipMemcpyAsync(dir, ir.data(), a * sizeof(BIr), hipMemcpyHostToDevice,
                                       st));
            hipLaunchKernelGGL(k_bresid, dim3(a), dim3(256), 0, st, dir, deta);
            EMU_TRY_HIP(hipGetLastError());
            EMU_TRY_HIP(hipMemcpyAsync(heta.data(), deta, a * sizeof(double),
                                       hipMemcpyDeviceToHost, st));
            EMU_TRY_HIP(hipStreamSynchronize(st));
            std::vector<int> next;
            sol.clear();
            for (int q = 0; q < a; ++q) {
                const int i = act[q];
                const double e = heta[q];
                berr[i] = e;
                if (e <= tol) continue;
                if (it >= maxiter || (prev[i] >= 0.0 && !(e <= 0.5 * prev[i])) || e != e) {
                    fall.push_back(i);
                    continue;
                }
                prev[i] = e;
                ++iters[i];
                next.push_back(i);
                BSys S{};
                S.A = LUp(i);
                S.lda = n[i];
                S.n = n[i];
                S.nrhs = nrhs[i];
                S.ipiv = PIVp(i);
                S.info = dinfo;
                S.B = Rp(i);
                S.ldb = n[i];
                sol.push_back(S);
            }
            if (!next.empty()) {
                // correction: d = solve(LU, r) in R, then x += d
                const int b = (int)next.size();
                static_assert(sizeof(BSys) <= 2 * sizeof(BCopy), "descriptor space");
                BSys *dsys = reinterpret_cast<BSys *>(dcp);     // the copies are done
                EMU_TRY_HIP(hipMemcpyAsync(dsys, sol.data(), b * sizeof(BSys),
                                           hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_bgetrs, dim3(b), dim3(1024), 0, st, dsys);
                ir2.resize(b);
                for (int q = 0; q < b; ++q) {
                    const int i = next[q];
                    ir2[q] = {A[i], lda[i], B[i], ldb[i], X[i], ldx[i], Rp(i), n[i], nrhs[i]};
                }
                EMU_TRY_HIP(hipMemcpyAsync(dir, ir2.data(), b * sizeof(BIr),
                                           hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_badd, dim3(b), dim3(256), 0, st, dir);
                EMU_TRY_HIP(hipGetLastError());
            }
            act.swap(next);
        }
        if (fall.empty()) break;
        if (s >= GROUPED_MAX_SLICES) {
            set_error("batched refinement: %zu system(s) missed %g at %d slices", fall.size(),
                      tol, s);
            rc_all = EMU_ERR_NOT_CONVERGED;
            break;
        }
        s = s + 2 < GROUPED_MAX_SLICES ? s + 2 : GROUPED_MAX_SLICES;
        todo.swap(fall);
    }
    return rc_all;
}

int emu_autotune_batched(int count, const int *n, const int *nrhs, double *const *A,
                         const int *lda, double *const *B, const int *ldb, int nslices,
                         int *best_nb, int *best_mult, double *best_ms, int *best_tile) {
    if (count <= 0) return -1;
    if (!best_nb || !best_mult || !best_ms || !best_tile) return -9;
    std::vector<int *> piv(count, nullptr);
    // private copies: the tuning runs factor in place
    std::vector<double *> Ac(count, nullptr), Bc(count, nullptr);
    std::vector<int> ldc(count), ldbc(count);
    int *dinfo = nullptr;
    int rc = 0;
    Device *dev;
    hipStream_t st;
    EMU_TRY(current(&dev, &st));
    EMU_TRY_HIP(hipMalloc(&dinfo, count * sizeof(int)));
    for (int i = 0; i < count && rc == 0; ++i) {
        ldc[i] = n[i];
        ldbc[i] = n[i];
        if (hipMalloc(&Ac[i], (size_t)n[i] * n[i] * sizeof(double)) != hipSuccess ||
            hipMalloc(&Bc[i], (size_t)n[i] * nrhs[i] * sizeof(double)) != hipSuccess ||
            hipMalloc(&piv[i], n[i] * sizeof(int)) != hipSuccess)
            rc = EMU_ERR_WORKSPACE;
    }
    const int nbs[2] = {16, 32};
    const int mults[2] = {1, 2};
    const int ntiles = nslices >= 6 ? 2 : 1;    // 64 x 128 and 64 x 64 (s >= 6)
    double best = 1e30;
    int bnb = BMAX_NB, bm = 1, bt = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == 0 && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = EMU_ERR_HIP;
    for (int a = 0; a < 2 && rc == 0; ++a)
        for (int b = 0; b < 2 && rc == 0; ++b)
        for (int c = 0; c < ntiles && rc == 0; ++c) {
            float ms = 0.f;
            for (int rep = 0; rep < 2 && rc == 0; ++rep) {
                for (int i = 0; i < count; ++i) {
                    (void)hipMemcpy2DAsync(Ac[i], n[i] * sizeof(double), A[i],
                                           lda[i] * sizeof(double), n[i] * sizeof(double), n[i],
                                           hipMemcpyDeviceToDevice, st);
                    (void)hipMemcpy2DAsync(Bc[i], n[i] * sizeof(double), B[i],
                                           ldb[i] * sizeof(double), n[i] * sizeof(double),
                                           nrhs[i], hipMemcpyDeviceToDevice, st);
                }
                (void)hipEventRecord(e0, st);
                rc = run_batch(count, n, nrhs, Ac.data(), ldc.data(), piv.data(), dinfo,
                               Bc.data(), ldbc.data(), nbs[a], nslices, mults[b], true, c);
                (void)hipEventRecord(e1, st);
                (void)hipEventSynchronize(e1);
                (void)hipEventElapsedTime(&ms, e0, e1);
            }
            if (rc == 0 && ms < best) {
                best = ms;
                bnb = nbs[a];
                bm = mults[b];
                bt = c;
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    for (int i = 0; i < count; ++i) {
        if (Ac[i]) (void)hipFree(Ac[i]);
        if (Bc[i]) (void)hipFree(Bc[i]);
        if (piv[i]) (void)hipFree(piv[i]);
    }
    (void)hipFree(dinfo);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        tune_load();
        const int nmax = *std::max_element(n, n + count);
        g_tuned[tune_key(count, nmax, nslices)] = {bnb, bm, bt};
        tune_save();
    }
    *best_nb = bnb;
    *best_mult = bm;
    *best_ms = best;
    *best_tile = bt;
    return 0;
}

}  // extern "C"
