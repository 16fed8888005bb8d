// Internal declarations shared by the library's translation units.
// Not installed; the public interface is include/emu.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <limits.h>

#include "../../include/emu.h"

namespace emu {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
int fail_hip(hipError_t e, const char *what);

#define EMU_TRY_HIP(call)                                   \
    do {                                                     \
        hipError_t e__ = (call);                             \
        if (e__ != hipSuccess) return ::emu::fail_hip(e__, #call); \
    } while (0)

#define EMU_TRY(call)                                       \
    do {                                                     \
        int r__ = (call);                                    \
        if (r__ != 0) return r__;                            \
    } while (0)

// ------------------------------------------------------ device context
struct Device {
    int id = -1;
    int *status = nullptr;        // device word: OR of EMU_STATUS_* bits (a
                                  // file-scope __device__ variable of the library)
    char *scratch = nullptr;      // device address of this device's copy of the
                                  // fixed scratch array of emu_dgemm_noalloc
};

// State of one thread on one device.  Scratch belongs to a thread, so two
// threads never share it; a thread that moves to another stream has its next
// call ordered after the work of its previous call (an event), so one
// thread's calls never overlap on its scratch either.
struct ThreadCtx {
    int dev = -1;
    char *own = nullptr;          // library-owned scratch (grown on demand)
    size_t own_bytes = 0;
    char *user = nullptr;         // caller's workspace (emu_set_workspace)
    size_t user_bytes = 0;
    hipStream_t last = nullptr;   // stream of the previous call
    hipEvent_t done = nullptr;    // recorded on it at the end of that call
    bool pending = false;
    hipStream_t side = nullptr;   // LU look-ahead: trailing updates (default priority)
    hipEvent_t ev_go = nullptr;   // main stream -> side stream
    hipEvent_t ev_done = nullptr; // side stream -> main stream
    void *blas = nullptr;         // rocBLAS handle of the native comparison updates
};

// Current device's state (initialised on first use) and the thread's stream.
int current(Device **dev, hipStream_t *stream);
// The calling thread's context on the device.
ThreadCtx *thread_ctx(const Device *dev);
// Scratch of at least `bytes` for a call on `st`: the caller's workspace when
// one is registered (EMU_ERR_WORKSPACE if it is too small), else the thread's
// own buffer (grown after a device synchronization).  Orders `st` after the
// thread's previous call when that ran on another stream.
int acquire(const Device *dev, hipStream_t st, size_t bytes, char **ws);
// End of a call's work on `st` (records the ordering event).
void release(const Device *dev, hipStream_t st);
// The thread's side stream and its two events (created on first use).
int side_stream(ThreadCtx *c);

// One entry point's use of the device: begin() finds the device and stream
// and takes `bytes` of scratch; the destructor marks the end of the call.
struct Call {
    Device *dev = nullptr;
    hipStream_t st = nullptr;
    char *ws = nullptr;
    bool held = false;
    int begin(size_t bytes) {
        int r = current(&dev, &st);
        if (r) return r;
        r = acquire(dev, st, bytes, &ws);
        if (r) return r;
        held = true;
        return 0;
    }
    ~Call() {
        if (held) release(dev, st);
    }
};

// Slice counts of the grouped launches (batched LU, adaptive LU and its
// learned map, whose classes are s = 3..9): 1..9.  The plain emulated GEMM
// and LU take 1..EMU_MAX_SLICES.
constexpr int GROUPED_MAX_SLICES = 9;

// ----------------------------------------------------------- geometry
// Exponent codes kept per line during a scan: INT_MIN for a line of zeros
// (finalised to exponent 0), INT_MAX for a line holding Inf/NaN, otherwise
// the frexp exponent of the line's largest magnitude.
constexpr int CODE_ZERO = INT_MIN;
constexpr int CODE_NONFINITE = INT_MAX;

// Digit planes are stored in MFMA fragment order.  A "line" is a row of A or
// a column of B; lines are padded to LINE_PAD, K to K_BLOCK.  Block (lb, kb)
// of plane d covers lines lb*32..+32 and k = kb*32..+32 and is 1024 bytes:
// byte (kh*32 + line%32)*16 + k%16 with kh = (k%32)/16.  One wave loads a
// block with one 16-byte load per lane; lane l receives line l%32 and the
// k-half l/32, the operand layout of v_mfma_i32_32x32x32_i8 (the same k
// assignment on the A and the B side is all the dot product needs).
constexpr int LINE_PAD = 128;
constexpr int K_BLOCK = 32;
constexpr int FRAG_BYTES = 1024;

struct Planes {
    int lines = 0, k = 0;        // logical sizes
    int LB = 0, KB = 0;          // 32-line blocks (padded), 32-k blocks
    size_t plane_bytes = 0;      // bytes of one digit plane
};

inline Planes plane_geom(int lines, int k) {
    Planes p;
    p.lines = lines;
    p.k = k;
    int lp = (lines + LINE_PAD - 1) / LINE_PAD * LINE_PAD;
    p.LB = lp / 32;
    p.KB = (k + K_BLOCK - 1) / K_BLOCK;
    p.plane_bytes = (size_t)p.LB * p.KB * FRAG_BYTES;
    return p;
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Last q in [0, n) with prefix[q] <= x, for a non-decreasing prefix with
// prefix[0] <= x (so entries of empty items are skipped): a 64-ary search by
// the calling wave (all lanes active, x and n wave-uniform).  Each level reads
// 64 entries at once and keeps the interval after the last one <= x, so n
// up to 4096 takes two dependent reads instead of twelve.
__device__ __forceinline__ int wave_search(const int *prefix, int n, int x) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int step = (hi - lo + 64) / 64;          // 64 lanes cover [lo, hi]
        const int q = lo + lane * step;
        const bool le = q <= hi && prefix[q] <= x;
        const unsigned long long m = __ballot(le);      // lane 0 always set
        const int last = 63 - __builtin_clzll(m);
        lo = lo + last * step;
        const int h = lo + step - 1;
        hi = h < hi ? h : hi;
    }
    return lo;
}

// ---------------------------------------------------------- launchers
// Exponent scan + slicing of one operand into packed planes.
//   by_rows = 1: X is lines x k (rows of A are lines), element (l, kk) at
//               X[l + kk*ldx];
//   by_rows = 0: X is k x lines (columns of B are lines), element (kk, l) at
//               X[kk + l*ldx].
// code receives the per-line exponent codes (length >= lines); planes
// receives s planes of geometry g; status gets EMU_STATUS_NONFINITE.
int launch_slice(const double *X, long long ldx, int by_rows, const Planes &g,
                 int s, int *code, int8_t *planes, int *status,
                 hipStream_t stream);

// One operand of a grouped slicing pass with K <= 32 (one fragment block
// along K): exponent scan and digits in a single pass.
struct SliceJob {
    const double *X;
    long long ldx;
    int lines, k, by_rows, LB;
    int *code;
    int8_t *planes;
    size_t plane_bytes;
};
// jobs and wave_prefix (nj + 1 running sums of LB) are device arrays.
int launch_slice_small_grouped(const SliceJob *jobs, const int *wave_prefix, int nj,
                               int total_waves, int s, int *status, hipStream_t stream);

// Unpack planes to plain column-major int8 (debug entry).
int launch_unpack(const int8_t *planes, const Planes &g, int s, int by_rows,
                  int8_t *out, hipStream_t stream);
int launch_codes_to_exps(const int *code, int lines, int *exps, int *nonfinite,
                         hipStream_t stream);

// One slice-product GEMM problem (device pointers; planes in fragment order).
struct GemmArgs {
    const int8_t *Ap;
    const int8_t *Bp;
    size_t a_plane, b_plane;
    const int *codeA;
    const int *codeB;
    int M, N, KB;         // logical sizes, K in 32-blocks
    int chunk_kb;         // K-blocks per chunk (chunked partial mode)
    int tiles_m, tiles_n;
    double alpha, beta;
    double *C;
    long long ldc;
    int32_t *part;        // chunk partials [chunk][g-2][n][m]
    int map;              // tile order of the plain launch (tile_of)
    int lower;            // store only entries with row >= column (symmetric update)
};

// Tile order of the plain slice-GEMM launches on the calling thread
// (emu_set_param "gemm_map"; 1 by default); bits are unaffected.
void set_gemm_map(int map);
// Grouped-GEMM tile of the batched form for calls with an explicit block
// size (emu_set_param "batched_tile": 0 = 64 x 128, 1 = 64 x 64, s >= 6).
void set_batched_tile(int tile);
// Block size emu_autotune_getrf recorded for an LU of this shape and slice
// count on this device and runtime (0: none), and recording one (kept in the
// same table, and file, as the batched form's choices).
int tuned_getrf_nb(int m, int n, int s);
void record_getrf_nb(int m, int n, int s, int nb);
int gemm_map();

// Slice-product GEMM with fused recombination, or the raw diagonal sums
// D_g (Dout != null, int64 [t-1][n][m]).  ws_part: INT32 scratch for K-chunk
// partial sums of gemm_chunk_bytes(..., raw_sums = Dout != null) bytes; may
// be null when that is 0.
size_t gemm_chunk_bytes(int m, int n, int k, int s, int t, bool raw_sums);
// lower = true (the Cholesky update A22 - L21 L21^T, Bp = Ap): entries above
// the diagonal are neither computed nor stored; K must not need chunks.
int launch_slicegemm(const int8_t *Ap, const Planes &ga, const int8_t *Bp,
                     const Planes &gb, const int *codeA, const int *codeB,
                     int m, int n, int k, int s, int t, double alpha,
                     double beta, double *C, long long ldc, int64_t *Dout,
                     int32_t *ws_part, hipStream_t stream, bool lower = false);
bool gemm_supported(int s, int t);
// Unequal splits: A with s slices (2..9), B with sb (1..s-1) slices, t = s + 1,
// K within one exact pass (EMU_ERR_UNSUPPORTED otherwise).
int launch_slicegemm_ab(const int8_t *Ap, const Planes &ga, const int8_t *Bp, const Planes &gb,
                        const int *codeA, const int *codeB, int m, int n, int k, int s, int sb,
                        double alpha, double beta, double *C, long long ldc, hipStream_t stream);
// Many problems of one (s, t = s + 1) in one persistent launch: probs[q]
// (device) holds problem q with tiles_m/tiles_n set by gemm_tile_counts;
// tile_prefix (device, nprob + 1) is the running sum of tiles_m * tiles_n.
// K of every problem must not need chunking (K <= 32 * 462 for s = 9).
// shape 1 (s >= 6, one-K-step grouped launches): 64 x 64 tiles instead of
// 64 x 128.
void gemm_tile_counts(int s, int m, int n, int *tiles_m, int *tiles_n, int shape = 0);
// Output tile of the slice GEMM at t = s + 1: tile_rows(s) x GEMM_TILE_COLS.
__host__ __device__ constexpr int gemm_tile_rows(int s) { return s <= 5 ? 128 : 64; }
constexpr int GEMM_TILE_COLS = 128;
int gemm_grouped_blocks_per_cu(int s, int shape = 0);
// one_kstep: every problem has K <= 32 (one K step); selects the
// pipelined kernel for s >= 6.
int launch_slicegemm_grouped(const GemmArgs *probs, const int *tile_prefix, int nprob,
                             int total_tiles, int grid, int s, hipStream_t stream,
                             bool one_kstep = false, int shape = 0);
// The same with the problem count and the tile total read on the device
// (counts[0], counts[1]), so the list can be built by a kernel; no launch
// work is skipped on the host when the list is empty.
int launch_slicegemm_grouped_dev(const GemmArgs *probs, const int *tile_prefix,
                                 const int *counts, int grid, int s, hipStream_t stream);

// FP64 LU pieces.
int launch_fill_int(int *p, int v, int count, hipStream_t stream);
// Panel factorization (recursive, see panel.hip) of the rows x jb block at
// A (global row/column row0); ws: panel_scratch_bytes(rows) bytes; status:
// the device status word (EMU_STATUS_PANEL_WAIT on an aborted tall leaf);
// pivot = false: no interchanges (ipiv receives the identity); one_xcd =
// false: leaves of several workgroups stay spread over the XCDs (for callers
// whose concurrent kernels keep compute units of every XCD occupied).
size_t panel_scratch_bytes(int rows);
// Launch multi-workgroup panel leaves cooperatively (calling thread's switch).
void set_leaf_cooperative(int on);
// Gather leaves of at most 16 workgroups on one XCD (calling thread's switch, default on).
void set_leaf_one_xcd(int on);
int launch_panel(double *A, long long lda, int rows, int jb, int *ipiv,
                 int row0, int *info, char *ws, int *status, hipStream_t stream,
                 bool pivot = true, bool one_xcd = true);
// Lower Cholesky of the rows x jb panel at A (its top jb x jb block on the
// diagonal; global column col0), FP64; *info receives the first column
// (1-based, global) whose pivot is not positive, if it is still 0.
int launch_chol_panel(double *A, long long lda, int rows, int jb, int col0, int *info,
                      hipStream_t stream);
// C (m x n) <- C - A B in native FP64 (rocBLAS dgemm) on `stream`: the
// trailing update of the LU when emu_set_param("lu_update", 1) asks for the
// native comparison.
int native_update(int m, int n, int k, const double *A, long long lda, const double *B,
                  long long ldb, double *C, long long ldc, hipStream_t stream);
// Destroy the thread context's rocBLAS handle (emu_finalize).
void native_release(ThreadCtx *c);
// C (m x m, lower triangle) <- C - A A^T in native FP64 (rocBLAS dsyrk).
int native_syrk_update(int m, int k, const double *A, long long lda, double *C, long long ldc,
                       hipStream_t stream);
// Interchanges ipiv[k1..k2) on columns [0, ncols_left) and [col_right,
// col_right + ncols_right); plan: laswp_plan_bytes(nrows) bytes of scratch.
size_t laswp_plan_bytes(int nrows);
// perm (optional, nrows ints): the row permutation so far, updated by these
// interchanges (the plan is then made even when no other column moves).
int launch_laswp(double *A, long long lda, int nrows, int ncols_left, int col_right,
                 int ncols_right, const int *ipiv, int k1, int k2, int row0, int *plan,
                 hipStream_t stream, int *perm = nullptr);
// perm <- identity (n ints).
int launch_perm_init(int *perm, int n, hipStream_t stream);
// The apply step alone, with the plan a launch_laswp call of the same
// (nrows, k1, k2) left in `plan` (ordered after it on the device).
int launch_laswp_apply(double *A, long long lda, int nrows, int ncols_left, int col_right,
                       int ncols_right, int k1, int k2, const int *plan, hipStream_t stream);
int launch_trsm_llnu(const double *L, long long ldl, int jb, double *B,
                     long long ldb, int ncols, hipStream_t stream);
// perm_ws holds the composed row permutation after a call; perm_ready
// reuses it (same factors) instead of composing it again; perm_ext gives
// the permutation itself (the factorization tracked it).
// status: the device status word; with it (and at most four right-hand
// sides) each sweep runs as one persistent launch, which with inv (the
// inverted diagonal blocks of launch_tri_inv) multiplies each block by its
// inverse instead of resolving it by substitution.
int launch_getrs(int n, int nrhs, const double *LU, long long lda,
                 const int *ipiv, double *B, long long ldb, int *perm_ws,
                 hipStream_t stream, bool perm_ready = false, int *status = nullptr,
                 const int *perm_ext = nullptr, const double *inv = nullptr);
// Inverses of the 64 x 64 diagonal blocks of L (unit lower) and U.
size_t tri_inv_bytes(int n);
int launch_tri_inv(const double *LU, long long lda, int n, double *inv, hipStream_t stream);
// Scratch bytes of launch_getrs.
size_t getrs_ws_bytes(int n, int nrhs);

// Precision form (refine.hip).
size_t refine_partial_bytes(int n, int nrhs);
int launch_norm_inf(const double *A, long long lda, int n, double *partial, double *out,
                    hipStream_t stream);
int launch_residual(const double *A, long long lda, int n, const double *X, long long ldx,
                    const double *B, long long ldb, int nrhs, double *R, long long ldr,
                    double *partial, double *stats, hipStream_t stream);
int launch_add_cols(double *X, long long ldx, const double *D, long long ldd, int n,
                    int nrhs, hipStream_t stream);
int launch_copy_mat(const double *src, long long lds_, double *dst, long long ldd, int n,
                    int cols, hipStream_t stream);

// Learned slice count (learned.hip).
int learned_nparam();
size_t features_ws_bytes(int m, int n);
// line statistics of `lines` rows (by_rows) or columns of an operand with
// k elements per line; tile features of an m x n update from the row and
// column statistics (tile (I, J) at I + J ceil(m / 256))
size_t feat_stat_bytes(int lines);
int launch_feat_lines(const double *X, long long ldx, int lines, int k, int by_rows,
                      void *stats, hipStream_t st);
int launch_feat_tiles(const void *row_stats, const void *col_stats, int m, int n, float *feat,
                      hipStream_t st);
int launch_features(const double *L21, long long ldl, const double *U12, long long ldu, int m,
                    int n, int k, float *feat, void *stat_ws, hipStream_t st);
size_t mlp_train_ws_bytes(int B);
int launch_mlp_train_step(float *params, const float *X, const int *label, int B, float *m,
                          float *v, int step, float lr, void *ws, float *loss_out,
                          hipStream_t st);
int launch_mlp_grad_only(const float *params, const float *X, const int *label, int B,
                         float *grad_out, void *ws, hipStream_t st);
int launch_mlp_infer(const float *params, const float *X, int B, float *prob, int *s_out,
                     float conf, hipStream_t st);
int launch_tile_err(const double *Xs, const double *Xr, long long ld, int m, int n,
                    double *err2, double *ref2, hipStream_t st);
int launch_tile_label(const double *err2, const double *ref2, int ntiles, int s, double tau,
                      int *label, hipStream_t st);
// Adaptive LU: the 256 x 256 tiles of one Schur update C -= L21 U12 and the
// digit planes of L21 and U12 (sliced once at the largest count).
struct AdaptiveTiles {
    const int8_t *pa, *pb;
    size_t a_plane, b_plane;
    int KB;
    const int *codeA, *codeB;
    double *C;
    long long ldc;
    int M, N, tm;        // update size; tile rows tm = ceil(M / 256)
};
// For every count s = 1..9 the grouped-GEMM problem list of the tiles in
// tile columns [jlo, jhi) whose slice count min(smap[q], s_cap) is s, in
// tile order: probs[(s-1) nt + i], prefix[(s-1) (nt+1) + i],
// counts[2 (s-1)] = problems, counts[2 (s-1) + 1] = GEMM tiles.
int launch_adaptive_lists(const int *smap, int nt, int s_cap, const AdaptiveTiles &t, int jlo,
                          int jhi, GemmArgs *probs, int *prefix, int *counts, hipStream_t st);

}  // namespace emu
