/*
 * emu.h - FP64 matrix multiply emulated with INT8 slices on AMD MI355X
 * (gfx950), and the partially pivoted LU solver whose Schur-complement update
 * uses it.
 *
 * Method (arXiv 2509.23565, section "Emulation of FP64 and INT8 Splitting",
 * eqns (1)-(2)): each operand is split into s slices, the product is the sum
 * of the slice products A_i B_j, and products with i + j > t are dropped.
 * Readings this library fixes where the paper is silent:
 *   - a slice is an INT8 digit: 7 magnitude bits and the element's sign,
 *     q in [-127, 127];
 *   - A is scaled per row, B per column, by 2^-e where e is the frexp exponent
 *     of the line's largest magnitude (0 for an all-zero line);
 *   - digits are truncated toward zero: x 2^-e = sum_i q_i 128^-i + r,
 *     |r| < 128^-s;
 *   - t = s + 1 (s(s+1)/2 slice products) unless stated otherwise;
 *   - slice products are exact: D_g = sum_{i+j=g} A_i B_j accumulated in
 *     INT32 inside K-chunks short enough that no INT32 sum can overflow,
 *     and in INT64 across chunks;
 *   - recombination in one fixed order: S = 0; for g = t down to 2:
 *     S = fl(S + D_g 2^-7g); X = S 2^(e_p + f_q); C = fma(alpha, X, beta C)
 *     (beta = 0: fma(alpha, X, 0), C not read).  Results therefore do not
 *     depend on tile shapes or launch configuration.
 *   - a row of A or a column of B holding Inf or NaN makes the matching row
 *     or column of C NaN and sets EMU_STATUS_NONFINITE in the status word.
 *
 * Conventions for every entry point:
 *   - matrices are column-major FP64 in DEVICE memory with leading
 *     dimensions; pivots and info are DEVICE int32; the caller owns every
 *     buffer passed in, the library never frees or retains them;
 *   - dimensions are int; all index arithmetic inside is 64-bit;
 *   - calls are asynchronous on the calling thread's current stream (see
 *     emu_set_stream) unless stated otherwise;
 *   - scratch memory (digit planes, exponents, partial sums) belongs to the
 *     calling thread: either a workspace the caller registered with
 *     emu_set_workspace (then no entry point allocates or synchronizes for
 *     scratch; a call that needs more returns EMU_ERR_WORKSPACE), or a buffer
 *     the library allocates on first use, grows when a larger problem
 *     arrives (after synchronizing the device) and releases in emu_finalize.
 *     Threads never share scratch, so threads may call the library
 *     concurrently, each on its own stream.  When one thread moves to another
 *     stream, its next call waits (an event) for the work of its previous
 *     call, so one thread's calls never overlap on its scratch.  Two threads
 *     that register the same workspace must order their calls themselves;
 *     emu_finalize may not run while another thread is inside a call.
 *   - return value 0 on success; -i if argument i is invalid (LAPACK
 *     xerbla style, counting from 1); a positive EMU_ERR_* code otherwise.
 *     emu_last_error() describes the last failure of the calling thread.
 */
#ifndef EMU_H
#define EMU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMU_SUCCESS            0
#define EMU_ERR_HIP            1001  /* a HIP runtime call failed */
#define EMU_ERR_WORKSPACE      1002  /* scratch allocation failed, or the
                                        registered workspace is too small */
#define EMU_ERR_UNSUPPORTED    1003  /* valid request the library does not support */
#define EMU_ERR_NOT_CONVERGED  1004  /* refinement missed its tolerance at the
                                        largest slice count */
#define EMU_ERR_PANEL_WAIT     1005  /* a factorization the call waited for was
                                        aborted (see EMU_INFO_ABORTED) */

#define EMU_STATUS_NONFINITE   1     /* an emulated GEMM met Inf/NaN input */
#define EMU_STATUS_PANEL_WAIT  2     /* a multi-workgroup panel leaf (more than
                                        2048 rows) gave up a grid-wide wait that
                                        exceeded its bound; those LU factors are
                                        invalid */

#define EMU_STATUS_SOLVE_WAIT  4     /* a triangular solve (emu_dgetrs and the
                                        solves inside emu_dgesv_ir, emu_refine)
                                        gave up a wait between its blocks that
                                        exceeded its bound; that solution is
                                        invalid */

/* Value an LU writes to its device *info when a multi-workgroup panel leaf
 * gave up its bounded grid-wide wait (the factors are then invalid; the
 * status word also carries EMU_STATUS_PANEL_WAIT).  Entry points that wait
 * for their factorization return EMU_ERR_PANEL_WAIT instead. */
#define EMU_INFO_ABORTED       (-1000)

#define EMU_MAX_NB             2048  /* largest block size of emu_dgetrf and
                                        emu_dgesv_ir */
#define EMU_MAX_SLICES         16    /* slice counts of the plain GEMM and LU:
                                        1..16 (grouped forms: 1..9) */

/* Library version as major*10000 + minor*100 + patch. */
int emu_version(void);

/* Initialise the HIP device state for the current device.  Optional: every
 * entry point initialises on first use. */
int emu_init(void);

/* Release the scratch memory, streams and events the library holds for every
 * thread on every device it touched (synchronizing each device first) and
 * forget registered workspaces. */
int emu_finalize(void);

/* Set the HIP stream (hipStream_t passed as void*) used by later calls from
 * the calling thread; NULL selects the default (null) stream. */
int emu_set_stream(void *hip_stream);

/*
 * emu_set_workspace: register `bytes` of DEVICE memory at dptr (owned by the
 * caller, on the current device) as the calling thread's scratch for later
 * calls on that device; dptr = NULL with bytes = 0 returns to the library's
 * own scratch.  While a workspace is registered no entry point allocates or
 * synchronizes to obtain scratch (the batched calls, the autotuner and
 * emu_dgesv_ir still synchronize for their own reasons, and the autotuner
 * allocates copies); a call that needs more than `bytes` fails with
 * EMU_ERR_WORKSPACE and emu_last_error names the size it needs.  The
 * library reads and writes the workspace only during calls, in stream order.
 * Argument numbers: dptr=1 bytes=2.
 */
int emu_set_workspace(void *dptr, size_t bytes);

/* Scratch bytes emu_dgemm needs for that shape (0 for invalid arguments). */
size_t emu_workspace_bytes(int m, int n, int k, int nslices);
/* Scratch bytes emu_dgetrf needs (nb <= 0: the block size emu_dgetrf would
 * select; 0 for invalid arguments). */
size_t emu_getrf_workspace_bytes(int m, int n, int nb, int nslices);
/* Scratch bytes emu_dgetrs needs (0 for invalid arguments). */
size_t emu_getrs_workspace_bytes(int n, int nrhs);

/* Text of the last error raised on the calling thread ("" if none). */
const char *emu_last_error(void);

/* Synchronize the current stream and return, in *status, the OR of the
 * EMU_STATUS_* bits raised since the previous call (then cleared). */
int emu_status(int *status);

/* Kernel-time profiling on the calling thread's stream.  emu_profile_start
 * clears earlier records and makes every later call bracket its kernel
 * groups with HIP events on the stream they run on; emu_profile_stop ends
 * recording; emu_profile_read waits for the recorded events and returns the
 * summed milliseconds and the number of launches of one group:
 * EMU_PROF_SLICE (exponent scans and digit slicing of both operands) or
 * EMU_PROF_GEMM (the slice-product GEMM with its recombination epilogue).
 * Argument numbers: kind=1 total_ms=2 count=3. */
#define EMU_PROF_SLICE 0
#define EMU_PROF_GEMM  1
int emu_profile_start(void);
int emu_profile_stop(void);
int emu_profile_read(int kind, double *total_ms, int *count);

/*
 * emu_dgemm: C <- alpha * A B + beta * C, A m x k (lda >= max(1,m)),
 * B k x n (ldb >= max(1,k)), C m x n (ldc >= max(1,m)), no transposes,
 * emulated with nslices INT8 slices per operand and threshold t = s + 1
 * (paper: emulation section, eqns (1)-(2) and the truncation threshold).
 * nslices must lie in 1..EMU_MAX_SLICES.
 * Quick returns as in BLAS: m = 0 or n = 0 does nothing; k = 0 or
 * alpha = 0 gives C <- beta C (C not read when beta = 0).
 * Argument numbers for errors: m=1 n=2 k=3 alpha=4 A=5 lda=6 B=7 ldb=8
 * beta=9 C=10 ldc=11 nslices=12.
 */
int emu_dgemm(int m, int n, int k, double alpha, const double *A, int lda,
              const double *B, int ldb, double beta, double *C, int ldc,
              int nslices);

/*
 * emu_dgemm_noalloc: emu_dgemm for callers that cannot allocate device
 * memory or synchronize (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, argument numbers and
 * quick returns as emu_dgemm, and bit-identical results.  It allocates
 * nothing, creates no HIP objects and never synchronizes: its scratch (digit
 * planes, exponent codes, chunk partial sums) is a fixed array of
 * EMU_NOALLOC_SCRATCH_BYTES in the library's own device memory, one per
 * device, held until the process ends.  A shape whose emu_workspace_bytes
 * exceeds that size returns EMU_ERR_WORKSPACE (nothing is launched).  Every
 * call on one device uses the same array, so calls that overlap on one
 * device (two streams, two threads) race and give wrong results: the caller
 * orders them.  The array keeps the last call's contents; no call relies on
 * it starting at zero.  It ignores emu_set_workspace and takes no part in
 * emu_profile_*.
 */
#define EMU_NOALLOC_SCRATCH_BYTES (64u << 20)   /* 64 MiB */
int emu_dgemm_noalloc(int m, int n, int k, double alpha, const double *A, int lda,
                      const double *B, int ldb, double beta, double *C, int ldc,
                      int nslices);

/*
 * emu_dgemm_ab: emu_dgemm with unequal splits (the paper's related-work
 * section names splits of unequal size as a way to fewer products): A is
 * split into nslices_a slices, B into nslices_b <= nslices_a, t =
 * nslices_a + 1, so the pairs are i <= nslices_a, j <= nslices_b, i + j <=
 * t: sum over i of min(nslices_b, t - i) products instead of s(s+1)/2.  When
 * every column of B is represented exactly by nslices_b digits (integers or
 * fixed-point data below 2^(7 nslices_b) times the column's scale), the
 * result is bit-identical to emu_dgemm with nslices_a slices.  Supported:
 * nslices_b = nslices_a (then exactly emu_dgemm), or 1 <= nslices_b <
 * nslices_a <= 9 with k at most the one-pass exact length for nslices_b
 * pairs per diagonal (2^31 / (nslices_b 127^2), rounded down to 32: 14784
 * for 9) — longer k returns EMU_ERR_UNSUPPORTED.  Scratch: at most
 * emu_workspace_bytes(m, n, k, nslices_a).  Argument numbers as emu_dgemm,
 * nslices_a=12, nslices_b=13.
 */
int emu_dgemm_ab(int m, int n, int k, double alpha, const double *A, int lda,
                 const double *B, int ldb, double beta, double *C, int ldc, int nslices_a,
                 int nslices_b);

/*
 * emu_dgemm_t: emu_dgemm with an explicit truncation threshold t (the
 * paper's t: products A_i B_j with i + j > t are dropped).  Supported:
 * t = s + 1 for s in 1..16 and t = 2s (all s^2 products) for s in 1..5.
 * Argument 13 is t.
 */
int emu_dgemm_t(int m, int n, int k, double alpha, const double *A, int lda,
                const double *B, int ldb, double beta, double *C, int ldc,
                int nslices, int t);

/*
 * emu_dgetrf: PA = LU of the m x n matrix A (lda >= max(1,m)) in place,
 * right-looking blocked with block size nb (at most EMU_MAX_NB; nb <= 0
 * selects the block size emu_autotune_getrf recorded for (m, n, nslices) on
 * this device and runtime, else 64; interchanges are applied to the other
 * columns in chunks of 1024, in order), partial
 * pivoting (paper: solvers section, eqns (5)-(8)).  Per block column:
 * FP64 panel factorization (first row of largest magnitude is the pivot;
 * the column below is scaled by the reciprocal of the pivot, or divided
 * when |pivot| < DBL_MIN); the panel's interchanges applied to the other
 * columns; FP64 unit-lower triangular solve for U12; then the Schur update
 * A22 <- A22 - L21 U12 as an emulated GEMM with nslices slices
 * (nslices in 1..EMU_MAX_SLICES, threshold t = s + 1).
 * ipiv (device, min(m,n) int32) receives 1-based row interchanges in
 * LAPACK order.  *info (device int32) receives 0, or i > 0 when U(i,i) is
 * exactly zero (the first such i; the factorization still completes), or
 * EMU_INFO_ABORTED when a panel taller than 2048 rows gave up its bounded
 * grid-wide wait (the factors are then invalid; the call returned 0 before
 * this happened, since it does not wait for the GPU).
 * Argument numbers: m=1 n=2 A=3 lda=4 ipiv=5 info=6 nb=7 nslices=8.
 */
int emu_dgetrf(int m, int n, double *A, int lda, int *ipiv, int *info,
               int nb, int nslices);

/*
 * emu_autotune_getrf: time emu_dgetrf of a private copy of A (m x n,
 * lda >= m, device; A itself is not modified) once per candidate block size
 * (count > 0: nbs[0..count) on the host, each in 1..EMU_MAX_NB; count = 0:
 * 256, 512, 768 and 1024 up to min(m, n), or min(m, n, 64) when none is),
 * after one untimed run with the candidate of the largest scratch; record
 * the fastest for (device architecture, HIP runtime version, m, n,
 * nslices), which emu_dgetrf, emu_dgesv_ir and emu_getrf_workspace_bytes
 * then use for nb <= 0, and return it with its time (host outputs).  The
 * paper leaves the block size open; its figures compare block sizes.  With
 * EMU_AUTOTUNE_CACHE set the record joins the batched form's table in that
 * file.  Allocates and frees device memory for the copy; synchronizes.
 * Argument numbers: m=1 n=2 A=3 lda=4 nslices=5 nbs=6 count=7 best_nb=8
 * best_ms=9.
 */
int emu_autotune_getrf(int m, int n, const double *A, int lda, int nslices, const int *nbs,
                       int count, int *best_nb, double *best_ms);

/*
 * emu_dpotrf: Cholesky A = L L^T of the symmetric positive definite n x n
 * matrix A (lda >= max(1,n)), lower triangle, in place; the strictly upper
 * part is neither read nor written (the symmetric case the paper names
 * beside LU, solvers section and conclusions).  Right-looking blocked with
 * block size nb (nb <= 0 selects 64, at most EMU_MAX_NB).  Per block column:
 * FP64 panel (l_jj = sqrt(a_jj), the column below multiplied by 1 / l_jj,
 * each a_ij, i >= j, losing l_ik l_jk for k = 0..j-1 in order), then the
 * update A22 <- A22 - L21 L21^T of the lower triangle as an emulated GEMM
 * with nslices slices (1..EMU_MAX_SLICES, t = s + 1) whose two operands are
 * the same digit planes of L21 (sliced once; the product is exactly
 * symmetric).  With emu_set_param("lu_update", 1) the update is rocBLAS
 * dsyrk instead.  *info (device int32) receives 0, or the first column j
 * (1-based) whose pivot a_jj was not positive or was NaN; then columns
 * 1..j-1 of L are complete and the rest of the lower triangle is
 * unspecified (the call does not wait to find out).
 * Argument numbers: n=1 A=2 lda=3 info=4 nb=5 nslices=6.
 */
int emu_dpotrf(int n, double *A, int lda, int *info, int nb, int nslices);
/* Scratch bytes emu_dpotrf needs (0 for invalid arguments). */
size_t emu_potrf_workspace_bytes(int n, int nb, int nslices);

/*
 * emu_dgetrs: solve A X = B (no transpose) with the factors of emu_dgetrf:
 * row interchanges, forward substitution with unit L, back substitution
 * with U, all FP64 (paper: eqn (5)).  LU n x n (lda >= max(1,n)), ipiv
 * device int32[n], B n x nrhs (ldb >= max(1,n)) overwritten with X.  Each
 * element receives its updates in the order of column-by-column
 * substitution.  With at most four right-hand sides each sweep is one
 * launch whose 64-row blocks wait for the earlier blocks' solutions (the
 * wait is bounded: see EMU_STATUS_SOLVE_WAIT); with more, one launch per
 * 64-row block and sweep.
 * Argument numbers: n=1 nrhs=2 LU=3 lda=4 ipiv=5 B=6 ldb=7.
 */
int emu_dgetrs(int n, int nrhs, const double *LU, int lda, const int *ipiv,
               double *B, int ldb);

/*
 * emu_set_param: library knobs (thread-local).  Keys:
 *   "ir_force_fail" (value >= 0): the next `value` convergence checks of
 *   emu_dgesv_ir on this thread count as failed, which exercises the
 *   fallback to more slices (a test hook; the checks still run).
 *   "lu_pivot" (0 or 1, default 1): 0 makes emu_dgetrf (and the LU inside
 *   emu_dgesv_ir) factor without interchanges, A = LU: the pivot of column
 *   c is the entry in row c, ipiv receives the identity, and *info still
 *   reports the first exactly zero pivot (the performance section of the
 *   paper times this simplified LU).
 *   "lu_update" (0 or 1, default 0): 1 makes the same factorizations (and
 *   emu_dpotrf) do their Schur-complement update in native FP64 (rocBLAS
 *   dgemm, dsyrk for the Cholesky) instead of the emulated GEMM, for
 *   comparisons at an equal block size; panel, interchanges and triangular
 *   solves are unchanged.
 *   "lu_lookahead" (0 or 1, default 1): emu_dgetrf (and the LU inside
 *   emu_dgesv_ir, and emu_dgetrf_adaptive) updates the columns right of
 *   the next panel on a library-owned side stream of the device while that
 *   panel is factored;
 *   the caller's stream waits for it, so the call stays ordered on the
 *   caller's stream.  The factors are identical either way.
 *   "batched_tile" (0 or 1, default 0): grouped-GEMM output tile of the
 *   batched calls given an explicit block size (0: 64 x 128, 1: 64 x 64;
 *   six slices and more); nb = 0 uses the autotuned tile.  Bits unchanged.
 *   "gemm_map" (0 or 1, default 1): order in which the workgroups of an
 *   emulated GEMM visit the output tiles: 1 lets all eight XCDs work on one
 *   block of tiles at a time (used when both tile counts are multiples of
 *   16), 0 gives each XCD its own contiguous range.  Results are identical.
 *   "leaf_cooperative" (0 or 1, default 0): panel leaves taller than 2048
 *   rows (several workgroups that wait for each other) are launched with
 *   hipLaunchCooperativeKernel instead of a plain launch.  The factors are
 *   identical either way; the plain launch avoids the cooperative launch's
 *   fixed cost.
 *   "leaf_one_xcd" (0 or 1, default 1): plain launches of
 *   such leaves with at most 16 workgroups (at most 16384 rows) place all
 *   of them on one XCD, where their exchange of pivot candidates is about
 *   twice as fast; they then need 16 compute units of that XCD at once.
 *   Callers that keep part of every XCD busy for long stretches beside the
 *   factorization (persistent kernels on other streams) should set 0, or
 *   the leaves' bounded waits may run out (EMU_STATUS_PANEL_WAIT).
 *   emu_dgetrf_adaptive spreads its leaves regardless.  Factors identical.
 * Returns -1 for an unknown key, -2 for an invalid value.
 */
int emu_set_param(const char *key, long long value);

/*
 * emu_dgesv_ir: solve A X = B to a backward-error tolerance with the
 * precision form: emulated LU with a reduced slice count, FP64 solves and
 * FP64 iterative refinement, falling back to more slices when refinement
 * stalls (this form is not in the paper; the stopping quantity is eqn (9)'s
 * scaled residual without its n eps factor).
 *   1. LU of a copy of A (A itself is not modified) with `nslices` slices and
 *      block size nb (nb <= 0: as emu_dgetrf selects it for (n, n, nslices),
 *      kept for the fallback factorizations); X = getrs(B).
 *   2. Repeat: R = B - A X in FP64; eta = max over columns of
 *      ||R||_inf / (||A||_inf ||X||_inf + ||B||_inf).  Stop when eta <= tol.
 *      Otherwise, if eta did not fall below half its previous value, or
 *      `maxiter` corrections were applied, or eta is NaN: fall back (step 3);
 *      else X += getrs(R).
 *   The solves (up to four right-hand sides) multiply each 64 x 64 diagonal
 *   block of L and U by its inverse, computed once per factorization, so X
 *   differs from emu_dgetrs's substitution in rounding; the refinement
 *   corrects it.
 *   3. Fallback: refactor with s = min(s + 2, s_cap) and restart at step 1's
 *      solve, where s_cap = 9 for a start nslices <= 9 and EMU_MAX_SLICES
 *      above (beyond nine slices the update is already below the FP64 panel's
 *      own rounding at LU block sizes); if s was already s_cap return
 *      EMU_ERR_NOT_CONVERGED.
 * A n x n (lda >= max(1,n)), B and X n x nrhs (ldb, ldx >= max(1,n)), all
 * device; outputs on the HOST: *iters = corrections applied (all
 * factorizations), *berr = last eta, *s_final = slice count of the last
 * factorization, *info = its LAPACK info (> 0: exactly singular U, X not
 * refined).  Synchronizes the stream once per refinement step.  Returns
 * EMU_ERR_PANEL_WAIT if a factorization was aborted (EMU_INFO_ABORTED).
 * Argument numbers: n=1 nrhs=2 A=3 lda=4 B=5 ldb=6 X=7 ldx=8 nb=9
 * nslices=10 tol=11 maxiter=12 iters=13 berr=14 s_final=15 info=16.
 */
int emu_dgesv_ir(int n, int nrhs, const double *A, int lda, const double *B, int ldb,
                 double *X, int ldx, int nb, int nslices, double tol, int maxiter,
                 int *iters, double *berr, int *s_final, int *info);

/*
 * emu_refine: FP64 iterative refinement of an existing solution X of
 * A X = B with existing factors (LU, ipiv from any emu_dgetrf variant):
 * repeat R = B - A X, eta = max over columns of ||R||_inf /
 * (||A||_inf ||X||_inf + ||B||_inf); stop at eta <= tol; else, unless eta
 * failed to halve or `maxiter` corrections were applied (then
 * EMU_ERR_NOT_CONVERGED), X += getrs(R), with the inverted diagonal blocks
 * of emu_dgesv_ir's solves (computed once per call, before the first
 * correction).  *iters, *berr on the HOST.
 * Argument numbers: n=1 nrhs=2 A=3 lda=4 LU=5 ldlu=6 ipiv=7 B=8 ldb=9 X=10
 * ldx=11 tol=12 maxiter=13 iters=14 berr=15.
 */
int emu_refine(int n, int nrhs, const double *A, int lda, const double *LU, int ldlu,
               const int *ipiv, const double *B, int ldb, double *X, int ldx, double tol,
               int maxiter, int *iters, double *berr);

/*
 * emu_scaled_residual: the scaled residual of eqn (9),
 * ||A X - B||_inf / ((||A||_inf ||X||_inf + ||B||_inf) n eps) with
 * eps = 2^-53, evaluated in FP64 on the GPU (residual columns summed in a
 * fixed order), the largest over the nrhs columns; *sres on the HOST.  The
 * HPL acceptance test is *sres < 16.  Synchronizes the stream.
 * Argument numbers: n=1 nrhs=2 A=3 lda=4 X=5 ldx=6 B=7 ldb=8 sres=9.
 */
int emu_scaled_residual(int n, int nrhs, const double *A, int lda, const double *X, int ldx,
                        const double *B, int ldb, double *sres);

/*
 * Batched grouped form (not in the paper; every system is the paper's LU):
 * `count` independent systems i with n[i] in 1..1024 (host array), A[i]
 * (host array of DEVICE pointers, lda[i] >= n[i]), ipiv[i] (host array of
 * DEVICE int32[n[i]]), info (DEVICE int32[count]).  Per block step one
 * launch per phase covers every active system (panel, interchanges, TRSM,
 * slicing) and one persistent grouped launch runs all slice-pair GEMMs of
 * that step's updates; the sequence is captured once per batch shape into a
 * hipGraph and replayed (descriptors refreshed per call; the call
 * synchronizes the stream once to upload them).  nb in 1..32 (0: the
 * autotuned value for this batch shape, else 32); nslices in 1..9.  Each
 * system's factors and pivots equal emu_dgetrf's with the same nb.
 * Argument numbers: count=1 n=2 A=3 lda=4 ipiv=5 info=6 nb=7 nslices=8.
 */
int emu_dgetrf_batched(int count, const int *n, double *const *A, const int *lda,
                       int *const *ipiv, int *info, int nb, int nslices);

/*
 * emu_dgesv_batched: emu_dgetrf_batched followed by the solve of each
 * system with its nrhs[i] in 1..8 right-hand sides B[i] (host array of
 * DEVICE pointers, ldb[i] >= n[i]), overwritten with the solutions; same
 * solve order as emu_dgetrs.  Argument numbers: count=1 n=2 nrhs=3 A=4
 * lda=5 ipiv=6 info=7 B/ldb=8 nb=9 nslices=10.
 */
int emu_dgesv_batched(int count, const int *n, const int *nrhs, double *const *A,
                      const int *lda, int *const *ipiv, int *info, double *const *B,
                      const int *ldb, int nb, int nslices);

/*
 * emu_dgetrs_batched: solve A_i X_i = B_i for every system of a batch from
 * factors and pivots that emu_dgetrf_batched (or emu_dgetrf with the same
 * layout) left: LU[i] (host array of DEVICE pointers, lda[i] >= n[i],
 * read only), ipiv[i] (host array of DEVICE int32[n[i]], 1-based), B[i]
 * (host array of DEVICE pointers, ldb[i] >= n[i], nrhs[i] in 1..8
 * columns) overwritten with X_i; n[i] in 1..1024.  Row interchanges, then
 * forward substitution with the unit lower factor and back substitution
 * with the upper one (the solve step of the solvers section, eqn (8)), one
 * workgroup per system, in the per-element order of emu_dgetrs, so the
 * results equal emu_dgesv_batched's solve bit for bit.  No check of the
 * factors: an exactly zero U(j,j) gives Inf/NaN as in LAPACK's getrs.
 * Synchronizes the stream once to upload the descriptors, then enqueues
 * one launch.  Argument numbers: count=1 n=2 nrhs=3 LU=4 lda=5 ipiv=6 B=7
 * ldb=8.
 */
int emu_dgetrs_batched(int count, const int *n, const int *nrhs, const double *const *LU,
                       const int *lda, const int *const *ipiv, double *const *B,
                       const int *ldb);

/*
 * emu_dgesv_batched_ir: the precision form for a batch (the single-system
 * form is emu_dgesv_ir): A[i] and B[i] (host arrays of DEVICE pointers,
 * n[i] in 1..1024, nrhs[i] in 1..8) are left untouched; X[i] (ldx[i] >=
 * n[i]) receives the solutions.  All systems are factored together from
 * copies of A with nslices slices (1..9; grouped launches as in
 * emu_dgesv_batched, block size nb in 1..32, 0 selects 32) and solved;
 * then every system not yet at tol takes a refinement step: FP64 residual
 * r = B - A X and its backward error eta = max over columns of
 * ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf); eta <= tol ends the
 * system; eta not below half the previous one, more than maxiter steps or
 * NaN sends it back to be refactored with two slices more (at most nine);
 * otherwise d = solve(LU, r), x += d.  Systems still refining share one
 * grouped launch per phase.  Host outputs per system: iters[i] (corrections
 * applied), berr[i] (last eta), s_final[i], info[i] (> 0: U(info,info) is
 * exactly zero; no refinement).  Synchronizes; allocates and frees device
 * memory for the factors and residuals.  Returns 0, or
 * EMU_ERR_NOT_CONVERGED when a system missed tol at nine slices.
 * Argument numbers: count=1 n/nrhs=2 A/lda=4 B/ldb=6 X/ldx=8 nb=10
 * nslices=11 tol=12 maxiter=13 outputs=14.
 */
int emu_dgesv_batched_ir(int count, const int *n, const int *nrhs, const double *const *A,
                         const int *lda, const double *const *B, const int *ldb,
                         double *const *X, const int *ldx, int nb, int nslices, double tol,
                         int maxiter, int *iters, double *berr, int *s_final, int *info);

/*
 * emu_autotune_batched: time the batched solve of this batch on private
 * copies (inputs untouched) over block sizes {16, 32}, grouped-GEMM grid
 * sizes {1, 2} x (CUs x resident workgroups) and, from six slices on, the
 * grouped GEMM's output tile (0: 64 x 128, eight waves; 1: 64 x 64, four
 * waves), record the fastest for the batch shape (device architecture, HIP
 * runtime version, count, largest n, nslices) — used when nb = 0 — and
 * return it (host outputs; best_tile last).  With EMU_AUTOTUNE_CACHE set
 * the table is read from and written to that file (one line per shape:
 * key nb grid tile).  Allocates and frees device memory.  Tile shapes
 * change no bit of the results.
 */
int emu_autotune_batched(int count, const int *n, const int *nrhs, double *const *A,
                         const int *lda, double *const *B, const int *ldb, int nslices,
                         int *best_nb, int *best_mult, double *best_ms, int *best_tile);

/*
 * Learned slice count (not in the paper; it builds on the paper's
 * observation that an element loses the digits by which its exponent sits
 * below its row's or column's largest, eqn (3)).
 *
 * emu_features: 16 features per 256 x 256 tile (I, J) of the update
 * C = L21 U12 (L21 m x k, ldl; U12 k x n, ldu; device): over the nonzero
 * finite elements of L21's rows in block I and U12's columns in block J,
 * rho = (frexp exponent) - (largest frexp exponent of its row / column);
 * features = [min rho, max rho, mean rho, std rho, fraction of -rho in each
 * of the 12 bins [0,7), [7,14), ..., [77, inf)] (zeros for an empty tile).
 * feat: device float[tiles][16], tile index I + J * ceil(m/256).
 * Argument numbers: m=1 n=2 k=3 L21=4 ldl=5 U12=6 ldu=7 feat=8.
 */
int emu_features(int m, int n, int k, const double *L21, int ldl, const double *U12, int ldu,
                 float *feat);

/* Number of MLP parameters (5703): W1[64][16] b1[64] W2[64][64] b2[64]
 * W3[7][64] b3[7], float32, in that order. */
int emu_mlp_nparam(void);

/*
 * emu_mlp_train_step: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected with `step` >= 1) of the MLP 16 -> 64 (ReLU) -> 64 (ReLU)
 * -> 7 (softmax over s = 3..9) on the mean cross-entropy of B samples:
 * X device float[B][16], labels device int32[B] in 0..6 (class = s - 3),
 * params/m/v device float[nparam], updated in place; loss (device float[B],
 * may be NULL) receives the per-sample losses before the step.
 * Argument numbers: params=1 X=2 labels=3 B=4 m=5 v=6 step=7 lr=8 loss=9.
 */
int emu_mlp_train_step(float *params, const float *X, const int *labels, int B, float *m,
                       float *v, int step, float lr, float *loss);

/* emu_mlp_grad: the gradient of that loss (device float[nparam]) without
 * an update.  Argument numbers: params=1 X=2 labels=3 B=4 grad=5. */
int emu_mlp_grad(const float *params, const float *X, const int *labels, int B, float *grad);

/* emu_mlp_infer: class probabilities (device float[B][7]) and, if s_out is
 * not NULL, the slice count per sample: the smallest s whose cumulative
 * probability reaches conf (device int32[B], values 3..9).
 * Argument numbers: params=1 X=2 B=3 prob=4 s_out=5 conf=6. */
int emu_mlp_infer(const float *params, const float *X, int B, float *prob, int *s_out,
                  float conf);

/*
 * emu_tile_labels: training labels produced by the emulator: X_s = L21 U12
 * emulated with s slices for s = s_lo..s_hi; label of 256 x 256 tile q =
 * the smallest s with ||X_s - X_shi||_F <= tau ||X_shi||_F on that tile
 * (s_hi if none), 1 <= s_lo <= s_hi <= 9.  labels: device int32[tiles]
 * (values s, not classes).
 * Argument numbers: m=1 n=2 k=3 L21=4 ldl=5 U12=6 ldu=7 s_lo=8 s_hi=9
 * tau=10 labels=11.
 */
int emu_tile_labels(int m, int n, int k, const double *L21, int ldl, const double *U12, int ldu,
                    int s_lo, int s_hi, double tau, int *labels);

/*
 * emu_dgetrf_adaptive: emu_dgetrf whose every Schur update uses a slice count
 * per 256 x 256 tile predicted by the MLP (params, device) from
 * emu_features of that update, capped at s_full (3..9); operands are sliced once at
 * s_full and each tile uses the leading digit planes.  The problem lists of
 * every step are built on the device, and with "lu_lookahead" the tiles
 * right of the next panel are updated on the side stream as in emu_dgetrf.
 * smaps (HOST int32, capacity smaps_cap, may be NULL) receives every step's
 * tile counts in order (a step whose tiles do not fit is left out); products
 * (HOST int64[3]) receives the slice products used (sum of tile area x
 * s(s+1)/2), the same at s_full, and the number of tiles.  Synchronizes the
 * stream once, at the end (to return the maps); returns EMU_ERR_PANEL_WAIT
 * when *info then holds EMU_INFO_ABORTED.
 * Argument numbers: m=1 n=2 A=3 lda=4 ipiv=5 info=6 nb=7 params=8
 * s_full=9 conf=10 smaps=11 smaps_cap=12 products=13.
 */
int emu_dgetrf_adaptive(int m, int n, double *A, int lda, int *ipiv, int *info, int nb,
                        const float *params, int s_full, float conf, int *smaps,
                        long long smaps_cap, long long *products);

/*
 * emu_debug_slices: expose the exponent scan and digit slicing of one
 * operand, for bit-exact checks.  X is rows x cols column-major (ldx).
 * by_rows = 1 scales per row (the A side), 0 per column (the B side).
 * exps (device int32[by_rows ? rows : cols]) receives e (0 for zero or
 * non-finite lines; non-finite lines also get flags bit 0 in nonfinite,
 * device int32[same length], may be NULL).  digits (device int8) receives
 * nslices planes, plane i (0-based) holding digit i+1 of every element in
 * the same column-major rows x cols layout with leading dimension rows.
 */
int emu_debug_slices(int rows, int cols, const double *X, int ldx, int by_rows,
                     int nslices, int *exps, int *nonfinite, int8_t *digits);

/*
 * emu_debug_products: the exact slice-product sums D_g, g = 2..t, of the
 * emulated product of A (m x k) and B (k x n) with nslices slices and
 * threshold t, computed by the same MFMA kernels as emu_dgemm_t.  D (device
 * int64) receives t-1 planes, plane g-2 being D_g as an m x n column-major
 * matrix with leading dimension m.
 */
int emu_debug_products(int m, int n, int k, const double *A, int lda,
                       const double *B, int ldb, int nslices, int t,
                       int64_t *D);

#ifdef __cplusplus
}
#endif

#endif /* EMU_H */
