// FP64 panel factorization and triangular solves of the blocked LU
// (paper: section "Dense Numerical Solvers Using FP64 Emulation": the panel,
// where partial pivoting picks the pivots and U11^-1 reaches A21, stays in
// hand-written FP64 code; eqn (8)'s Schur update is the only emulated step).
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
//   * leaves of at most 16 columns, the block in registers (4 rows x 16
//     columns per thread: 1024 rows per 256-thread workgroup, 2048 per
//     512-thread one; a leaf of at most 1024 rows takes the smaller one,
//     one wave per SIMD, whose per-column instruction chain then has its
//     SIMD to itself: an n = 1024 factorization runs 6% faster).  Each column
//     costs one workgroup barrier: every wave publishes its pivot candidate
//     together with a copy of the candidate row (and the owner of row c a
//     copy of row c) into a double-buffered LDS slot, so after the barrier
//     every wave picks the winner and reads both rows without a second
//     round.  Leaves taller than 2048 rows run as one launch of up to 32
//     workgroups (256 threads and 1024 rows each up to 32768 rows, else 512
//     threads and 2048 rows) that exchange their candidates the same way through global
//     memory, with one grid-wide wait per column: every wave reads a share
//     of all workgroups' records, then a workgroup barrier (bounded: a wait
//     that exceeds its bound aborts the leaf, sets info to EMU_INFO_ABORTED
//     and raises EMU_STATUS_PANEL_WAIT).
#include "common.h"
#include "devutil.h"

#include <atomic>
#include <float.h>

namespace emu {

constexpr int LEAF_W = 16;
constexpr int LF_THREADS = 512;
constexpr int LF_WAVES = LF_THREADS / 64;
constexpr int LF_R = 4;                        // rows per thread
constexpr int LF_ROWS = LF_THREADS * LF_R;     // rows per workgroup
constexpr int LF_MAX_G = 32;                   // workgroups of one leaf (65536 rows)
constexpr int LF_SPIN_LIMIT = 1 << 20;         // polls of one grid-wide wait
constexpr int LF_XCDS = 8;                     // XCDs that workgroups are dealt over in turn
constexpr int LF_XCD_MAX_G = 16;              // leaves of at most this many workgroups on one XCD

// Cross-workgroup exchange of a multi-workgroup leaf (global scratch).
// Per column and workgroup one record of 64-bit words, each holding a
// 32-bit payload in its low half and the column's tag in its high half, so
// every word is validated on its own and one read of the records follows
// the last write (no separate flag to poll).  Words: [0] pivot key high,
// [1] key low, [2] its row, [3] the XCD of the workgroup, [4 + 2j],
// [5 + 2j] low and high half of element j of that row, [36 + 2j], [37 + 2j]
// the same for row c (workgroup 0 only, which owns it).  Double-buffered by
// column parity; tags number the columns of all panels of the process from
// 1 (the words are zeroed once per panel).
//
// Where the exchange runs: the dispatcher deals workgroups over the XCDs in
// turn (block b to XCD b mod 8), so a leaf of at most 16 workgroups is
// launched with 8 blocks per workgroup and only blocks 0, 8, 16, ... work,
// all on one XCD.  The records' device-scope loads are served by that XCD's
// L2 for lines written there, so from the second column on (once the first
// column's records have shown every workgroup on one XCD) the records are
// written with plain stores into that L2 instead of through to memory: a
// round trip of about 1500 instead of 2900 shader-clock ticks.  Leaves on
// several XCDs, and larger ones, keep device-scope stores.  Larger leaves
// stay spread out: 17-32 workgroups on one XCD made the n = 32768 LU 11%
// slower.
constexpr int RW = 68;              // words per record
constexpr int RW_MAIN = 36;         // words every workgroup publishes
struct LeafX {
    unsigned long long *rec;        // [2][LF_MAX_G][RW]
    int *abort;                     // set by a workgroup whose wait exceeded the bound
    int *status;                    // device status word (EMU_STATUS_PANEL_WAIT)
    int nopiv;                      // no interchanges: row c is the pivot of column c
    int xs;                         // launch stride: workgroup g is block g xs (1 or LF_XCDS)
};

// The XCD this wave runs on.
__device__ __forceinline__ unsigned xcc_id() {
    unsigned id;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(id));
    return id;
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
__device__ __forceinline__ unsigned ld_relaxed(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct LeafLds {
    long long val[2][LF_WAVES];   // pivot keys
    int idx[2][LF_WAVES];
    double row[2][LF_WAVES][LEAF_W];
    double xrow[2][LEAF_W];
    double grow[2][LF_MAX_G][LEAF_W];   // multi-workgroup: every record's row
    unsigned gkey[2][LF_MAX_G][3];      // and its key (high, low) and row
    unsigned gxcc[LF_MAX_G];            // XCD of each workgroup (first column's records)
    int l2x;                            // all on one XCD: plain record stores
    double xr[2][LEAF_W];
    int abort;
    int piv[LEAF_W];          // pivot row (leaf coordinates) of each column
    int srow[2 * LEAF_W];     // panel-row interchanges: row of each slot
    int ssrc[2 * LEAF_W];     // and the row whose old values it receives
    int nslot;
    int zc;                   // first column with a zero pivot (w if none)
};

// Wave-uniform copy of a double held in a VGPR.
__device__ __forceinline__ double uniform_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// x of the lane that the DPP control CTRL names (rows outside ROWS keep x).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, ROWS, 0xF,
                                               false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// Largest x of the wave, NaN ignored (fmax), as a wave-uniform value: four
// butterfly levels inside rows of 16 lanes, then the row broadcasts that
// leave the maximum in lane 63.
__device__ __forceinline__ double wave_max_f64(double x) {
    x = fmax(x, dpp_f64<0xB1, 0xF>(x));      // quad_perm [1, 0, 3, 2]
    x = fmax(x, dpp_f64<0x4E, 0xF>(x));      // quad_perm [2, 3, 0, 1]
    x = fmax(x, dpp_f64<0x141, 0xF>(x));     // row_half_mirror
    x = fmax(x, dpp_f64<0x140, 0xF>(x));     // row_mirror
    x = fmax(x, dpp_f64<0x142, 0xA>(x));     // row_bcast:15 into rows 1, 3
    x = fmax(x, dpp_f64<0x143, 0xC>(x));     // row_bcast:31 into rows 2, 3
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// Double j (0..15) of the 16-double row r (0..7) of an LDS block that lane l
// holds as doubles 2l and 2l + 1 (see leaf_col): wave-uniform.
__device__ __forceinline__ double row_elem(double e0, double e1, int r, int j) {
    const double e = (j & 1) ? e1 : e0;
    const long long b = __double_as_longlong(e);
    const int src = r * (LEAF_W / 2) + (j >> 1);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// Column c of a leaf: pivot search, interchange, scaling, rank-1 update of
// this thread's rows.  Returns false when a multi-workgroup wait aborted.
// Every decision that depends on the pivot is taken on wave-uniform values,
// so the branches are scalar and each wave issues only the work of its rows.
//
// Pivot search inside a wave: the largest magnitude M by a DPP maximum over
// doubles, then one ballot per row slot q for "valid and |x| == M" (and one
// for NaN, which ranks first); rows are numbered q-major, so the smallest
// row is the lowest set bit of the first non-empty mask.  The wave's
// candidate is published with the key of the pivot order (the magnitude's
// bits, NaN above +inf, -1 for none).
template <bool MULTI, int NT, int k>
__device__ __forceinline__ bool leaf_col(double (&v)[LF_R][LEAF_W], LeafLds &L, int rows,
                                         int base_row, int g, const LeafX &x, unsigned base,
                                         int b) {
    const int c = b + k;                  // column of the leaf, at position k of v
    const int lim = LEAF_W - b;           // positions [lim, 16) hold finished columns
    const int t = threadIdx.x, lane = t & 63;
    const int wid = __builtin_amdgcn_readfirstlane(t >> 6);
    constexpr int buf = k & 1;
    // this wave's candidate
    double m = -1.0;
    bool valid[LF_R];
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * NT;
        // without pivoting row c is the only candidate, so it wins the
        // search below and no interchange follows
        valid[q] = (x.nopiv ? i == c : i >= c) && i < rows;
        if (valid[q]) m = fmax(m, fabs(v[q][k]));
    }
    const double M = wave_max_f64(m);
    int qb = -1;
    unsigned long long mask = 0ull;
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const unsigned long long nm = __ballot(valid[q] && __builtin_isnan(v[q][k]));
        if (qb < 0 && nm != 0ull) {
            qb = q;
            mask = nm;
        }
    }
    const bool wnan = qb >= 0;
    if (!wnan) {
#pragma unroll
        for (int q = 0; q < LF_R; ++q) {
            const unsigned long long mm = __ballot(valid[q] && fabs(v[q][k]) == M);
            if (qb < 0 && mm != 0ull) {
                qb = q;
                mask = mm;
            }
        }
    }
    const int lb = qb >= 0 ? __builtin_ctzll(mask) : 0;
    const long long bk = qb < 0 ? -1ll : wnan ? 0x7FF8000000000000ll : __double_as_longlong(M);
    const int bi = qb < 0 ? INT_MAX : base_row + qb * NT + wid * 64 + lb;
    // the candidate row, and row c (thread c of workgroup 0), to LDS
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        if (q == qb && lane == lb)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) L.row[buf][wid][j] = v[q][j];
    }
    if (g == 0 && wid == 0 && lane == c)
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j) L.xrow[buf][j] = v[0][j];
    if (lane == 0) {
        L.val[buf][wid] = bk;
        L.idx[buf][wid] = bi;
    }
    __syncthreads();
    // the workgroup's winner, and with it (single workgroup) the pivot row:
    // lane l reads doubles 2l, 2l + 1 of the candidate rows, the winner's
    // are then taken with lane reads into scalar registers
    long long wk = L.val[buf][lane & (NT / 64 - 1)];
    int wi = L.idx[buf][lane & (NT / 64 - 1)];
    double pr[LEAF_W];
    double e0 = 0.0, e1 = 0.0;
    if constexpr (!MULTI) {
        const double *flat = &L.row[buf][0][0];
        e0 = flat[2 * lane];
        e1 = flat[2 * lane + 1];
    }
    key_best<NT / 64>(wk, wi);
    wi = __builtin_amdgcn_readfirstlane(wi);
    int p;
    const double *xr;
    if constexpr (!MULTI) {
        p = wi;
        const int wr = ((p - base_row) % NT) / 64;
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j) pr[j] = row_elem(e0, e1, wr, j);
        xr = L.xrow[buf];
    } else {
        const int G = (int)gridDim.x / x.xs;
        const bool l2x = L.l2x != 0;
        const unsigned long long tag = (unsigned long long)(base + (unsigned)c + 1u) << 32;
        if (wid == 0) {
            const long long wkv = (long long)(((unsigned long long)(unsigned)
                                                   __builtin_amdgcn_readfirstlane((int)(wk >> 32))
                                               << 32) |
                                              (unsigned)__builtin_amdgcn_readfirstlane((int)wk));
            // publish: words 0..35 (and 36..67 from workgroup 0), tagged
            unsigned long long *mine = x.rec + ((long long)buf * LF_MAX_G + g) * RW;
            const double *wrow = L.row[buf][((wi - base_row) % NT) / 64];
#pragma unroll 1
            for (int e = lane; e < (g == 0 ? RW : RW_MAIN); e += 64) {
                unsigned pl;
                if (e == 0) {
                    pl = (unsigned)((unsigned long long)wkv >> 32);
                } else if (e == 1) {
                    pl = (unsigned)(unsigned long long)wkv;
                } else if (e == 2) {
                    pl = (unsigned)wi;
                } else if (e == 3) {
                    pl = xcc_id();
                } else {
                    const int j = (e - 4) % 32 / 2, hi = e & 1;
                    const double d = e < RW_MAIN ? wrow[j] : L.xrow[buf][j];
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(d);
                    pl = hi ? (unsigned)(bits >> 32) : (unsigned)bits;
                }
                if (l2x)
                    __hip_atomic_store(mine + e, tag | pl, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                else
                    __hip_atomic_store(mine + e, tag | pl, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // collect: every wave reads its share of the records' words (64-word
        // blocks dealt round-robin over the waves), all loads of a poll in
        // flight together, until all carry this tag; validated payloads go
        // straight to LDS
        {
            const unsigned long long *recs = x.rec + (long long)buf * LF_MAX_G * RW;
            unsigned *grow_w = reinterpret_cast<unsigned *>(&L.grow[buf][0][0]);
            unsigned *xr_w = reinterpret_cast<unsigned *>(&L.xr[buf][0]);
            const int nw = RW_MAIN * G + 32;            // words to read
            constexpr int NWV = NT / 64;
            constexpr int NBLK = (RW_MAIN * LF_MAX_G + 32 + 63) / 64;
            constexpr int NLD = (NBLK + NWV - 1) / NWV;  // loads per lane, at most
            int spins = 0;
            for (;;) {
                bool ok = true;
                unsigned long long wd[NLD];
#pragma unroll
                for (int u = 0; u < NLD; ++u) {
                    const int e = (u * NWV + wid) * 64 + lane;
                    const int sl = e < RW_MAIN * G ? e / RW_MAIN : 0;
                    const int wo = e < RW_MAIN * G ? e % RW_MAIN : RW_MAIN + (e - RW_MAIN * G);
                    wd[u] = e < nw ? __hip_atomic_load(recs + (long long)sl * RW + wo,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                   : tag;
                }
#pragma unroll
                for (int u = 0; u < NLD; ++u) {
                    const int e = (u * NWV + wid) * 64 + lane;
                    if (e >= nw) continue;
                    if ((wd[u] & 0xFFFFFFFF00000000ull) != tag) {
                        ok = false;
                        continue;
                    }
                    const unsigned pl = (unsigned)wd[u];
                    if (e < RW_MAIN * G) {
                        const int sl = e / RW_MAIN, wo = e % RW_MAIN;
                        if (wo < 3)
                            L.gkey[buf][sl][wo] = pl;
                        else if (wo == 3)
                            L.gxcc[sl] = pl;
                        else
                            grow_w[sl * 2 * LEAF_W + (wo - 4)] = pl;
                    } else {
                        xr_w[e - RW_MAIN * G] = pl;
                    }
                }
                if (__ballot(!ok) == 0ull) break;
                if ((++spins & 63) == 0) {
                    if (ld_relaxed(x.abort) != 0) {
                        if (lane == 0) L.abort = 1;
                        break;
                    }
                    if (spins > LF_SPIN_LIMIT) {
                        if (lane == 0) {
                            st_relaxed(x.abort, 1);
                            __hip_atomic_fetch_or(x.status, EMU_STATUS_PANEL_WAIT,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            L.abort = 1;
                        }
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (L.abort) return false;
        // after the launch's first column: when every workgroup runs on one
        // XCD (the same finding in every workgroup), the later columns'
        // records are written into that XCD's L2
        if (c == 0 && t == 0 && x.xs > 1) {
            int same = 1;
            for (int s2 = 1; s2 < G; ++s2) same &= L.gxcc[s2] == L.gxcc[0];
            L.l2x = same;
        }
        // the grid's winner from the staged keys (every wave, same result)
        {
            const int l = lane & (LF_MAX_G - 1);
            long long gv = -1;
            int gi = INT_MAX;
            if (l < G) {
                gv = (long long)(((unsigned long long)L.gkey[buf][l][0] << 32) |
                                 L.gkey[buf][l][1]);
                gi = (int)L.gkey[buf][l][2];
            }
            key_best<LF_MAX_G>(gv, gi);
            p = __builtin_amdgcn_readfirstlane(gi);
        }
        const int gp = (p >= 0 && p < G * (NT * LF_R)) ? p / (NT * LF_R) : 0;
        // the grid winner's row: lane l < 32 reads word l, lane reads make
        // it wave-uniform (scalar registers)
        const unsigned ew = reinterpret_cast<const unsigned *>(L.grow[buf][gp])[lane & 31];
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j) {
            const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)ew, 2 * j);
            const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)ew, 2 * j + 1);
            pr[j] = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
        }
        xr = L.xr[buf];
    }
    const double piv = pr[k];
    if (t == 0) {
        L.piv[c] = p;
        if (piv == 0.0 && L.zc > c) L.zc = c;
    }
    if (piv != 0.0 && p != c) {
        // interchange: row c receives the pivot row, row p the old row c
        if (g == 0 && wid == 0 && lane == c)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) v[0][j] = pr[j];
        const int tp = p - base_row;
        if (tp >= 0 && tp < (NT * LF_R) && wid == (tp % NT) / 64) {
#pragma unroll
            for (int q = 0; q < LF_R; ++q) {
                if (base_row + t + q * NT == p)
#pragma unroll
                    for (int j = 0; j < LEAF_W; ++j) v[q][j] = xr[j];
            }
        }
    }
    // row c after the interchange (the old row c when the pivot is zero)
    if (piv == 0.0) {
#pragma unroll
        for (int j = k + 1; j < LEAF_W; ++j) pr[j] = xr[j];
    }
    // multipliers (rows below c), then the rank-1 update of positions
    // k + 1 .. lim - 1 (rows at or above c keep theirs: l = 0 is not used,
    // so that signed zeros and non-finite pivots rows stay untouched)
    const bool recip = fabs(piv) >= DBL_MIN;
    const double rp = 1.0 / piv;
    double lq[LF_R];
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        double l = v[q][k];
        if (piv != 0.0) l = recip ? l * rp : l / piv;
        lq[q] = l;
    }
    const bool upd0 = base_row + t > c;    // rows of q = 0 below c (q > 0: always)
    if (upd0) v[0][k] = lq[0];
#pragma unroll
    for (int q = 1; q < LF_R; ++q) v[q][k] = lq[q];
#pragma unroll
    for (int j = k + 1; j < LEAF_W; ++j) {
        if (j < lim) {
            const double u = pr[j];
            if (upd0) v[0][j] = v[0][j] - lq[0] * u;
#pragma unroll
            for (int q = 1; q < LF_R; ++q) v[q][j] = v[q][j] - lq[q] * u;
        }
    }
    return true;
}

// The four columns b..b+3 of a group (positions 0..3 of v).
template <bool MULTI, int NT, int k>
__device__ __forceinline__ bool leaf_group(double (&v)[LF_R][LEAF_W], LeafLds &L, int rows,
                                           int w, int base_row, int g, const LeafX &x,
                                           unsigned base, int b) {
    if constexpr (k < 4) {
        if (b + k >= w) return true;
        if (!leaf_col<MULTI, NT, k>(v, L, rows, base_row, g, x, base, b)) return false;
        return leaf_group<MULTI, NT, k + 1>(v, L, rows, w, base_row, g, x, base, b);
    } else {
        return true;
    }
}

// All columns of a leaf: a loop over groups of four columns, each followed
// by a rotation of every row by four positions, so that the loop body names
// its columns by fixed positions (registers) and stays small enough to run
// from the instruction cache; four rotations restore the order.
template <bool MULTI, int NT>
__device__ __forceinline__ bool leaf_cols(double (&v)[LF_R][LEAF_W], LeafLds &L, int rows, int w,
                                          int base_row, int g, const LeafX &x, unsigned base) {
    bool ok = true;
#pragma unroll 1
    for (int b = 0; b < LEAF_W; b += 4) {
        if (b > 0) {
#pragma unroll
            for (int q = 0; q < LF_R; ++q) {
                const double r0 = v[q][0], r1 = v[q][1], r2 = v[q][2], r3 = v[q][3];
#pragma unroll
                for (int j = 0; j < LEAF_W - 4; ++j) v[q][j] = v[q][j + 4];
                v[q][LEAF_W - 4] = r0;
                v[q][LEAF_W - 3] = r1;
                v[q][LEAF_W - 2] = r2;
                v[q][LEAF_W - 1] = r3;
            }
        }
        if (ok && b < w) ok = leaf_group<MULTI, NT, 0>(v, L, rows, w, base_row, g, x, base, b);
    }
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const double r0 = v[q][0], r1 = v[q][1], r2 = v[q][2], r3 = v[q][3];
#pragma unroll
        for (int j = 0; j < LEAF_W - 4; ++j) v[q][j] = v[q][j + 4];
        v[q][LEAF_W - 4] = r0;
        v[q][LEAF_W - 3] = r1;
        v[q][LEAF_W - 2] = r2;
        v[q][LEAF_W - 1] = r3;
    }
    return ok;
}

// The leaf's interchanges applied to the other columns of its panel: ncl
// columns left of the leaf (ending at P - lda) and ncr right of it (from
// P + w lda), rows in leaf coordinates.  The w interchanges are composed
// into one permutation of at most 2w rows by wave 0 (lane x = slot x);
// then every workgroup moves its share of the columns, all reads of a round
// before any write.  Called after the leaf's last column (L.piv complete).
constexpr int SWAP_ROUND = 8;       // passes per read/write round
template <int NT>
__device__ void leaf_panel_swaps(double *P, long long lda, int w, int ncl, int ncr,
                                 LeafLds &L, int g, int G) {
    const int t = threadIdx.x, lane = t & 63;
    __syncthreads();
    if (t < 64) {
        int srow, content;
        const int nslot = wave_compose32(lane < w ? L.piv[lane] : -1, w, srow, content);
        if (lane < 2 * LEAF_W) {
            L.srow[lane] = srow;
            L.ssrc[lane] = content;
        }
        if (lane == 0) L.nslot = nslot;
    }
    __syncthreads();
    const int nslot = L.nslot;
    constexpr int CPP = NT / 32;        // columns per pass
    const int x = t & 31, jj = t >> 5;           // slot, column within a pass
    const int nc = ncl + ncr;
    const int srow = x < nslot ? L.srow[x] : 0;
    const int ssrc = x < nslot ? L.ssrc[x] : 0;
    const bool moves = x < nslot && srow != ssrc;
    for (int j0 = g * CPP; j0 < nc; j0 += CPP * G * SWAP_ROUND) {
        double vals[SWAP_ROUND];
#pragma unroll
        for (int r = 0; r < SWAP_ROUND; ++r) {
            const int j = j0 + r * CPP * G + jj;
            vals[r] = 0.0;
            if (moves && j < nc) {
                const double *col = j < ncl ? P + (long long)(j - ncl) * lda
                                            : P + (long long)(w + j - ncl) * lda;
                vals[r] = col[ssrc];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SWAP_ROUND; ++r) {
            const int j = j0 + r * CPP * G + jj;
            if (moves && j < nc) {
                double *col = j < ncl ? P + (long long)(j - ncl) * lda
                                      : P + (long long)(w + j - ncl) * lda;
                col[srow] = vals[r];
            }
        }
        __syncthreads();
    }
}

// P: top-left of the leaf (global row grow0), rows x w, w <= 16, rows >= w.
// NT threads per workgroup; workgroup g owns rows [4 NT g, 4 NT (g + 1)):
// thread t rows 4 NT g + t + NT q, q = 0..3.  MULTI (NT = 512): the
// workgroups of one leaf run together; the records of column c carry
// sequence number base + c + 1.
template <bool MULTI, int NT>
__global__ __launch_bounds__(NT) void k_leaf(double *__restrict__ P, long long lda,
                                                     int rows, int w, int *ipiv, int grow0,
                                                     int *info, LeafX x, unsigned base,
                                                     int ncl, int ncr) {
    __shared__ LeafLds L;
    const int t = threadIdx.x;
    if (MULTI && blockIdx.x % x.xs != 0) return;    // a slot on another XCD
    const int g = MULTI ? (int)blockIdx.x / x.xs : 0;
    const int base_row = g * (NT * LF_R);
    if (t == 0) {
        L.abort = 0;
        L.zc = w;
        L.l2x = 0;
    }
    double v[LF_R][LEAF_W];
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * NT;
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j)
            v[q][j] = (i < rows && j < w) ? P[i + (long long)j * lda] : 0.0;
    }
    if (!leaf_cols<MULTI, NT>(v, L, rows, w, base_row, g, x, base)) {
        // a grid-wide wait gave up: the factors are invalid; say so in info
        // (every aborting workgroup stores the same value)
        if (t == 0) __hip_atomic_store(info, EMU_INFO_ABORTED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
#pragma unroll
    for (int q = 0; q < LF_R; ++q) {
        const int i = base_row + t + q * NT;
        if (i < rows)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j)
                if (j < w) P[i + (long long)j * lda] = v[q][j];
    }
    // pivot indices and the first zero pivot, once per leaf
    __syncthreads();
    if (g == 0) {
        if (t < w) ipiv[t] = grow0 + L.piv[t] + 1;
        if (t == 0 && L.zc < w && *info == 0) *info = grow0 + L.zc + 1;
    }
    if (ncl + ncr > 0) leaf_panel_swaps<NT>(P, lda, w, ncl, ncr, L, g,
                                                MULTI ? (int)gridDim.x / x.xs : 1);
}

// --------------------------------------------- order-preserving FP64 tiles
// C (m x n) -= A (m x k) B (k x n): every element c_ij is updated for k in
// increasing order as c = c - a_ik b_kj (two roundings), as in elimination.
// Tile TM x 64 (TM = 64, 32 or 16; narrow tiles when the output is small,
// so the launch still covers the chip), 256 threads of (TM / 16) x 4.
// TB: B is given transposed (b_kj at B[j + k ldb]; the Cholesky panel's
// L21 L21^T); lower: only entries with i >= j are written (the rest of C
// is neither stored nor meant to change).
constexpr int GS_N = 64, GS_K = 16;
template <int TM, bool TB = false>
__global__ __launch_bounds__(256) void k_gemm_seq(const double *__restrict__ A, long long lda,
                                                  const double *__restrict__ B, long long ldb,
                                                  double *__restrict__ C, long long ldc, int m,
                                                  int n, int k, int lower = 0) {
    constexpr int RM = TM / 16;
    __shared__ double As[GS_K][TM + 1];
    __shared__ double Bs[GS_K][GS_N + 1];
    const int t = threadIdx.x;
    const int tr = t % 16, tc = t / 16;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * GS_N;
    double c[RM][4];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = m0 + tr + 16 * r, j = n0 + tc + 16 * s;
            c[r][s] = (i < m && j < n) ? C[i + (long long)j * ldc] : 0.0;
        }
    constexpr int PA = TM * GS_K / 256, PB = GS_N * GS_K / 256;
    for (int k0 = 0; k0 < k; k0 += GS_K) {
        // the chunk's loads all in flight before the first store
        double av[PA], bv[PB];
#pragma unroll
        for (int r = 0; r < PA; ++r) {
            const int e = t + 256 * r, ii = e % TM, kk = e / TM;
            const int i = m0 + ii, kx = k0 + kk;
            av[r] = (i < m && kx < k) ? A[i + (long long)kx * lda] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < PB; ++r) {
            const int e = t + 256 * r;
            const int kk = TB ? e / GS_N : e % GS_K, jj = TB ? e % GS_N : e / GS_K;
            const int j = n0 + jj, kx = k0 + kk;
            bv[r] = (j < n && kx < k) ? (TB ? B[j + (long long)kx * ldb]
                                            : B[kx + (long long)j * ldb])
                                      : 0.0;
        }
#pragma unroll
        for (int r = 0; r < PA; ++r) {
            const int e = t + 256 * r;
            As[e / TM][e % TM] = av[r];
        }
#pragma unroll
        for (int r = 0; r < PB; ++r) {
            const int e = t + 256 * r;
            if (TB)
                Bs[e / GS_N][e % GS_N] = bv[r];
            else
                Bs[e % GS_K][e / GS_K] = bv[r];
        }
        __syncthreads();
        const int kend = min(GS_K, k - k0);
        for (int kk = 0; kk < kend; ++kk) {
            double a[RM], b[4];
#pragma unroll
            for (int r = 0; r < RM; ++r) a[r] = As[kk][tr + 16 * r];
#pragma unroll
            for (int s = 0; s < 4; ++s) b[s] = Bs[kk][tc + 16 * s];
#pragma unroll
            for (int r = 0; r < RM; ++r)
#pragma unroll
                for (int s = 0; s < 4; ++s) c[r][s] = c[r][s] - a[r] * b[s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = m0 + tr + 16 * r, j = n0 + tc + 16 * s;
            if (i < m && j < n && (!lower || i >= j)) C[i + (long long)j * ldc] = c[r][s];
        }
}

template <bool TB = false>
static int gemm_seq(const double *A, long long lda, const double *B, long long ldb, double *C,
                    long long ldc, int m, int n, int k, hipStream_t st, int lower = 0) {
    if (m <= 0 || n <= 0 || k <= 0) return 0;
    const int gy = (n + GS_N - 1) / GS_N;
    const long long want = 1024;      // workgroups that keep every CU busy
    if ((long long)((m + 63) / 64) * gy >= want) {
        hipLaunchKernelGGL((k_gemm_seq<64, TB>), dim3((m + 63) / 64, gy), dim3(256), 0, st, A,
                           lda, B, ldb, C, ldc, m, n, k, lower);
    } else if ((long long)((m + 31) / 32) * gy >= want) {
        hipLaunchKernelGGL((k_gemm_seq<32, TB>), dim3((m + 31) / 32, gy), dim3(256), 0, st, A,
                           lda, B, ldb, C, ldc, m, n, k, lower);
    } else {
        hipLaunchKernelGGL((k_gemm_seq<16, TB>), dim3((m + 15) / 16, gy), dim3(256), 0, st, A,
                           lda, B, ldb, C, ldc, m, n, k, lower);
    }
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------- unit-lower TRSM
// B (jb x ncols) <- L^-1 B for jb <= 64: one wave per column, lane i holding
// b_i (the column is read and written contiguously); for k increasing, b_k
// is broadcast from lane k and lanes i > k compute b_i = b_i - l_ik b_k.
// L sits in LDS, column-major, so lane i reads l_ik without bank conflicts.
constexpr int TR_NB = 64;
constexpr int TR_WAVES = 4;
__global__ __launch_bounds__(64 * TR_WAVES) void k_trsm_lanes(const double *__restrict__ L,
                                                              long long ldl, int jb,
                                                              double *__restrict__ B,
                                                              long long ldb, int ncols) {
    __shared__ double Ls[TR_NB * TR_NB];
    {
        // thread (i = t % 64, k = t / 64 + 4 r): all loads before the stores
        constexpr int PER = TR_NB * TR_NB / (64 * TR_WAVES);
        double lv[PER];
        const int i = threadIdx.x & 63, kq = threadIdx.x >> 6;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int k = kq + TR_WAVES * r;
            lv[r] = (i < jb && k < jb) ? L[i + (long long)k * ldl] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) Ls[(kq + TR_WAVES * r) * TR_NB + i] = lv[r];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * TR_WAVES;
    for (int col = blockIdx.x * TR_WAVES + (threadIdx.x >> 6); col < ncols; col += nw) {
        double *bc = B + (long long)col * ldb;
        double b = lane < jb ? bc[lane] : 0.0;
#pragma unroll 8
        for (int k = 0; k < jb - 1; ++k) {
            const long long bits = __double_as_longlong(b);
            const int lo = __builtin_amdgcn_readlane((int)bits, k);
            const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), k);
            const double bk = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
            const double l = Ls[k * TR_NB + lane];
            if (lane > k) b = b - l * bk;
        }
        if (lane < jb) bc[lane] = b;
    }
}

// Blocked: 64-row diagonal solves, order-preserving tile updates between.
int launch_trsm_llnu(const double *L, long long ldl, int jb, double *B, long long ldb,
                     int ncols, hipStream_t stream) {
    if (ncols <= 0 || jb <= 1) return 0;
    constexpr int D = TR_NB;
    int blocks = (ncols + TR_WAVES - 1) / TR_WAVES;
    if (blocks > 1024) blocks = 1024;
    for (int k0 = 0; k0 < jb; k0 += D) {
        const int kb = jb - k0 < D ? jb - k0 : D;
        const double *Lkk = L + k0 + (long long)k0 * ldl;
        double *Bk = B + k0;
        if (kb > 1) {
            hipLaunchKernelGGL(k_trsm_lanes, dim3(blocks), dim3(64 * TR_WAVES), 0, stream, Lkk,
                               ldl, kb, Bk, ldb, ncols);
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
    return align256(2 * LF_MAX_G * RW * sizeof(unsigned long long) + sizeof(int));
}

size_t panel_scratch_bytes(int rows) {
    (void)rows;
    return leafx_bytes();
}

static LeafX leaf_x(char *ws, int *status) {
    LeafX x;
    x.rec = reinterpret_cast<unsigned long long *>(ws);
    x.abort = reinterpret_cast<int *>(x.rec + 2 * LF_MAX_G * RW);
    x.status = status;
    x.nopiv = 0;
    x.xs = 1;
    return x;
}

// One panel factorization: scratch, status word, and the record tag base:
// the panel's first tag (from leaf_tag_base) plus the columns its
// multi-workgroup leaves have finished so far.
struct PanelRun {
    char *ws;
    int *status;
    unsigned arrivals;
    bool pivot;
    bool one_xcd;                   // leaves of at most LF_XCD_MAX_G workgroups on one XCD
};

// Multi-workgroup leaves are plain launches unless this is set.  Their
// G <= 32 workgroups need G compute units at once; work that already holds
// compute units (the look-ahead updates on the side stream) runs to its end
// without them, so a workgroup that waits for one not yet started waits at
// most that long, well inside the bounded wait.  A cooperative launch gives
// the same guarantee at a cost of tens of microseconds per launch.
static thread_local bool g_leaf_cooperative = false;
void set_leaf_cooperative(int on) { g_leaf_cooperative = on != 0; }

// Leaves of at most LF_XCD_MAX_G workgroups gathered on one XCD unless this
// is cleared: they then need that many compute units of one XCD at once,
// which kernels that hold part of every XCD for their whole run (persistent
// launches on other streams) can withhold until they end.
static thread_local bool g_leaf_one_xcd = true;
void set_leaf_one_xcd(int on) { g_leaf_one_xcd = on != 0; }

static int leaf(double *P, long long lda, int rows, int w, int *ipiv, int grow0, int *info,
                int ncl, int ncr, PanelRun &pr, hipStream_t st) {
    LeafX x = leaf_x(pr.ws, pr.status);
    x.nopiv = pr.pivot ? 0 : 1;
    if (rows <= LF_ROWS / 2) {
        hipLaunchKernelGGL((k_leaf<false, LF_THREADS / 2>), dim3(1), dim3(LF_THREADS / 2), 0, st,
                           P, lda, rows, w, ipiv, grow0, info, x, 0u, ncl, ncr);
        EMU_TRY_HIP(hipGetLastError());
        return 0;
    }
    if (rows <= LF_ROWS) {
        hipLaunchKernelGGL((k_leaf<false, LF_THREADS>), dim3(1), dim3(LF_THREADS), 0, st, P, lda,
                           rows, w, ipiv, grow0, info, x, 0u, ncl, ncr);
        EMU_TRY_HIP(hipGetLastError());
        return 0;
    }
    // 256-thread workgroups (one wave per SIMD, 1024 rows each) while at most
    // LF_MAX_G of them cover the leaf, else 512-thread ones
    const bool narrow = rows <= LF_MAX_G * (LF_ROWS / 2);
    const int NTg = narrow ? LF_THREADS / 2 : LF_THREADS;
    const int G = (rows + NTg * LF_R - 1) / (NTg * LF_R);
    if (G > LF_MAX_G) {
        set_error("panel of %d rows above %d", rows, LF_MAX_G * LF_ROWS);
        return EMU_ERR_UNSUPPORTED;
    }
    unsigned base = pr.arrivals;
    const void *fn = narrow ? reinterpret_cast<const void *>(&k_leaf<true, LF_THREADS / 2>)
                            : reinterpret_cast<const void *>(&k_leaf<true, LF_THREADS>);
    if (g_leaf_cooperative) {
        x.xs = 1;
        void *args[] = {&P, &lda, &rows, &w, &ipiv, &grow0, &info, &x, &base, &ncl, &ncr};
        EMU_TRY_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(NTg), args, 0, st));
    } else if (narrow) {
        x.xs = pr.one_xcd && g_leaf_one_xcd && G <= LF_XCD_MAX_G ? LF_XCDS : 1;
        hipLaunchKernelGGL((k_leaf<true, LF_THREADS / 2>), dim3(G * x.xs), dim3(NTg), 0, st,
                           P, lda, rows, w, ipiv, grow0, info, x, base, ncl, ncr);
        EMU_TRY_HIP(hipGetLastError());
    } else {
        x.xs = pr.one_xcd && g_leaf_one_xcd && G <= LF_XCD_MAX_G ? LF_XCDS : 1;
        hipLaunchKernelGGL((k_leaf<true, LF_THREADS>), dim3(G * x.xs), dim3(NTg), 0, st,
                           P, lda, rows, w, ipiv, grow0, info, x, base, ncl, ncr);
        EMU_TRY_HIP(hipGetLastError());
    }
    pr.arrivals += (unsigned)w;
    return 0;
}

// Factor columns [c0, c0 + w) of the panel (pw columns) whose top-left is A
// (global row and column row0), rows [c0, m_rows) of it; ipiv/info as in
// getrf.  Every leaf applies its interchanges to all other columns of the
// panel itself, so no separate interchange pass is needed here.
static int panel_rec(double *A, long long lda, int m_rows, int pw, int c0, int w, int *ipiv,
                     int row0, int *info, PanelRun &pr, hipStream_t st) {
    double *P = A + c0 + (long long)c0 * lda;
    if (w <= LEAF_W)
        return leaf(P, lda, m_rows - c0, w, ipiv + c0, row0 + c0, info, c0, pw - c0 - w, pr,
                    st);
    int w1 = (w / 2) / LEAF_W * LEAF_W;
    if (w1 < LEAF_W) w1 = LEAF_W;
    const int w2 = w - w1;
    EMU_TRY(panel_rec(A, lda, m_rows, pw, c0, w1, ipiv, row0, info, pr, st));
    // U of the right part's top, then the rest of the right part
    EMU_TRY(launch_trsm_llnu(P, lda, w1, P + (long long)w1 * lda, lda, w2, st));
    EMU_TRY(gemm_seq(P + w1, lda, P + (long long)w1 * lda, lda, P + w1 + (long long)w1 * lda,
                     lda, m_rows - c0 - w1, w2, w1, st));
    EMU_TRY(panel_rec(A, lda, m_rows, pw, c0 + w1, w2, ipiv, row0, info, pr, st));
    return 0;
}

// Record tags continue over all panels of the process (never 0, the value of
// a zeroed word), so no record word left from an earlier panel, wherever it
// is cached, carries a tag a later wait looks for.
static std::atomic<unsigned> g_leaf_tags{0u};
static unsigned leaf_tag_base(int cols) {
    for (;;) {
        const unsigned s = g_leaf_tags.fetch_add((unsigned)cols + 1u);
        if (s <= 0xFFFFFFFFu - (unsigned)cols - 1u) return s;
    }
}

int launch_panel(double *A, long long lda, int rows, int jb, int *ipiv, int row0, int *info,
                 char *ws, int *status, hipStream_t stream, bool pivot, bool one_xcd) {
    PanelRun pr{ws, status, rows > LF_ROWS ? leaf_tag_base(jb) : 0u, pivot, one_xcd};
    if (rows > LF_ROWS) {
        // record words (tag 0: not yet written) and the abort flag start at
        // zero (a fill kernel, not a memset)
        LeafX x = leaf_x(ws, status);
        EMU_TRY(launch_fill_int(reinterpret_cast<int *>(x.rec), 0, 2 * 2 * LF_MAX_G * RW + 1,
                                stream));
    }
    return panel_rec(A, lda, rows, jb, 0, jb, ipiv, row0, info, pr, stream);
}


// ------------------------------------------------------ Cholesky panel
// Lower Cholesky of a tall panel (the symmetric variant of the factorization:
// the paper names it beside LU as a solver the emulated update serves).
// Same recursion as the LU panel, without interchanges: a strip of at most
// 16 columns is a leaf; the columns right of a strip lose L21 L_strip^T by
// the order-preserving FP64 tile kernel (B transposed, lower entries only).
// Element (i, j), i >= j, receives a_ij - l_ik l_jk for k = 0..j-1 in that
// order and then l_ij = a_ij * (1 / l_jj), with l_jj = sqrt(a_jj): the
// unblocked right-looking order.
//
// Leaf: every workgroup factors the strip's 16 x 16 diagonal block itself
// (one wave, lane i holding row i; every workgroup computes the same bits),
// so no workgroup waits for another; then each thread finishes its own rows
// below the block (4 per thread, 1024 per workgroup) with the block's L and
// reciprocals from LDS.  Workgroup 0 writes the block's lower triangle and
// the first column whose pivot is not positive (or NaN) into *info (if
// *info is still 0); the factorization is not stopped there, so entries
// from that column on are unspecified.
constexpr int CH_THREADS = 256;
constexpr int CH_R = 4;
constexpr int CH_ROWS = CH_THREADS * CH_R;

__global__ __launch_bounds__(CH_THREADS) void k_chol_leaf(double *__restrict__ P, long long lda,
                                                          int rows, int w, int gcol0,
                                                          int *__restrict__ info) {
    __shared__ double Ld[LEAF_W][LEAF_W + 1];
    __shared__ double rr[LEAF_W];
    __shared__ int fail;
    const int t = threadIdx.x, lane = t & 63;
    const int g = blockIdx.x;
    const int nd = w < rows ? w : rows;          // rows of the diagonal block
    if (t < 64) {
        // lane i < nd holds row i of the diagonal block (lower part)
        double d[LEAF_W];
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j)
            d[j] = (lane < nd && j < w && j <= lane) ? P[lane + (long long)j * lda] : 0.0;
        int first = -1;
#pragma unroll
        for (int c = 0; c < LEAF_W; ++c) {
            if (c < nd) {
                const double a = lane_read_f64(d[c], c);
                if (!(a > 0.0) && first < 0) first = c;
                const double l = sqrt(a);
                const double r = 1.0 / l;
                if (lane == c) d[c] = l;
                if (lane > c) d[c] = d[c] * r;
                if (lane == 0) rr[c] = r;
#pragma unroll
                for (int j = c + 1; j < LEAF_W; ++j) {
                    if (j < nd) {
                        const double ljc = lane_read_f64(d[c], j);
                        if (lane >= j) d[j] = d[j] - d[c] * ljc;
                    }
                }
            }
        }
        if (lane < nd)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j) Ld[lane][j] = d[j];
        if (lane == 0) fail = first;
        if (g == 0 && lane < nd)
#pragma unroll
            for (int j = 0; j < LEAF_W; ++j)
                if (j <= lane) P[lane + (long long)j * lda] = d[j];
    }
    __syncthreads();
    if (g == 0 && t == 0 && fail >= 0 && *info == 0) *info = gcol0 + fail + 1;
    // rows below the diagonal block
#pragma unroll
    for (int q = 0; q < CH_R; ++q) {
        const int i = g * CH_ROWS + t + q * CH_THREADS;
        if (i < nd || i >= rows) continue;
        double a[LEAF_W];
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j) a[j] = j < w ? P[i + (long long)j * lda] : 0.0;
#pragma unroll
        for (int c = 0; c < LEAF_W; ++c) {
            if (c < w) {
                const double x = a[c] * rr[c];
                a[c] = x;
#pragma unroll
                for (int j = c + 1; j < LEAF_W; ++j)
                    if (j < w) a[j] = a[j] - x * Ld[j][c];
            }
        }
#pragma unroll
        for (int j = 0; j < LEAF_W; ++j)
            if (j < w) P[i + (long long)j * lda] = a[j];
    }
}

// Columns [c0, c0 + w) of the panel at A (rows [c0, m_rows)); gcol0: global
// column of panel column 0.
static int chol_rec(double *A, long long lda, int m_rows, int c0, int w, int gcol0, int *info,
                    hipStream_t st) {
    double *P = A + c0 + (long long)c0 * lda;
    const int rows = m_rows - c0;
    if (rows <= 0) return 0;
    if (w <= LEAF_W) {
        const int G = (rows + CH_ROWS - 1) / CH_ROWS;
        hipLaunchKernelGGL(k_chol_leaf, dim3(G), dim3(CH_THREADS), 0, st, P, lda, rows, w,
                           gcol0 + c0, info);
        EMU_TRY_HIP(hipGetLastError());
        return 0;
    }
    int w1 = (w / 2) / LEAF_W * LEAF_W;
    if (w1 < LEAF_W) w1 = LEAF_W;
    const int w2 = w - w1;
    EMU_TRY(chol_rec(A, lda, m_rows, c0, w1, gcol0, info, st));
    // C = panel rows [c0 + w1, m_rows) x columns [c0 + w1, c0 + w) minus
    // L(those rows, strip) L(rows c0 + w1 .. c0 + w, strip)^T, lower part
    EMU_TRY(gemm_seq<true>(P + w1, lda, P + w1, lda, P + w1 + (long long)w1 * lda, lda,
                           rows - w1, w2, w1, st, 1));
    return chol_rec(A, lda, m_rows, c0 + w1, w2, gcol0, info, st);
}

int launch_chol_panel(double *A, long long lda, int rows, int jb, int col0, int *info,
                      hipStream_t stream) {
    return chol_rec(A, lda, rows, 0, jb, col0, info, stream);
}

}  // namespace emu
