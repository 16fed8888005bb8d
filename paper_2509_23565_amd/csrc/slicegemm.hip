// INT8 slice-product GEMM on gfx950 MFMA with the FP64 recombination fused
// into its epilogue.
//
// Paper: section "Emulation of FP64 and INT8 Splitting", eqn (2) and the
// truncation threshold t; the Schur update of eqn (8) is the call site in
// the LU.  For every output element the kernel forms the exact diagonal sums
// D_g = sum_{i+j=g} A_i B_j, g = 2..t, in INT32 accumulator tiles, one per
// diagonal ("slot"), loading each digit fragment once per K step and reusing
// it for every pair on every diagonal it takes part in.
//
// Data path per workgroup (8 waves, two per SIMD):
//   - the digit planes are stored in MFMA fragment order (1 KB per 32 lines
//     x 32 k), so a K step of the workgroup tile is a list of whole
//     fragments; they are copied global -> LDS with 16-byte direct-to-LDS
//     loads (no VGPR staging) into two to four LDS stages (more for the
//     short K steps of few digits), one barrier per K step;
//   - each wave reads its own A and B fragments of every digit from LDS and
//     issues all pairs (i, j) with i + j <= t on 32x32x32 INT8 MFMA;
//   - workgroups are numbered so that each of the 8 XCDs receives one
//     contiguous range of output tiles, walked in groups of 8 tile rows, so
//     the concurrently running tiles of an XCD share A and B panels in its L2.
//
// Exactness: a slot holding p pairs over a K range of length L is bounded by
// p L 127^2, which must stay below 2^31.  The longest diagonal (t = s + 1
// has s pairs) can be split over two slots ("split" variant) so that no slot
// holds more than max(s - 1, ceil(s / 2)) pairs; K up to 16640 then needs no
// chunking for any s <= 9 (s = 16: up to 16640 as well, eight pairs per slot).  Longer K is cut into chunks of the exact-INT32 length; each chunk
// writes its INT32 diagonal sums to scratch and a combine pass adds them in
// INT64 before recombining.  The cuts depend on (s, t, k) only, so tile
// shapes never change a bit of the result.
//
// Epilogue (fixed order): S = 0; for g = t..2: S = fl(S + D_g 2^-7g);
// X = ldexp(S, e_p + f_q); C = fma(alpha, X, beta C) (beta = 0: fma(alpha,
// X, 0)).  The D_g to double conversions and the power-of-two scalings are
// exact (|D_g| < 2^53).
//
// Operand roles: the MFMA's first operand is the B-digit fragment and its
// second the A-digit fragment, so the accumulator holds C^T blocks in which
// lane l owns row m = l%32 of C: stores to column-major C are 32 consecutive
// doubles per register.
#include "common.h"

namespace emu {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// s_waitcnt immediate for gfx9: vmcnt(0), expcnt/lgkmcnt unconstrained.
constexpr int WAIT_VMCNT0 = 0x0F70;

// One 1 KB fragment global -> LDS by the calling wave (16 bytes per lane,
// lane l's bytes at lds + 16 l).  Written as inline assembly so that the
// compiler's wait-count bookkeeping does not see an LDS-writing memory
// operation: with one in a loop it waits for every outstanding LDS read
// before each MFMA group.  The kernels wait for these loads explicitly
// (a vmcnt wait before the barrier that publishes an LDS stage).  M0 (a register
// the compiler reserves, so it cannot be named as clobbered) is set here;
// the compiled kernels of this file use M0 nowhere else (no LDS DMA or
// message instructions of their own), which the generated code shows.
__device__ __forceinline__ void dma_frag(const int8_t *gsrc, int8_t *lds) {
    // a flat (generic) address of LDS holds the LDS byte offset in its low
    // 32 bits (the shared aperture is in the high half)
    const unsigned dst = (unsigned)(uintptr_t)lds;
    asm volatile("s_mov_b32 m0, %1\n\t"
                 "s_nop 0\n\t"
                 "global_load_lds_dwordx4 %0, off"
                 :
                 : "v"(gsrc), "s"(__builtin_amdgcn_readfirstlane(dst))
                 : "memory");
}

// ------------------------------------------------------------- diagonals
__host__ __device__ constexpr int diag_pairs(int s, int g) {
    int lo = g - s > 1 ? g - s : 1;
    int hi = g - 1 < s ? g - 1 : s;
    return hi >= lo ? hi - lo + 1 : 0;
}

// Pairs (i <= s, j <= sb) on diagonal g.
static int diag_pairs_ab(int s, int sb, int g) {
    const int lo = g - sb > 1 ? g - sb : 1;
    const int hi = g - 1 < s ? g - 1 : s;
    return hi >= lo ? hi - lo + 1 : 0;
}

// Pairs per slot at most: s (plain), s - 1 (split longest diagonal); B with
// sb slices: at most sb.
static int max_slot_pairs(int s, int t, bool split, int sb = 0) {
    if (sb <= 0) sb = s;
    int m = 0;
    for (int g = 2; g <= t; ++g) {
        int p = diag_pairs_ab(s, sb, g);
        if (split && g == t) p = (p + 1) / 2;
        if (p > m) m = p;
    }
    return m;
}

// K-length (multiple of 32) whose INT32 slot sums cannot overflow.
static long long exact_len(int pairs) {
    long long L = 2147483647LL / ((long long)pairs * 127 * 127);
    return L / K_BLOCK * K_BLOCK;
}

template <int S, int T, bool SPLIT, int SB = S>
struct Cfg {
    // SB: B's slice count (unequal splits, SB < S: B digits beyond SB are
    // not there, so pairs (i, j) have j <= SB)
    static_assert(SB >= 1 && SB <= S && (SB == S || (!SPLIT && T == S + 1)), "unequal splits");
    static constexpr int NSLOT = (T - 1) + (SPLIT ? 1 : 0);
    // wave tile WM x WN blocks of 32x32; workgroup WAVES_M x WAVES_N waves.
    // Two 32x32 blocks per wave while the accumulators fit two waves per
    // SIMD (16 NSLOT VGPRs per block), else one.  Above ten slots (s >= 10)
    // the accumulators (16 NSLOT), the B digits kept in registers (4 S) and
    // the streamed A digit need more than half of a SIMD's 512 registers per
    // lane: four waves, one per SIMD, 64 x 64 tiles.
    static constexpr bool WIDE = NSLOT > 10;
    static constexpr int WM = 1;
    static constexpr int WN = (NSLOT <= 5) ? 2 : 1;
    static constexpr int WAVES_M = WIDE ? 2 : (WN == 2) ? 4 : 2;
    static constexpr int WAVES_N = WIDE ? 2 : (WN == 2) ? 2 : 4;
    static constexpr int NW = WAVES_M * WAVES_N;
    static constexpr int THREADS = 64 * NW;
    static constexpr int TM = WAVES_M * WM;     // 32-row blocks per tile
    static constexpr int TN = WAVES_N * WN;     // 32-column blocks per tile
    static constexpr int FRA = S * TM;
    static constexpr int FRB = SB * TN;
    static constexpr int FR = FRA + FRB;        // fragments per K step
    // LDS stages (K steps in flight).  With S <= 3 a K step is too short
    // (12 MFMAs per wave at S = 3) to cover the latency of its fragment
    // copies with one step of look-ahead: four stages (96 KB at S = 3) run
    // the 16384^3 product 10% faster.  From S = 4 on two stages measure as
    // fast as three or four (S = 6, 7 slower with more).
    static constexpr int STAGE = FR * FRAG_BYTES;
    static constexpr int NST = (S <= 3) ? 4 : 2;
    // copies each wave issues per K step, at least
    static constexpr int NQ_MIN = FR / NW;
    // slot of pair (i, j): diagonal g = i + j -> g - 2; with SPLIT the
    // upper half of the longest diagonal goes to the extra slot.
    static constexpr int slot(int i, int j) {
        return (SPLIT && i + j == T && i > (S + 1) / 2) ? T - 1 : i + j - 2;
    }
};


// XCD-aware tile order: consecutive workgroups go to different XCDs
// (round-robin dispatch).
// map 0: XCD x receives the contiguous range of tile ids x*per.., walked in
//   groups of GROUP_M tile rows, so the tiles running together on one XCD
//   share A and B panels in its L2.
// map 1 (tiles_m and tiles_n multiples of 16): the 256 workgroups that run
//   together (32 per XCD, one per CU) cover one block of 16 x 16 tiles, XCD x
//   its 8 x 4 sub-block (x % 2, x / 2); the XCDs then read the same A and B
//   panels at about the same K position, so the memory-side last-level cache
//   serves what one XCD fetched from HBM to the others, while each XCD's L2
//   still shares panels among its own 32 tiles (1-3% faster at s = 3, 5, 9
//   for m = n = k = 16384).
__device__ __forceinline__ void tile_of(int L, int tiles_m, int tiles_n, int map, int *tm,
                                        int *tn) {
    constexpr int NXCD = 8, GROUP_M = 8;
    const int xcd = L % NXCD, q = L / NXCD;
    if (map == 1) {
        const int sb = q / 32, r = q % 32;
        const int sbm = tiles_m / 16;
        *tm = (sb % sbm) * 16 + (xcd % 2) * 8 + r % 8;
        *tn = (sb / sbm) * 16 + (xcd / 2) * 4 + r / 8;
        return;
    }
    const int num = tiles_m * tiles_n;
    const int per = num / NXCD, rem = num % NXCD;
    const int pid = xcd < rem ? xcd * (per + 1) + q
                              : rem * (per + 1) + (xcd - rem) * per + q;
    const int group_size = GROUP_M * tiles_n;
    const int first_m = (pid / group_size) * GROUP_M;
    const int gm = min(tiles_m - first_m, GROUP_M);
    const int in = pid % group_size;
    *tm = first_m + in % gm;
    *tn = in / gm;
}

// One output tile (tm, tn) over K blocks [kb0, kb1) of problem p.
// MODE 0: recombine into C.  MODE 2: write the INT32 D_g of chunk `chunk`.
// PF: read this wave's C block (beta != 0) before the K loop, so that its
// latency overlaps the first fragment copies; for short K (the grouped
// launches of small updates, one K step) the C read is most of a tile's time.
template <int S, int T, bool SPLIT, int MODE, bool PF = false, int SB = S>
__device__ __forceinline__ void sgemm_tile(const GemmArgs &p, int tm, int tn, int kb0,
                                           int kb1, int chunk, int8_t *lds) {
    using CF = Cfg<S, T, SPLIT, SB>;
    static_assert(!PF || (MODE == 0 && CF::WM * CF::WN == 1), "C prefetch: one block per wave");
    constexpr int TM = CF::TM, TN = CF::TN, FRA = CF::FRA, FR = CF::FR, NW = CF::NW;
    constexpr int NSLOT = CF::NSLOT;

    const int lane = threadIdx.x & 63;
    // wave index as a uniform (scalar) value, so per-wave addresses live in SGPRs
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int mb0 = tm * TM, nb0 = tn * TN;
    const int wm = w % CF::WAVES_M, wn = w / CF::WAVES_M;

    // fragment sources of this wave for one K step (uniform per wave)
    const int8_t *src[(FR + NW - 1) / NW];
#pragma unroll
    for (int q = 0; q < (FR + NW - 1) / NW; ++q) {
        const int f = q * NW + w;
        const int8_t *s_ = nullptr;
        if (f < FRA) {
            const int d = f / TM, i = f % TM;
            s_ = p.Ap + d * p.a_plane + (size_t)(mb0 + i) * p.KB * FRAG_BYTES;
        } else if (f < FR) {
            const int g = f - FRA;
            const int d = g / TN, j = g % TN;
            s_ = p.Bp + d * p.b_plane + (size_t)(nb0 + j) * p.KB * FRAG_BYTES;
        }
        src[q] = s_ ? s_ + lane * 16 : nullptr;
    }
    auto issue = [&](int8_t *buf, int kb) {
#pragma unroll
        for (int q = 0; q < (FR + NW - 1) / NW; ++q) {
            const int f = q * NW + w;
            if (f < FR)
                dma_frag(src[q] + (size_t)kb * FRAG_BYTES, buf + f * FRAG_BYTES);
        }
    };

    v16i acc[CF::WM][CF::WN][NSLOT];
#pragma unroll
    for (int i = 0; i < CF::WM; ++i)
#pragma unroll
        for (int j = 0; j < CF::WN; ++j)
#pragma unroll
            for (int g = 0; g < NSLOT; ++g)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][g][r] = 0;

    double cpre[16];
    if constexpr (PF) {
        const int m = (mb0 + wm) * 32 + (lane & 31);
        const int nbase = (nb0 + wn) * 32 + 4 * (lane >> 5);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n = nbase + 8 * (r >> 2) + (r & 3);
            cpre[r] = (p.beta != 0.0 && m < p.M && n < p.N) ? p.C[(size_t)n * p.ldc + m] : 0.0;
        }
    }
    // Stage (kb - kb0) % NST holds K step kb.  Before the barrier that
    // publishes step kb, each wave waits for its own copies of that step:
    // the copies of the NST - 2 later steps already issued may stay in
    // flight (loads complete in order), near the end of K all of them.
    constexpr int NST = CF::NST;
    constexpr int AHEAD = (NST - 2) * CF::NQ_MIN;
    static_assert(AHEAD < 64, "vmcnt field");
    constexpr int WAIT_AHEAD = (AHEAD & 15) | ((AHEAD >> 4) << 14) | 0x0F70;
#pragma unroll
    for (int q = 0; q < NST - 1; ++q)
        if (kb0 + q < kb1) issue(lds + q * CF::STAGE, kb0 + q);
    int st = 0;                                   // stage of step kb
    for (int kb = kb0; kb < kb1; ++kb) {
        if (NST > 2 && kb + NST - 2 < kb1)
            __builtin_amdgcn_s_waitcnt(WAIT_AHEAD);
        else
            __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
        __syncthreads();
        const int8_t *cur = lds + st * CF::STAGE;
        // the stage read in the previous step is free for step kb + NST - 1
        const int fs = (st == 0) ? NST - 1 : st - 1;
        if (kb + NST - 1 < kb1) issue(lds + fs * CF::STAGE, kb + NST - 1);
        st = (st == NST - 1) ? 0 : st + 1;
#pragma unroll
        for (int i = 0; i < CF::WM; ++i) {
#pragma unroll
            for (int j = 0; j < CF::WN; ++j) {
                // A digits are streamed least significant first: digit ii
                // pairs with B digits 1..min(S, T - ii), so with T = S + 1
                // each step needs exactly one new B digit besides the next A
                // digit, and the first MFMA waits for two fragments instead
                // of S + 1 (all waves start a K step together after the
                // barrier, and LDS serves their reads in order).  B digits
                // stay in registers once read.
                static_assert(T == S + 1 || T == 2 * S, "supported thresholds");
                constexpr bool TRI = (T == S + 1);
                const int8_t *pa = cur + (wm * CF::WM + i) * FRAG_BYTES + lane * 16;
                const int8_t *pb = cur + (FRA + wn * CF::WN + j) * FRAG_BYTES + lane * 16;
                v4i b[SB];
                v4i a = *reinterpret_cast<const v4i *>(pa + (S - 1) * TM * FRAG_BYTES);
#pragma unroll
                for (int d = 0; d < (TRI ? 1 : SB); ++d)
                    b[d] = *reinterpret_cast<const v4i *>(pb + d * TN * FRAG_BYTES);
                __builtin_amdgcn_sched_group_barrier(0x100, TRI ? 2 : SB + 1, 0);
#pragma unroll
                for (int ii = S; ii >= 1; --ii) {
                    v4i an = a;
                    if (ii > 1) {
                        an = *reinterpret_cast<const v4i *>(pa + (ii - 2) * TM * FRAG_BYTES);
                        // the next B digit, while there is one (SB < S: the
                        // last S - SB A digits take no new B digit)
                        if (TRI && (S + 1 - ii) < SB) {
                            b[(S + 1 - ii) < SB ? S + 1 - ii : 0] = *reinterpret_cast<const v4i *>(
                                pb + (S + 1 - ii) * TN * FRAG_BYTES);
                            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                        } else {
                            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                        }
                    }
#pragma unroll
                    for (int jj = 1; jj <= SB; ++jj)
                        if (ii + jj <= T) {
                            const int sl = CF::slot(ii, jj);
                            acc[i][j][sl] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                b[jj - 1], a, acc[i][j][sl], 0, 0, 0);
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                        }
                    a = an;
                }
            }
        }
    }

    // ---------------------------------------------------------- epilogue
#pragma unroll
    for (int i = 0; i < CF::WM; ++i) {
        const int m = (mb0 + wm * CF::WM + i) * 32 + (lane & 31);
        if (m >= p.M) continue;
        const int ca = p.codeA[m];
        const bool badA = ca == CODE_NONFINITE;
        const int ea = (ca == CODE_ZERO || badA) ? 0 : ca;
#pragma unroll
        for (int j = 0; j < CF::WN; ++j) {
            const int nbase = (nb0 + wn * CF::WN + j) * 32 + 4 * (lane >> 5);
            // all C reads of the block before any store, so the 16 loads are
            // in flight together instead of one round trip per element
            double cin[16];
            if constexpr (PF) {
#pragma unroll
                for (int r = 0; r < 16; ++r) cin[r] = cpre[r];
            } else if (MODE != 2) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int n = nbase + 8 * (r >> 2) + (r & 3);
                    cin[r] = (p.beta != 0.0 && n < p.N) ? p.C[(size_t)n * p.ldc + m] : 0.0;
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int n = nbase + 8 * (r >> 2) + (r & 3);
                if (n >= p.N || (p.lower && n > m)) continue;
                if (MODE == 2) {
#pragma unroll
                    for (int g = 0; g < T - 1; ++g)
                        p.part[(((size_t)chunk * (T - 1) + g) * p.N + n) * p.M + m] =
                            acc[i][j][g][r];
                } else {
                    const int cb = p.codeB[n];
                    const bool badB = cb == CODE_NONFINITE;
                    const int eb = (cb == CODE_ZERO || badB) ? 0 : cb;
                    double Ssum = 0.0;
#pragma unroll
                    for (int g = T - 2; g >= 0; --g) {
                        long long D = acc[i][j][g][r];
                        if constexpr (SPLIT) {
                            if (g == T - 2) D += acc[i][j][T - 1][r];
                        }
                        // weight 2^-7(g+2), an exact power of two
                        const double wgt =
                            __longlong_as_double((long long)(1023 - 7 * (g + 2)) << 52);
                        Ssum = Ssum + (double)D * wgt;
                    }
                    const double X = ldexp(Ssum, ea + eb);
                    double *pc = p.C + (size_t)n * p.ldc + m;
                    double out = (p.beta == 0.0) ? fma(p.alpha, X, 0.0)
                                                 : fma(p.alpha, X, p.beta * cin[r]);
                    if (badA || badB) out = __builtin_nan("");
                    *pc = out;
                }
            }
        }
    }
}

template <int S, int T, bool SPLIT, int MODE, int SB = S>
__global__ __launch_bounds__((Cfg<S, T, SPLIT, SB>::THREADS)) void k_slicegemm(GemmArgs p) {
    using CF = Cfg<S, T, SPLIT, SB>;
    __shared__ __attribute__((aligned(1024))) int8_t lds[CF::NST * CF::STAGE];
    int tm, tn;
    tile_of(blockIdx.x, p.tiles_m, p.tiles_n, p.map, &tm, &tn);
    // lower-triangle update: a tile wholly above the diagonal has no work
    // (uniform per workgroup, before any barrier)
    if (p.lower && (tm + 1) * CF::TM * 32 <= tn * CF::TN * 32) return;
    int kb0 = 0, kb1 = p.KB;
    if (MODE == 2) {
        kb0 = blockIdx.y * p.chunk_kb;
        kb1 = min(p.KB, kb0 + p.chunk_kb);
    }
    sgemm_tile<S, T, SPLIT, MODE, false, SB>(p, tm, tn, kb0, kb1, blockIdx.y, lds);
}

// Persistent grouped form: every workgroup walks the concatenated tile list
// of all problems (tile_prefix[q] = first tile of problem q).
template <int S, int T>
__global__ __launch_bounds__(512) void k_slicegemm_grouped(const GemmArgs *__restrict__ probs,
                                                           const int *__restrict__ tile_prefix,
                                                           int nprob, int total,
                                                           const int *__restrict__ dcounts) {
    using CF = Cfg<S, T, false>;
    static_assert(CF::THREADS == 512, "launch bounds assume 8 waves");
    if (dcounts) {              // list built on the device
        nprob = dcounts[0];
        total = dcounts[1];
    }
    __shared__ __attribute__((aligned(1024))) int8_t lds[CF::NST * CF::STAGE];
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int lo = __builtin_amdgcn_readfirstlane(wave_search(tile_prefix, nprob, tile));
        const GemmArgs p = probs[lo];
        const int local = tile - tile_prefix[lo];
        const int tm = local % p.tiles_m, tn = local / p.tiles_m;
        __syncthreads();                          // LDS of the previous tile is free
        sgemm_tile<S, T, false, 0, Cfg<S, T, false>::WN == 1>(p, tm, tn, 0, p.KB, 0, lds);
    }
}

// Grouped form for problems of one K step (K <= 32: the updates of the
// batched LU), software-pipelined across the tiles a workgroup walks.  A
// tile of one K step is a chain of latencies (fragment copy, C read, a few
// MFMAs, the recombination and the C write), so tile t + 1's fragments are
// copied into the other LDS buffer while tile t is multiplied and
// recombined, the problem of tile t + 2 is looked up, and tile t + 1's C
// block and exponents are read, all before the barrier that starts t + 1.
// One 32x32 block per wave (the slot counts of s >= 6).
// Tile of the pipelined grouped kernel: 2 x WNW waves, one 32x32 block each
// (64 x 128 with four waves along N, 64 x 64 with two; the autotuner of the
// batched form chooses).
template <int S, int WNW>
struct G1Cfg {
    static constexpr int WAVES_M = 2, WAVES_N = WNW;
    static constexpr int NW = WAVES_M * WAVES_N, THREADS = 64 * NW;
    static constexpr int TM = WAVES_M, TN = WAVES_N;
    static constexpr int FRA = S * TM, FRB = S * TN, FR = FRA + FRB;
    static constexpr int NSLOT = S;          // t = s + 1: diagonals 2..s + 1
    static constexpr int slot(int i, int j) { return i + j - 2; }
};

template <int S, int WNW>
__global__ __launch_bounds__((G1Cfg<S, WNW>::THREADS)) void k_slicegemm_grouped1(
    const GemmArgs *__restrict__ probs, const int *__restrict__ tile_prefix, int nprob,
    int total) {
    constexpr int T = S + 1;
    using CF = G1Cfg<S, WNW>;
    constexpr int TM = CF::TM, TN = CF::TN, FRA = CF::FRA, FR = CF::FR, NW = CF::NW;
    constexpr int NSLOT = CF::NSLOT, NQ = (FR + NW - 1) / NW;
    __shared__ __attribute__((aligned(1024))) int8_t lds0[FR * FRAG_BYTES];
    __shared__ __attribute__((aligned(1024))) int8_t lds1[FR * FRAG_BYTES];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = w % CF::WAVES_M, wn = w / CF::WAVES_M;

    // problem and tile coordinates of a tile
    auto locate = [&](int tile, GemmArgs &q, int &tm, int &tn) {
        const int lo = __builtin_amdgcn_readfirstlane(wave_search(tile_prefix, nprob, tile));
        q = probs[lo];
        const int local = tile - tile_prefix[lo];
        tm = local % q.tiles_m;
        tn = local / q.tiles_m;
    };
    // this wave's share of the tile's fragments (one K step) into buf
    auto issue = [&](const GemmArgs &q, int tm, int tn, int8_t *buf) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int f = k * NW + w;
            if (f < FRA) {
                const int d = f / TM, i = f % TM;
                dma_frag(q.Ap + d * q.a_plane + (size_t)(tm * TM + i) * FRAG_BYTES + lane * 16,
                         buf + f * FRAG_BYTES);
            } else if (f < FR) {
                const int g = f - FRA;
                const int d = g / TN, j = g % TN;
                dma_frag(q.Bp + d * q.b_plane + (size_t)(tn * TN + j) * FRAG_BYTES + lane * 16,
                         buf + f * FRAG_BYTES);
            }
        }
    };
    // this lane's C elements (beta != 0) and exponent codes of the tile
    double cin[16];
    int ca, cb[16];
    auto prefetch = [&](const GemmArgs &q, int tm, int tn) {
        const int m = (tm * TM + wm) * 32 + (lane & 31);
        const int nbase = (tn * TN + wn) * 32 + 4 * (lane >> 5);
        ca = m < q.M ? q.codeA[m] : 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n = nbase + 8 * (r >> 2) + (r & 3);
            const bool in = m < q.M && n < q.N;
            cin[r] = (q.beta != 0.0 && in) ? q.C[(size_t)n * q.ldc + m] : 0.0;
            cb[r] = n < q.N ? q.codeB[n] : 0;
        }
    };

    int tile = blockIdx.x;
    if (tile >= total) return;                    // uniform per workgroup
    GemmArgs p, pn;
    int tm, tn, tmn = 0, tnn = 0;
    locate(tile, p, tm, tn);
    issue(p, tm, tn, lds0);
    prefetch(p, tm, tn);
    int next = tile + (int)gridDim.x;
    if (next < total) locate(next, pn, tmn, tnn);
    for (int it = 0;; ++it) {
        int8_t *cur = (it & 1) ? lds1 : lds0;
        int8_t *nxt = (it & 1) ? lds0 : lds1;
        // tile's fragments are in cur for every wave, its C block and
        // exponents in registers, the next tile's problem in pn
        __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
        __syncthreads();
        if (next < total) issue(pn, tmn, tnn, nxt);

        v16i acc[NSLOT];
#pragma unroll
        for (int g = 0; g < NSLOT; ++g)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[g][r] = 0;
        {
            const int8_t *pa = cur + wm * FRAG_BYTES + lane * 16;
            const int8_t *pb = cur + (FRA + wn) * FRAG_BYTES + lane * 16;
            v4i b[S];
            v4i a = *reinterpret_cast<const v4i *>(pa + (S - 1) * TM * FRAG_BYTES);
            b[0] = *reinterpret_cast<const v4i *>(pb);
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
            for (int ii = S; ii >= 1; --ii) {
                v4i an = a;
                if (ii > 1) {
                    an = *reinterpret_cast<const v4i *>(pa + (ii - 2) * TM * FRAG_BYTES);
                    b[S + 1 - ii] = *reinterpret_cast<const v4i *>(pb + (S + 1 - ii) * TN * FRAG_BYTES);
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                }
#pragma unroll
                for (int jj = 1; jj <= S; ++jj)
                    if (ii + jj <= T) {
                        const int sl = CF::slot(ii, jj);
                        acc[sl] = __builtin_amdgcn_mfma_i32_32x32x32_i8(b[jj - 1], a, acc[sl], 0, 0, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    }
                a = an;
            }
        }

        // recombination of the tile (fixed order, as in sgemm_tile)
        {
            const int m = (tm * TM + wm) * 32 + (lane & 31);
            const int nbase = (tn * TN + wn) * 32 + 4 * (lane >> 5);
            const bool badA = ca == CODE_NONFINITE;
            const int ea = (ca == CODE_ZERO || badA) ? 0 : ca;
            if (m < p.M) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int n = nbase + 8 * (r >> 2) + (r & 3);
                    if (n >= p.N) continue;
                    const bool badB = cb[r] == CODE_NONFINITE;
                    const int eb = (cb[r] == CODE_ZERO || badB) ? 0 : cb[r];
                    double Ssum = 0.0;
#pragma unroll
                    for (int g = T - 2; g >= 0; --g) {
                        const double wgt =
                            __longlong_as_double((long long)(1023 - 7 * (g + 2)) << 52);
                        Ssum = Ssum + (double)acc[g][r] * wgt;
                    }
                    const double X = ldexp(Ssum, ea + eb);
                    double out = (p.beta == 0.0) ? fma(p.alpha, X, 0.0)
                                                 : fma(p.alpha, X, p.beta * cin[r]);
                    if (badA || badB) out = __builtin_nan("");
                    p.C[(size_t)n * p.ldc + m] = out;
                }
            }
        }
        if (next >= total) break;
        // advance: tile <- next; look up the one after it and read the new
        // tile's C block and exponents (both land before the next barrier)
        tile = next;
        p = pn;
        tm = tmn;
        tn = tnn;
        next = tile + (int)gridDim.x;
        if (next < total) locate(next, pn, tmn, tnn);
        prefetch(p, tm, tn);
    }
}

// Chunk combine: D_g = sum over chunks (INT64), then either the raw sums
// (debug, Dout != null) or the recombination into C.
template <int T>
__global__ __launch_bounds__(256) void k_combine(GemmArgs p, int nchunks, int64_t *Dout) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long MN = (long long)p.M * p.N;
    if (idx >= MN) return;
    const int m = (int)(idx % p.M), n = (int)(idx / p.M);
    long long D[T - 1];
#pragma unroll
    for (int g = 0; g < T - 1; ++g) {
        long long acc = 0;
        for (int c = 0; c < nchunks; ++c) acc += p.part[((size_t)c * (T - 1) + g) * MN + idx];
        D[g] = acc;
    }
    if (Dout) {
#pragma unroll
        for (int g = 0; g < T - 1; ++g) Dout[(size_t)g * MN + idx] = D[g];
        return;
    }
    const int ca = p.codeA[m], cb = p.codeB[n];
    const bool bad = ca == CODE_NONFINITE || cb == CODE_NONFINITE;
    const int ea = (ca == CODE_ZERO || ca == CODE_NONFINITE) ? 0 : ca;
    const int eb = (cb == CODE_ZERO || cb == CODE_NONFINITE) ? 0 : cb;
    double Ssum = 0.0;
#pragma unroll
    for (int g = T - 2; g >= 0; --g) {
        const double wgt = __longlong_as_double((long long)(1023 - 7 * (g + 2)) << 52);
        Ssum = Ssum + (double)D[g] * wgt;
    }
    const double X = ldexp(Ssum, ea + eb);
    double *pc = p.C + (size_t)n * p.ldc + m;
    double out = (p.beta == 0.0) ? fma(p.alpha, X, 0.0) : fma(p.alpha, X, p.beta * *pc);
    if (bad) out = __builtin_nan("");
    *pc = out;
}

// ---------------------------------------------------------------- host
static thread_local int t_map = 1;

void set_gemm_map(int map) { t_map = map; }
int gemm_map() { return t_map; }

bool gemm_supported(int s, int t) {
    if (s < 1 || s > EMU_MAX_SLICES) return false;
    if (t == s + 1) return true;
    if (t == 2 * s && s <= 5) return true;
    return false;
}

static bool split_available(int s, int t) { return t == s + 1 && s >= 3; }

// How a product of depth k is cut: 0 chunks = one pass (split tells the
// variant); otherwise nchunks partial passes of chunk_kb K-blocks.
struct Plan {
    bool split = false;
    int nchunks = 0;
    int chunk_kb = 0;
    int plain_kb = 0;     // longest exact K (in blocks) of one plain pass
};

static Plan plan_for(int k, int s, int t) {
    Plan pl;
    const long long KB = (k + K_BLOCK - 1) / K_BLOCK;
    const long long plain = exact_len(max_slot_pairs(s, t, false)) / K_BLOCK;
    pl.plain_kb = (int)plain;
    if (KB <= plain) return pl;
    if (split_available(s, t)) {
        const long long sp = exact_len(max_slot_pairs(s, t, true)) / K_BLOCK;
        if (KB <= sp) {
            pl.split = true;
            return pl;
        }
    }
    pl.chunk_kb = (int)plain;
    pl.nchunks = (int)((KB + plain - 1) / plain);
    return pl;
}

size_t gemm_chunk_bytes(int m, int n, int k, int s, int t, bool raw_sums) {
    Plan pl = plan_for(k, s, t);
    if (pl.nchunks == 0 && !raw_sums) return 0;
    const int KB = (k + K_BLOCK - 1) / K_BLOCK;
    const int nchunks = (KB + pl.plain_kb - 1) / pl.plain_kb;
    return (size_t)nchunks * (t - 1) * (size_t)m * n * sizeof(int32_t);
}

template <int S, int T, bool SPLIT, int MODE>
static int launch_cfg(const GemmArgs &a0, int nchunks, hipStream_t stream) {
    using CF = Cfg<S, T, SPLIT>;
    GemmArgs a = a0;
    a.tiles_m = (a.M + CF::TM * 32 - 1) / (CF::TM * 32);
    a.tiles_n = (a.N + CF::TN * 32 - 1) / (CF::TN * 32);
    a.map = (t_map == 1 && a.tiles_m % 16 == 0 && a.tiles_n % 16 == 0) ? 1 : 0;
    dim3 grid((unsigned)(a.tiles_m * a.tiles_n), MODE == 2 ? nchunks : 1);
    hipLaunchKernelGGL((k_slicegemm<S, T, SPLIT, MODE>), grid, dim3(CF::THREADS), 0,
                       stream, a);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

template <int S, int T>
static int launch_st(const GemmArgs &a, const Plan &pl, int64_t *Dout,
                     hipStream_t stream) {
    if (pl.nchunks == 0 && Dout == nullptr) {
        if constexpr (T == S + 1 && S >= 3) {
            if (pl.split) return launch_cfg<S, T, true, 0>(a, 0, stream);
        }
        return launch_cfg<S, T, false, 0>(a, 0, stream);
    }
    // chunked partial passes of exact INT32 length (also the raw-sum debug
    // path, which always lands in the combine kernel)
    GemmArgs b = a;
    b.chunk_kb = pl.plain_kb;
    const int nchunks = (a.KB + pl.plain_kb - 1) / pl.plain_kb;
    EMU_TRY((launch_cfg<S, T, false, 2>(b, nchunks, stream)));
    const long long MN = (long long)a.M * a.N;
    hipLaunchKernelGGL(k_combine<T>, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0,
                       stream, b, nchunks, Dout);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_slicegemm(const int8_t *Ap, const Planes &ga, const int8_t *Bp,
                     const Planes &gb, const int *codeA, const int *codeB, int m,
                     int n, int k, int s, int t, double alpha, double beta,
                     double *C, long long ldc, int64_t *Dout, int32_t *ws_part,
                     hipStream_t stream, bool lower) {
    if (!gemm_supported(s, t)) {
        set_error("unsupported slice count / threshold (s=%d, t=%d)", s, t);
        return EMU_ERR_UNSUPPORTED;
    }
    Plan pl = plan_for(k, s, t);
    if (lower && (pl.nchunks > 0 || Dout)) {
        set_error("lower-triangle update with chunked K (k=%d) not supported", k);
        return EMU_ERR_UNSUPPORTED;
    }
    if ((pl.nchunks > 0 || Dout) && ws_part == nullptr) {
        set_error("chunk scratch missing");
        return EMU_ERR_WORKSPACE;
    }
    GemmArgs a{};
    a.Ap = Ap;
    a.Bp = Bp;
    a.a_plane = ga.plane_bytes;
    a.b_plane = gb.plane_bytes;
    a.codeA = codeA;
    a.codeB = codeB;
    a.M = m;
    a.N = n;
    a.KB = ga.KB;
    a.alpha = alpha;
    a.beta = beta;
    a.C = C;
    a.ldc = ldc;
    a.part = ws_part;
    a.lower = lower ? 1 : 0;
#define EMU_CASE(S_, T_) \
    if (s == S_ && t == T_) return launch_st<S_, T_>(a, pl, Dout, stream);
    EMU_CASE(1, 2) EMU_CASE(2, 3) EMU_CASE(3, 4) EMU_CASE(4, 5) EMU_CASE(5, 6)
    EMU_CASE(6, 7) EMU_CASE(7, 8) EMU_CASE(8, 9) EMU_CASE(9, 10)
    EMU_CASE(10, 11) EMU_CASE(11, 12) EMU_CASE(12, 13) EMU_CASE(13, 14) EMU_CASE(14, 15)
    EMU_CASE(15, 16) EMU_CASE(16, 17)
    EMU_CASE(2, 4) EMU_CASE(3, 6) EMU_CASE(4, 8) EMU_CASE(5, 10)
#undef EMU_CASE
    set_error("no kernel for s=%d t=%d", s, t);
    return EMU_ERR_UNSUPPORTED;
}

// Unequal splits: A with s slices, B with sb < s, t = s + 1; one pass (no
// K chunks: the longest slot holds sb pairs, so K up to the plain exact
// length of sb pairs needs none).
template <int S, int SB>
static int launch_ab(const GemmArgs &a0, hipStream_t stream) {
    using CF = Cfg<S, S + 1, false, SB>;
    GemmArgs a = a0;
    a.tiles_m = (a.M + CF::TM * 32 - 1) / (CF::TM * 32);
    a.tiles_n = (a.N + CF::TN * 32 - 1) / (CF::TN * 32);
    a.map = (t_map == 1 && a.tiles_m % 16 == 0 && a.tiles_n % 16 == 0) ? 1 : 0;
    hipLaunchKernelGGL((k_slicegemm<S, S + 1, false, 0, SB>), dim3((unsigned)(a.tiles_m * a.tiles_n)),
                       dim3(CF::THREADS), 0, stream, a);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

template <int S, int SB>
static int dispatch_ab(int s, int sb, const GemmArgs &a, hipStream_t stream) {
    if constexpr (S > GROUPED_MAX_SLICES) {
        set_error("unequal splits: s = %d, sb = %d unsupported", s, sb);
        return EMU_ERR_UNSUPPORTED;
    } else if constexpr (SB >= S) {
        return dispatch_ab<S + 1, 1>(s, sb, a, stream);
    } else {
        if (s == S && sb == SB) return launch_ab<S, SB>(a, stream);
        return dispatch_ab<S, SB + 1>(s, sb, a, stream);
    }
}

int launch_slicegemm_ab(const int8_t *Ap, const Planes &ga, const int8_t *Bp, const Planes &gb,
                        const int *codeA, const int *codeB, int m, int n, int k, int s, int sb,
                        double alpha, double beta, double *C, long long ldc, hipStream_t stream) {
    if (s < 2 || s > GROUPED_MAX_SLICES || sb < 1 || sb >= s) {
        set_error("unequal splits: s = %d, sb = %d (need 1 <= sb < s <= %d)", s, sb,
                  GROUPED_MAX_SLICES);
        return EMU_ERR_UNSUPPORTED;
    }
    const long long KB = (k + K_BLOCK - 1) / K_BLOCK;
    if (KB * K_BLOCK > exact_len(max_slot_pairs(s, s + 1, false, sb))) {
        set_error("unequal splits: k = %d exceeds the one-pass exact length", k);
        return EMU_ERR_UNSUPPORTED;
    }
    GemmArgs a{};
    a.Ap = Ap;
    a.Bp = Bp;
    a.a_plane = ga.plane_bytes;
    a.b_plane = gb.plane_bytes;
    a.codeA = codeA;
    a.codeB = codeB;
    a.M = m;
    a.N = n;
    a.KB = ga.KB;
    a.alpha = alpha;
    a.beta = beta;
    a.C = C;
    a.ldc = ldc;
    return dispatch_ab<2, 1>(s, sb, a, stream);
}

void gemm_tile_counts(int s, int m, int n, int *tiles_m, int *tiles_n, int shape) {
    // plain t = s + 1 shapes (Cfg): 128 x 128 tiles while s <= 5, else 64 x 128
    static_assert(Cfg<5, 6, false>::TM * 32 == gemm_tile_rows(5) &&
                      Cfg<6, 7, false>::TM * 32 == gemm_tile_rows(6) &&
                      Cfg<5, 6, false>::TN * 32 == GEMM_TILE_COLS &&
                      Cfg<6, 7, false>::TN * 32 == GEMM_TILE_COLS,
                  "tile shape");
    static_assert(G1Cfg<6, 4>::TM == Cfg<6, 7, false>::TM &&
                      G1Cfg<6, 4>::TN == Cfg<6, 7, false>::TN,
                  "default grouped tile");
    const int tmr = gemm_tile_rows(s);
    const int tnc = (shape == 1 && s >= 6) ? G1Cfg<6, 2>::TN * 32 : GEMM_TILE_COLS;
    *tiles_m = (m + tmr - 1) / tmr;
    *tiles_n = (n + tnc - 1) / tnc;
}

int gemm_grouped_blocks_per_cu(int s, int shape) {
    // LDS per workgroup: stages (4 while s <= 3, else 2) x s digits x
    // (TM + TN) fragments of 1 KB
    const int frags = (s <= 5) ? 8 : (shape == 1 ? 4 : 6);
    const int kb = (s <= 3 ? 4 : 2) * s * frags;
    int b = 160 / (kb > 0 ? kb : 1);
    return b < 1 ? 1 : (b > 2 ? 2 : b);
}

int launch_slicegemm_grouped(const GemmArgs *probs, const int *tile_prefix, int nprob,
                             int total_tiles, int grid, int s, hipStream_t stream,
                             bool one_kstep, int shape) {
    if (total_tiles <= 0 || nprob <= 0) return 0;
    if (grid > total_tiles) grid = total_tiles;
    if (one_kstep && s >= 6 && s <= 9) {
#define EMU_G1CASE(S_)                                                                       \
    case S_:                                                                                 \
        if (shape == 1)                                                                      \
            hipLaunchKernelGGL((k_slicegemm_grouped1<S_, 2>), dim3(grid), dim3(256), 0, stream, \
                               probs, tile_prefix, nprob, total_tiles);                      \
        else                                                                                 \
            hipLaunchKernelGGL((k_slicegemm_grouped1<S_, 4>), dim3(grid), dim3(512), 0, stream, \
                               probs, tile_prefix, nprob, total_tiles);                      \
        break;
        switch (s) {
            EMU_G1CASE(6) EMU_G1CASE(7) EMU_G1CASE(8) EMU_G1CASE(9)
            default:
                break;
        }
#undef EMU_G1CASE
        EMU_TRY_HIP(hipGetLastError());
        return 0;
    }
#define EMU_GCASE(S_)                                                                  \
    case S_:                                                                           \
        hipLaunchKernelGGL((k_slicegemm_grouped<S_, S_ + 1>), dim3(grid), dim3(512), 0, \
                           stream, probs, tile_prefix, nprob, total_tiles, nullptr);   \
        break;
    switch (s) {
        EMU_GCASE(1) EMU_GCASE(2) EMU_GCASE(3) EMU_GCASE(4) EMU_GCASE(5) EMU_GCASE(6)
        EMU_GCASE(7) EMU_GCASE(8) EMU_GCASE(9)
        default:
            set_error("grouped GEMM: slice count %d unsupported", s);
            return EMU_ERR_UNSUPPORTED;
    }
#undef EMU_GCASE
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_slicegemm_grouped_dev(const GemmArgs *probs, const int *tile_prefix,
                                 const int *counts, int grid, int s, hipStream_t stream) {
    if (grid <= 0) return 0;
#define EMU_GCASE(S_)                                                                  \
    case S_:                                                                           \
        hipLaunchKernelGGL((k_slicegemm_grouped<S_, S_ + 1>), dim3(grid), dim3(512), 0, \
                           stream, probs, tile_prefix, 0, 0, counts);                  \
        break;
    switch (s) {
        EMU_GCASE(1) EMU_GCASE(2) EMU_GCASE(3) EMU_GCASE(4) EMU_GCASE(5) EMU_GCASE(6)
        EMU_GCASE(7) EMU_GCASE(8) EMU_GCASE(9)
        default:
            set_error("grouped GEMM: slice count %d unsupported", s);
            return EMU_ERR_UNSUPPORTED;
    }
#undef EMU_GCASE
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

}  // namespace emu
