// INT8 slice-product GEMM on gfx950 MFMA with the FP64 recombination fused
// into its epilogue.
//
// Paper: section "Emulation of FP64 and INT8 Splitting", eqn (2) and the
// truncation threshold t; the Schur update of eqn (8) is the call site in
// the LU.  For every output element the kernel forms the exact diagonal sums
// D_g = sum_{i+j=g} A_i B_j, g = 2..t, with one INT32 accumulator tile per
// diagonal, loading each digit fragment once per K step and reusing it for
// every pair on every diagonal it takes part in.
//
// Exactness: |D_g| over a K-range of length L is at most pairs(g) L 127^2.
// The host picks a chunk length (a multiple of 32) that keeps this below
// 2^31 for the diagonal with the most pairs; longer K are split into chunks
// whose INT32 sums are folded into an INT64 scratch tile owned by the
// workgroup.  Chunking depends on (s, t, k) only, so tile shapes never
// change a bit of the result.
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

template <int S, int T>
struct Diag {
    static constexpr int NACC = T - 1;                       // diagonals 2..T
    static constexpr int pairs(int g) {
        int lo = g - S > 1 ? g - S : 1;
        int hi = g - 1 < S ? g - 1 : S;
        return hi >= lo ? hi - lo + 1 : 0;
    }
    static constexpr int max_pairs() {
        int m = 0;
        for (int g = 2; g <= T; ++g) m = pairs(g) > m ? pairs(g) : m;
        return m;
    }
};

// Largest multiple of 32 such that max_pairs * L * 127^2 <= 2^31 - 1.
static int chunk_len(int s, int t) {
    int lo_pairs = 0;
    for (int g = 2; g <= t; ++g) {
        int lo = g - s > 1 ? g - s : 1;
        int hi = g - 1 < s ? g - 1 : s;
        if (hi - lo + 1 > lo_pairs) lo_pairs = hi - lo + 1;
    }
    long long L = 2147483647LL / ((long long)lo_pairs * 127 * 127);
    return (int)(L / 32 * 32);
}

constexpr int WG_M = 64;   // workgroup tile: 64 rows x 64 columns of C
constexpr int WG_N = 64;

// MODE 0: recombine into C.  MODE 1: write D_g (int64) to Dout.
// CHUNKED: K is longer than one exactness chunk (separate instantiation so
// that the common case carries no INT64 bookkeeping in its registers).
template <int S, int T, int MODE, bool CHUNKED>
__global__ __launch_bounds__(256) void k_slicegemm(
    const int8_t *__restrict__ Ap, size_t a_plane, int a_KB,
    const int8_t *__restrict__ Bp, size_t b_plane, int b_KB,
    const int *__restrict__ codeA, const int *__restrict__ codeB, int M, int N,
    int KB, int chunk_blocks, double alpha, double beta, double *__restrict__ C,
    long long ldc, int64_t *__restrict__ Dout, int64_t *__restrict__ ws) {
    constexpr int NACC = Diag<S, T>::NACC;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int mb = blockIdx.x * 2 + (w & 1);    // 32-row block of C / A lines
    const int nbk = blockIdx.y * 2 + (w >> 1);  // 32-column block of C / B lines

    v16i acc[NACC];
#pragma unroll
    for (int g = 0; g < NACC; ++g)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[g][r] = 0;

    const int8_t *pa = Ap + (size_t)mb * a_KB * FRAG_BYTES + (size_t)lane * 16;
    const int8_t *pb = Bp + (size_t)nbk * b_KB * FRAG_BYTES + (size_t)lane * 16;
    constexpr bool chunked = CHUNKED;
    int64_t *wsp = nullptr;
    if (chunked) {
        size_t tile = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        wsp = ws + ((tile * 4 + w) * NACC) * 16 * 64 + lane;
    }

    for (int kb = 0; kb < KB; ++kb) {
        v4i a[S], b[S];
#pragma unroll
        for (int d = 0; d < S; ++d)
            a[d] = *reinterpret_cast<const v4i *>(pa + d * a_plane + (size_t)kb * FRAG_BYTES);
#pragma unroll
        for (int d = 0; d < S; ++d)
            b[d] = *reinterpret_cast<const v4i *>(pb + d * b_plane + (size_t)kb * FRAG_BYTES);
#pragma unroll
        for (int i = 1; i <= S; ++i)
#pragma unroll
            for (int j = 1; j <= S; ++j)
                if (i + j <= T)
                    acc[i + j - 2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                        b[j - 1], a[i - 1], acc[i + j - 2], 0, 0, 0);
        if (chunked && (kb % chunk_blocks) == chunk_blocks - 1 && kb != KB - 1) {
            const bool first = kb == chunk_blocks - 1;
#pragma unroll
            for (int g = 0; g < NACC; ++g)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    int64_t *p = wsp + (g * 16 + r) * 64;
                    *p = (first ? 0 : *p) + (int64_t)acc[g][r];
                    acc[g][r] = 0;
                }
        }
    }

    const int m = mb * 32 + (lane & 31);
    if (m >= M) return;
    int ca = codeA[m];
    const bool badA = ca == CODE_NONFINITE;
    const int ea = (ca == CODE_ZERO || badA) ? 0 : ca;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int n = nbk * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (n >= N) continue;
        int64_t D[NACC];
#pragma unroll
        for (int g = 0; g < NACC; ++g) {
            D[g] = (int64_t)acc[g][r];
            if (chunked) D[g] += wsp[(g * 16 + r) * 64];
        }
        if (MODE == 1) {
#pragma unroll
            for (int g = 0; g < NACC; ++g)
                Dout[((size_t)g * N + n) * M + m] = D[g];
        } else {
            const int cb = codeB[n];
            const bool badB = cb == CODE_NONFINITE;
            const int eb = (cb == CODE_ZERO || badB) ? 0 : cb;
            double Ssum = 0.0;
#pragma unroll
            for (int g = NACC - 1; g >= 0; --g) {
                // weight 2^-7(g+2), exact power of two
                const double wgt = __longlong_as_double(
                    (long long)(1023 - 7 * (g + 2)) << 52);
                Ssum = Ssum + (double)D[g] * wgt;
            }
            const double X = ldexp(Ssum, ea + eb);
            double *pc = C + (size_t)n * ldc + m;
            double out = (beta == 0.0) ? fma(alpha, X, 0.0) : fma(alpha, X, beta * *pc);
            if (badA || badB) out = __builtin_nan("");
            *pc = out;
        }
    }
}

bool gemm_supported(int s, int t) {
    if (s < 1 || s > EMU_MAX_SLICES) return false;
    if (t == s + 1) return true;
    if (t == 2 * s && s <= 5) return true;
    return false;
}

size_t gemm_chunk_bytes(int m, int n, int k, int s, int t) {
    int L = chunk_len(s, t);
    int KB = (k + K_BLOCK - 1) / K_BLOCK;
    if (KB <= L / K_BLOCK) return 0;
    size_t tiles = (size_t)((m + WG_M - 1) / WG_M) * ((n + WG_N - 1) / WG_N);
    return tiles * 4 * (size_t)(t - 1) * 16 * 64 * sizeof(int64_t);
}

template <int S, int T>
static void launch_st(const int8_t *Ap, const Planes &ga, const int8_t *Bp,
                      const Planes &gb, const int *codeA, const int *codeB, int m,
                      int n, int KB, int chunk_blocks, double alpha, double beta,
                      double *C, long long ldc, int64_t *Dout, int64_t *ws,
                      hipStream_t stream) {
    dim3 grid((m + WG_M - 1) / WG_M, (n + WG_N - 1) / WG_N);
    const bool chunked = chunk_blocks < KB;
#define EMU_LAUNCH(MODE_, CH_)                                                      \
    hipLaunchKernelGGL((k_slicegemm<S, T, MODE_, CH_>), grid, dim3(256), 0, stream, Ap, \
                       ga.plane_bytes, ga.KB, Bp, gb.plane_bytes, gb.KB, codeA, codeB, \
                       m, n, KB, chunk_blocks, alpha, beta, C, ldc, Dout, ws)
    if (Dout) {
        if (chunked) EMU_LAUNCH(1, true); else EMU_LAUNCH(1, false);
    } else {
        if (chunked) EMU_LAUNCH(0, true); else EMU_LAUNCH(0, false);
    }
#undef EMU_LAUNCH
}

int launch_slicegemm(const int8_t *Ap, const Planes &ga, const int8_t *Bp,
                     const Planes &gb, const int *codeA, const int *codeB, int m,
                     int n, int k, int s, int t, double alpha, double beta,
                     double *C, long long ldc, int64_t *Dout, int64_t *ws_chunk,
                     hipStream_t stream) {
    if (!gemm_supported(s, t)) {
        set_error("unsupported slice count / threshold (s=%d, t=%d)", s, t);
        return EMU_ERR_UNSUPPORTED;
    }
    const int KB = (k + K_BLOCK - 1) / K_BLOCK;
    const int chunk_blocks = chunk_len(s, t) / K_BLOCK;
    if (chunk_blocks < KB && ws_chunk == nullptr) {
        set_error("K-chunk scratch missing");
        return EMU_ERR_WORKSPACE;
    }
#define EMU_CASE(S_, T_)                                                          \
    if (s == S_ && t == T_) {                                                     \
        launch_st<S_, T_>(Ap, ga, Bp, gb, codeA, codeB, m, n, KB, chunk_blocks,    \
                          alpha, beta, C, ldc, Dout, ws_chunk, stream);           \
    } else
    EMU_CASE(1, 2) EMU_CASE(2, 3) EMU_CASE(3, 4) EMU_CASE(4, 5) EMU_CASE(5, 6)
    EMU_CASE(6, 7) EMU_CASE(7, 8) EMU_CASE(8, 9) EMU_CASE(9, 10)
    EMU_CASE(2, 4) EMU_CASE(3, 6) EMU_CASE(4, 8) EMU_CASE(5, 10)
    {
        set_error("no kernel for s=%d t=%d", s, t);
        return EMU_ERR_UNSUPPORTED;
    }
#undef EMU_CASE
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

}  // namespace emu
