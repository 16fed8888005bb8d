// Exponent scan and INT8 digit slicing of one FP64 operand (gfx950).
//
// Paper: section "Emulation of FP64 and INT8 Splitting" (eqns (1)-(3)): the
// operand is split into slices that fit the integer units; eqn (3) shows why
// the scale must follow the magnitude of each row (of A) / column (of B).
//
// Pass 1 (k_scan_*): per-line exponent code = max over the line of the
//   frexp exponent of each element (the exponent of the largest magnitude),
//   with zeros ignored and Inf/NaN dominating; combined across workgroups
//   with atomicMax, since the exponent of a maximum is the maximum of the
//   exponents.
// Pass 2 (k_slice_*): digits by exact integer arithmetic on the significand:
//   with |x| = M 2^E (M the 53-bit significand), Z = floor(|x| 2^(7s - e))
//   is M shifted by E - e + 7s bits (Z < 2^(7s): 64-bit words up to s = 9,
//   128-bit words for s = 10..16), and digit i
//   (1-based) is bits 7(s-i)..7(s-i)+6 of Z with the sign of x.  This equals
//   the truncated base-128 expansion of x 2^-e digit by digit.
// Both passes read the operand once (8 bytes per element each); pass 2
// writes s bytes per element in MFMA fragment order.  For K <= 128 (the
// panels of an LU's trailing updates) one launch does both: each slicing
// wave first takes the exponents of its 32 lines over all of K (reading
// the line K / 32 times in all, from cache), and the wave of the first K
// block stores them; no fill and no scan launch precede it.
#include "common.h"

#include <type_traits>

namespace emu {

__device__ __forceinline__ int exp_code(double x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    int eb = (int)((b >> 52) & 0x7ff);
    unsigned long long fr = b & 0xFFFFFFFFFFFFFull;
    if (eb == 0x7ff) return CODE_NONFINITE;
    if (eb == 0) {
        if (fr == 0) return CODE_ZERO;
        return (63 - __clzll((long long)fr)) - 1073;   // subnormal
    }
    return eb - 1022;
}

// The same code with selects instead of branches, for loops that keep
// several loads in flight before the first code is formed (with branches
// the compiler waits for each load in turn).  Only there: in the grouped
// slicer it lets the compiler hoist all sixteen loads and both address
// forms, and the register count grows threefold.
__device__ __forceinline__ int exp_code_sel(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int eb = (int)((b >> 52) & 0x7ff);
    const unsigned long long fr = b & 0xFFFFFFFFFFFFFull;
    // subnormal: the exponent of the leading fraction bit (fr | 1 has the
    // same leading bit whenever fr != 0)
    const int sub = (63 - __clzll((long long)(fr | 1ull))) - 1073;
    const int fin = eb == 0 ? (fr == 0 ? CODE_ZERO : sub) : eb - 1022;
    return eb == 0x7ff ? CODE_NONFINITE : fin;
}

__device__ __forceinline__ int code_to_exp(int c) {
    return (c == CODE_ZERO || c == CODE_NONFINITE) ? 0 : c;
}

// Z = floor(|x| 2^(7s - e)), sign of x, in 64 bits while 7s <= 63 and in
// 128 bits above (s = 10..16: Z < 2^(7s) <= 2^112).  |x| < 2^e gives
// E - e < -52 for the 53-bit significand M = |x| 2^-E, so the left shift
// below is at most 7s - 53 bits (at most 10 for s <= 9, 59 for s = 16).
template <int S>
using ZWord = typename std::conditional<(S <= 9), unsigned long long, unsigned __int128>::type;

template <int S>
__device__ __forceinline__ ZWord<S> digits_word(double x, int e, int *neg) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    *neg = (int)(b >> 63);
    int eb = (int)((b >> 52) & 0x7ff);
    unsigned long long M = b & 0xFFFFFFFFFFFFFull;
    int E;
    if (eb == 0) {
        E = -1074;
    } else {
        M |= (1ull << 52);
        E = eb - 1075;
    }
    if (M == 0) return 0;
    int sh = E - e + 7 * S;
    if (sh >= 0) return (ZWord<S>)M << sh;   // value < 2^(7S) by choice of e
    if (sh <= -64) return 0;
    return (ZWord<S>)(M >> (-sh));
}

// ------------------------------------------------------------------ scans
__global__ void k_fill_int(int *p, int v, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Rows of X (lines x k, column-major): thread per row, k split over grid.y.
__global__ __launch_bounds__(256) void k_scan_rows(const double *__restrict__ X,
                                                   long long ldx, int lines, int k,
                                                   int kper, int *code, int *status) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= lines) return;
    int k0 = blockIdx.y * kper;
    int k1 = min(k, k0 + kper);
    int m = CODE_ZERO;
    for (int c = k0; c < k1; ++c) m = max(m, exp_code(X[r + (long long)c * ldx]));
    if (m != CODE_ZERO) atomicMax(&code[r], m);
    if (m == CODE_NONFINITE) atomicOr(status, EMU_STATUS_NONFINITE);
}

// Columns of X (k x lines, column-major): one wave per (column, k-chunk).
__global__ __launch_bounds__(256) void k_scan_cols(const double *__restrict__ X,
                                                   long long ldx, int lines, int k,
                                                   int kper, int *code, int *status) {
    int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    int col = wave;
    if (col >= lines) return;
    int k0 = blockIdx.y * kper;
    int k1 = min(k, k0 + kper);
    const double *x = X + (long long)col * ldx;
    int m = CODE_ZERO;
    for (int r = k0 + lane; r < k1; r += 64) m = max(m, exp_code(x[r]));
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if (lane == 0) {
        if (m != CODE_ZERO) atomicMax(&code[col], m);
        if (m == CODE_NONFINITE) atomicOr(status, EMU_STATUS_NONFINITE);
    }
}

// ---------------------------------------------------------------- slicing
// One wave writes fragment block (lb, kb) of every plane.  Lane l handles
// line lb*32 + l%32 and k = kb*32 + (l/32)*16 + 0..15.  Columns of B
// (ROWS = false) are first copied into a wave-private LDS tile with reads
// that run down each column (16 lanes per 256-byte column segment), since
// lanes reading 32 different columns directly would each touch their own
// cache line 16 times.
constexpr int SL_TILE_LD = 33;     // doubles per column of the LDS tile (padded)
template <int S, bool ROWS, bool FUSED>
__global__ __launch_bounds__(256) void k_slice(const double *__restrict__ X,
                                               long long ldx, int lines, int k,
                                               int LB, int KB, int *__restrict__ code,
                                               int8_t *__restrict__ planes,
                                               size_t plane_bytes, int *status) {
    long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (wave >= (long long)LB * KB) return;
    int lb = (int)(wave / KB);
    int kb = (int)(wave % KB);
    int line = lb * 32 + (lane & 31);
    int kbase = kb * 32 + (lane >> 5) * 16;
    int c;
    if constexpr (FUSED) {
        // the exponent code of this lane's line: lanes l and l + 32 share
        // the line and take alternate (rows) or half (columns) of K
        int m = CODE_ZERO;
        if (line < lines) {
            // eight loads in flight per round (a zero stands in past K)
            if constexpr (ROWS) {
                for (int kx0 = lane >> 5; kx0 < k; kx0 += 16) {
                    double xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int kx = kx0 + 2 * u;
                        xv[u] = kx < k ? X[line + (long long)kx * ldx] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) m = max(m, exp_code_sel(xv[u]));
                }
            } else {
                const double *xl = X + (long long)line * ldx;
                const int half = (k + 1) / 2;
                const int k0 = (lane >> 5) * half, k1 = min(k, k0 + half);
                for (int kx0 = k0; kx0 < k1; kx0 += 8) {
                    double xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) xv[u] = kx0 + u < k1 ? xl[kx0 + u] : 0.0;
#pragma unroll
                    for (int u = 0; u < 8; ++u) m = max(m, exp_code_sel(xv[u]));
                }
            }
        }
        c = max(m, __shfl_xor(m, 32, 64));
        if (kb == 0 && lane < 32 && line < lines) {
            code[line] = c;
            if (c == CODE_NONFINITE) atomicOr(status, EMU_STATUS_NONFINITE);
        }
    } else {
        c = line < lines ? code[line] : CODE_ZERO;
    }
    bool ok = line < lines && c != CODE_NONFINITE;
    int e = code_to_exp(c);

    __shared__ double tile[ROWS ? 1 : 4][ROWS ? 1 : 32 * SL_TILE_LD];
    if constexpr (!ROWS) {
        double *tw = tile[(threadIdx.x >> 6) & 3];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int ecol = q * 2 + (lane >> 5);      // column within the block
            const int ek = lane & 31;                  // k within the block
            const int ln = lb * 32 + ecol, kx = kb * 32 + ek;
            tw[ecol * SL_TILE_LD + ek] =
                (ln < lines && kx < k) ? X[kx + (long long)ln * ldx] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    unsigned int w[S][4];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[d][q] = 0u;

#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        int kx = kbase + kk;
        double x = 0.0;
        if (ok && kx < k) {
            if constexpr (ROWS)
                x = X[line + (long long)kx * ldx];
            else
                x = tile[(threadIdx.x >> 6) & 3][(lane & 31) * SL_TILE_LD + (lane >> 5) * 16 + kk];
        }
        int neg;
        const ZWord<S> Z = digits_word<S>(x, e, &neg);
#pragma unroll
        for (int d = 0; d < S; ++d) {
            int q = (int)((Z >> (7 * (S - 1 - d))) & 127u);
            if (neg) q = -q;
            w[d][kk >> 2] |= ((unsigned int)(q & 0xff)) << (8 * (kk & 3));
        }
    }
    size_t off = ((size_t)lb * KB + kb) * FRAG_BYTES + (size_t)lane * 16;
#pragma unroll
    for (int d = 0; d < S; ++d) {
        uint4 v;
        v.x = w[d][0];
        v.y = w[d][1];
        v.z = w[d][2];
        v.w = w[d][3];
        *reinterpret_cast<uint4 *>(planes + d * plane_bytes + off) = v;
    }
}

template <int S, bool FUSED>
static void launch_slice_s(const double *X, long long ldx, int by_rows,
                           const Planes &g, int *code, int8_t *planes, int *status,
                           hipStream_t stream) {
    long long waves = (long long)g.LB * g.KB;
    if (waves == 0) return;
    dim3 grid((unsigned)((waves + 3) / 4));
    if (by_rows)
        hipLaunchKernelGGL((k_slice<S, true, FUSED>), grid, dim3(256), 0, stream, X, ldx,
                           g.lines, g.k, g.LB, g.KB, code, planes, g.plane_bytes, status);
    else
        hipLaunchKernelGGL((k_slice<S, false, FUSED>), grid, dim3(256), 0, stream, X, ldx,
                           g.lines, g.k, g.LB, g.KB, code, planes, g.plane_bytes, status);
}

template <int S>
static void launch_slice_s(const double *X, long long ldx, int by_rows, const Planes &g,
                           int *code, int8_t *planes, int *status, bool fused,
                           hipStream_t stream) {
    if (fused)
        launch_slice_s<S, true>(X, ldx, by_rows, g, code, planes, status, stream);
    else
        launch_slice_s<S, false>(X, ldx, by_rows, g, code, planes, status, stream);
}

// K up to which one launch scans and slices (each wave rereads its lines)
constexpr int FUSED_MAX_K = 128;

int launch_fill_int(int *p, int v, int count, hipStream_t stream) {
    if (count <= 0) return 0;
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, stream,
                       p, v, count);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_slice(const double *X, long long ldx, int by_rows, const Planes &g,
                 int s, int *code, int8_t *planes, int *status,
                 hipStream_t stream) {
    if (s < 1 || s > EMU_MAX_SLICES) {
        set_error("slice count %d outside 1..%d", s, EMU_MAX_SLICES);
        return EMU_ERR_UNSUPPORTED;
    }
    const bool fused = g.k > 0 && g.k <= FUSED_MAX_K;
    if (!fused) EMU_TRY(launch_fill_int(code, CODE_ZERO, g.lines, stream));
    if (!fused && g.k > 0 && g.lines > 0) {
        if (by_rows) {
            // enough workgroups to cover the chip when the panel is narrow
            // (an LU's L21 has k = nb): split k so that about 2048
            // workgroups run, at least 8 columns each
            const int gx = (g.lines + 255) / 256;
            int gy = (2048 + gx - 1) / gx;
            const int gy_max = (g.k + 7) / 8;
            if (gy > gy_max) gy = gy_max;
            if (gy < 1) gy = 1;
            const int kper = (g.k + gy - 1) / gy;
            dim3 grid(gx, (g.k + kper - 1) / kper);
            hipLaunchKernelGGL(k_scan_rows, grid, dim3(256), 0, stream, X, ldx,
                               g.lines, g.k, kper, code, status);
        } else {
            int kper = 2048;
            dim3 grid((g.lines + 3) / 4, (g.k + kper - 1) / kper);
            hipLaunchKernelGGL(k_scan_cols, grid, dim3(256), 0, stream, X, ldx,
                               g.lines, g.k, kper, code, status);
        }
        EMU_TRY_HIP(hipGetLastError());
    }
    switch (s) {
        case 1: launch_slice_s<1>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 2: launch_slice_s<2>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 3: launch_slice_s<3>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 4: launch_slice_s<4>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 5: launch_slice_s<5>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 6: launch_slice_s<6>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 7: launch_slice_s<7>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 8: launch_slice_s<8>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 9: launch_slice_s<9>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 10: launch_slice_s<10>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 11: launch_slice_s<11>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 12: launch_slice_s<12>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 13: launch_slice_s<13>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 14: launch_slice_s<14>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 15: launch_slice_s<15>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        case 16: launch_slice_s<16>(X, ldx, by_rows, g, code, planes, status, fused, stream); break;
        default:
            set_error("slice count %d outside 1..%d", s, EMU_MAX_SLICES);
            return EMU_ERR_UNSUPPORTED;
    }
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ------------------------------------------------ grouped, K <= 32
// One wave per 32-line block of one job: lane l holds line l%32 and the
// k-half l/32; the two lanes of a line exchange their maxima, so exponent
// and digits come from one read of the operand.
template <int S>
__global__ __launch_bounds__(256) void k_slice_small_grouped(const SliceJob *__restrict__ jobs,
                                                             const int *__restrict__ prefix,
                                                             int nj, int total, int *status) {
    const int wave = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= total) return;
    const int lo = __builtin_amdgcn_readfirstlane(wave_search(prefix, nj, wave));
    const SliceJob J = jobs[lo];
    const int lb = wave - prefix[lo];
    const int line = lb * 32 + (lane & 31);
    const int kbase = (lane >> 5) * 16;
    const bool ok = line < J.lines;
    double x[16];
    int code = CODE_ZERO;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        const int kx = kbase + kk;
        x[kk] = 0.0;
        if (ok && kx < J.k)
            x[kk] = J.by_rows ? J.X[line + (long long)kx * J.ldx] : J.X[kx + (long long)line * J.ldx];
        code = max(code, exp_code(x[kk]));
    }
    code = max(code, __shfl_xor(code, 32, 64));
    if (ok && lane < 32) J.code[line] = code;
    if (code == CODE_NONFINITE && lane < 32 && ok) atomicOr(status, EMU_STATUS_NONFINITE);
    const int e = code_to_exp(code);
    const bool good = ok && code != CODE_NONFINITE;
    unsigned int w[S][4];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[d][q] = 0u;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        int neg;
        const ZWord<S> Z = digits_word<S>(good ? x[kk] : 0.0, e, &neg);
#pragma unroll
        for (int d = 0; d < S; ++d) {
            int q = (int)((Z >> (7 * (S - 1 - d))) & 127u);
            if (neg) q = -q;
            w[d][kk >> 2] |= ((unsigned int)(q & 0xff)) << (8 * (kk & 3));
        }
    }
    const size_t off = (size_t)lb * FRAG_BYTES + (size_t)lane * 16;
#pragma unroll
    for (int d = 0; d < S; ++d) {
        uint4 v;
        v.x = w[d][0];
        v.y = w[d][1];
        v.z = w[d][2];
        v.w = w[d][3];
        *reinterpret_cast<uint4 *>(J.planes + d * J.plane_bytes + off) = v;
    }
}

int launch_slice_small_grouped(const SliceJob *jobs, const int *wave_prefix, int nj,
                               int total_waves, int s, int *status, hipStream_t stream) {
    if (total_waves <= 0 || nj <= 0) return 0;
    dim3 grid((unsigned)((total_waves + 3) / 4));
#define EMU_SCASE(S_)                                                                   \
    case S_:                                                                            \
        hipLaunchKernelGGL(k_slice_small_grouped<S_>, grid, dim3(256), 0, stream, jobs,  \
                           wave_prefix, nj, total_waves, status);                       \
        break;
    switch (s) {
        EMU_SCASE(1) EMU_SCASE(2) EMU_SCASE(3) EMU_SCASE(4) EMU_SCASE(5) EMU_SCASE(6)
        EMU_SCASE(7) EMU_SCASE(8) EMU_SCASE(9)
        default:
            set_error("grouped slicing: slice count %d unsupported", s);
            return EMU_ERR_UNSUPPORTED;
    }
#undef EMU_SCASE
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

// ------------------------------------------------------------ debug views
__global__ void k_unpack(const int8_t *__restrict__ planes, int lines, int k, int LB,
                         int KB, size_t plane_bytes, int s, int by_rows,
                         int8_t *__restrict__ out) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)lines * k;
    if (idx >= total) return;
    // output is column-major in the operand's own orientation
    int line, kk;
    if (by_rows) {
        line = (int)(idx % lines);
        kk = (int)(idx / lines);
    } else {
        kk = (int)(idx % k);
        line = (int)(idx / k);
    }
    int lb = line / 32, kb = kk / 32;
    int kh = (kk % 32) / 16;
    size_t off = ((size_t)lb * KB + kb) * FRAG_BYTES +
                 (size_t)(kh * 32 + line % 32) * 16 + (kk % 16);
    for (int d = 0; d < s; ++d) out[d * total + idx] = planes[d * plane_bytes + off];
}

__global__ void k_codes_to_exps(const int *code, int lines, int *exps, int *nonfinite) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= lines) return;
    int c = code[i];
    exps[i] = code_to_exp(c);
    if (nonfinite) nonfinite[i] = (c == CODE_NONFINITE) ? 1 : 0;
}

int launch_unpack(const int8_t *planes, const Planes &g, int s, int by_rows,
                  int8_t *out, hipStream_t stream) {
    long long total = (long long)g.lines * g.k;
    if (total == 0) return 0;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       stream, planes, g.lines, g.k, g.LB, g.KB, g.plane_bytes, s,
                       by_rows, out);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_codes_to_exps(const int *code, int lines, int *exps, int *nonfinite,
                         hipStream_t stream) {
    if (lines <= 0) return 0;
    hipLaunchKernelGGL(k_codes_to_exps, dim3((lines + 255) / 256), dim3(256), 0,
                       stream, code, lines, exps, nonfinite);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

}  // namespace emu
