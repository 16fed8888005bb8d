// Learned slice count: exponent-spread features of the update's operands,
// a small MLP (16 -> 64 -> 64 -> 7, FP32, ReLU, softmax over s = 3..9) with
// hand-written forward, backward and Adam kernels, tile labels produced by
// the emulator itself, and an LU whose Schur updates use a per-tile slice
// count (this form is not in the paper; its motivating observation is the
// paper's: the digits an element loses depend on how far its exponent sits
// below the largest one of its row or column, eqn (3)).
//
// Features of the 256 x 256 tile (I, J) of the update C = L21 U12, over the
// nonzero elements of L21's rows I (exponent relative to the row's largest)
// and of U12's columns J (relative to the column's largest): rho <= 0;
// features = [min rho, max rho, mean rho, std rho, 12 fractions of -rho in
// bins [0,7), [7,14), ..., [77, inf)].  All statistics are integer sums, so
// the features are reproducible bit for bit.
#include "common.h"

#include <cmath>
#include <vector>

namespace emu {

constexpr int FT = 256;             // feature tile edge
constexpr int NBIN = 12;
constexpr int NFEAT = 16;
constexpr int H = 64;
constexpr int NCLS = 7;             // s = 3..9
constexpr int NPARAM = H * NFEAT + H + H * H + H + NCLS * H + NCLS;   // 5703
// parameter layout: W1[H][NFEAT] b1[H] W2[H][H] b2[H] W3[NCLS][H] b3[NCLS]
constexpr int P_W1 = 0, P_B1 = P_W1 + H * NFEAT, P_W2 = P_B1 + H, P_B2 = P_W2 + H * H,
              P_W3 = P_B2 + H, P_B3 = P_W3 + NCLS * H;

struct Stat {            // integer statistics of rho over one line block
    long long cnt, sum, sumsq;
    int mn, mx;
    int hist[NBIN];
};

__device__ __forceinline__ int fexp(double x) {   // frexp exponent (x != 0, finite)
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int eb = (int)((b >> 52) & 0x7ff);
    const unsigned long long fr = b & 0xFFFFFFFFFFFFFull;
    // subnormal: the exponent of the leading fraction bit (selects, no branch)
    const int sub = (63 - __clzll((long long)(fr | 1ull))) - 1073;
    return eb == 0 ? sub : eb - 1022;
}

__device__ __forceinline__ bool usable(double x) { return x != 0.0 && isfinite(x); }

// Statistics of one block of up to FL = 64 lines of an operand (a feature
// tile's 256 lines are four such blocks, combined exactly when the tile's
// features are formed).  by_rows: lines are rows of X (rows x k), else
// columns of X (k x cols).  Four threads per line, each over a quarter of K
// with eight loads in flight: the line's largest exponent first (combined
// through LDS), then the integer sums.
constexpr int FL = 64;
constexpr int FQ = 4;
static_assert(FT % FL == 0, "line blocks tile a feature tile");
__global__ __launch_bounds__(FL * FQ) void k_feat_lines(const double *__restrict__ X,
                                                        long long ldx, int lines, int k,
                                                        int by_rows, Stat *__restrict__ out) {
    __shared__ long long s_cnt, s_sum, s_sq;
    __shared__ int s_mn, s_mx, s_hist[NBIN];
    __shared__ int s_e[FQ][FL];
    const int t = threadIdx.x, tl = t % FL, qk = t / FL;
    if (t == 0) {
        s_cnt = 0;
        s_sum = 0;
        s_sq = 0;
        s_mn = INT_MAX;
        s_mx = INT_MIN;
    }
    if (t < NBIN) s_hist[t] = 0;
    const int line = blockIdx.x * FL + tl;
    const int kq = (k + FQ - 1) / FQ, k0 = qk * kq, k1 = min(k, k0 + kq);
    auto load8 = [&](int kk0, double (&xv)[8]) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kk = kk0 + u;
            xv[u] = kk < k1 ? (by_rows ? X[line + (long long)kk * ldx]
                                       : X[kk + (long long)line * ldx])
                            : 0.0;
        }
    };
    int e = INT_MIN;
    if (line < lines) {
        for (int kk0 = k0; kk0 < k1; kk0 += 8) {
            double xv[8];
            load8(kk0, xv);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (usable(xv[u])) e = max(e, fexp(xv[u]));
        }
    }
    s_e[qk][tl] = e;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < FQ; ++q) e = max(e, s_e[q][tl]);
    long long cnt = 0, sum = 0, sq = 0;
    int mn = INT_MAX, mx = INT_MIN;
    int hist[NBIN];
#pragma unroll
    for (int b = 0; b < NBIN; ++b) hist[b] = 0;
    if (line < lines) {
        for (int kk0 = k0; kk0 < k1; kk0 += 8) {
            double xv[8];
            load8(kk0, xv);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (!usable(xv[u])) continue;
                const int rho = fexp(xv[u]) - e;
                ++cnt;
                sum += rho;
                sq += (long long)rho * rho;
                mn = min(mn, rho);
                mx = max(mx, rho);
                const int bin = min(NBIN - 1, (-rho) / 7);
#pragma unroll
                for (int b = 0; b < NBIN; ++b)
                    if (b == bin) ++hist[b];
            }
        }
    }
    atomicAdd((unsigned long long *)&s_cnt, (unsigned long long)cnt);
    atomicAdd((unsigned long long *)&s_sum, (unsigned long long)sum);
    atomicAdd((unsigned long long *)&s_sq, (unsigned long long)sq);
    atomicMin(&s_mn, mn);
    atomicMax(&s_mx, mx);
#pragma unroll
    for (int b = 0; b < NBIN; ++b)
        if (hist[b]) atomicAdd(&s_hist[b], hist[b]);
    __syncthreads();
    if (t == 0) {
        Stat &o = out[blockIdx.x];
        o.cnt = s_cnt;
        o.sum = s_sum;
        o.sumsq = s_sq;
        o.mn = s_mn;
        o.mx = s_mx;
        for (int b = 0; b < NBIN; ++b) o.hist[b] = s_hist[b];
    }
}

// Tile (I, J) features from the line blocks of row block I of L21 (m rows)
// and of column block J of U12 (n columns): integer sums, then the floats.
__global__ void k_feat_tiles(const Stat *__restrict__ rs, const Stat *__restrict__ cs, int m,
                             int n, float *__restrict__ feat) {
    const int tiles_m = (m + FT - 1) / FT, tiles_n = (n + FT - 1) / FT;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tiles_m * tiles_n) return;
    const int I = idx % tiles_m, J = idx / tiles_m;
    constexpr int PER = FT / FL;
    const int nr = (m + FL - 1) / FL, nc = (n + FL - 1) / FL;
    long long cnt = 0, sum = 0, sq = 0;
    int mn = INT_MAX, mx = INT_MIN;
    long long hist[NBIN] = {};
    auto take = [&](const Stat &a) {
        cnt += a.cnt;
        sum += a.sum;
        sq += a.sumsq;
        mn = min(mn, a.mn);
        mx = max(mx, a.mx);
        for (int q = 0; q < NBIN; ++q) hist[q] += a.hist[q];
    };
    for (int b = I * PER; b < min(nr, (I + 1) * PER); ++b) take(rs[b]);
    for (int b = J * PER; b < min(nc, (J + 1) * PER); ++b) take(cs[b]);
    float *f = feat + (long long)idx * NFEAT;
    if (cnt == 0) {
        for (int q = 0; q < NFEAT; ++q) f[q] = 0.0f;
        return;
    }
    const double c = (double)cnt;
    const double mean = (double)sum / c;
    const double var = (double)sq / c - mean * mean;
    f[0] = (float)mn;
    f[1] = (float)mx;
    f[2] = (float)mean;
    f[3] = (float)sqrt(var > 0.0 ? var : 0.0);
    for (int q = 0; q < NBIN; ++q) f[4 + q] = (float)((double)hist[q] / c);
}

// ------------------------------------------------------------------- MLP
// Thread per sample, parameters in LDS.  Saves h1, h2 and the deltas
// (feature-major, [unit][B]) for the gradient pass; loss[b] = -log p_label.
__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(const float *__restrict__ params,
                                                     const float *__restrict__ X,
                                                     const int *__restrict__ label, int B,
                                                     float *__restrict__ h1s,
                                                     float *__restrict__ h2s,
                                                     float *__restrict__ d1s,
                                                     float *__restrict__ d2s,
                                                     float *__restrict__ d3s,
                                                     float *__restrict__ prob,
                                                     float *__restrict__ loss) {
    __shared__ float P[NPARAM];
    for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) P[e] = params[e];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float x[NFEAT];
#pragma unroll
    for (int q = 0; q < NFEAT; ++q) x[q] = X[(long long)b * NFEAT + q];
    float h1[H], h2[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float a = P[P_B1 + i];
#pragma unroll
        for (int q = 0; q < NFEAT; ++q) a = fmaf(P[P_W1 + i * NFEAT + q], x[q], a);
        h1[i] = a > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float a = P[P_B2 + i];
#pragma unroll
        for (int q = 0; q < H; ++q) a = fmaf(P[P_W2 + i * H + q], h1[q], a);
        h2[i] = a > 0.0f ? a : 0.0f;
    }
    float z[NCLS];
    float zmax = -INFINITY;
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
        float a = P[P_B3 + c];
#pragma unroll
        for (int q = 0; q < H; ++q) a = fmaf(P[P_W3 + c * H + q], h2[q], a);
        z[c] = a;
        zmax = fmaxf(zmax, a);
    }
    float den = 0.0f;
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
        z[c] = expf(z[c] - zmax);
        den += z[c];
    }
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
        z[c] = z[c] / den;
        if (prob) prob[(long long)b * NCLS + c] = z[c];
    }
    if (!label) return;
    const int y = label[b];
    float py = 0.0f;
#pragma unroll
    for (int c = 0; c < NCLS; ++c)
        if (c == y) py = z[c];
    loss[b] = -logf(fmaxf(py, 1e-30f));
    // backward: d3 = p - onehot; d2 = (W3^T d3) * relu'(h2); d1 = (W2^T d2) * relu'(h1)
    float d3[NCLS];
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
        d3[c] = z[c] - (c == y ? 1.0f : 0.0f);
        d3s[(long long)c * B + b] = d3[c];
    }
    float d2[H];
#pragma unroll
    for (int q = 0; q < H; ++q) {
        float a = 0.0f;
#pragma unroll
        for (int c = 0; c < NCLS; ++c) a = fmaf(P[P_W3 + c * H + q], d3[c], a);
        d2[q] = h2[q] > 0.0f ? a : 0.0f;
        d2s[(long long)q * B + b] = d2[q];
        h2s[(long long)q * B + b] = h2[q];
    }
#pragma unroll
    for (int q = 0; q < H; ++q) {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < H; ++i) a = fmaf(P[P_W2 + i * H + q], d2[i], a);
        d1s[(long long)q * B + b] = h1[q] > 0.0f ? a : 0.0f;
        h1s[(long long)q * B + b] = h1[q];
    }
}

// Gradient rows, one workgroup each: rows 0..63 of layer 1 (16 weights +
// bias), 64..127 of layer 2 (64 + bias), 128..134 of layer 3 (64 + bias).
// Sums over samples in a fixed order (per-thread strided, then a tree), and
// the mean over the batch.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ X,
                                                  const float *__restrict__ h1s,
                                                  const float *__restrict__ h2s,
                                                  const float *__restrict__ d1s,
                                                  const float *__restrict__ d2s,
                                                  const float *__restrict__ d3s, int B,
                                                  float *__restrict__ grad) {
    __shared__ float red[256];
    const int row = blockIdx.x;
    const float *delta;
    const float *inp;          // [fan_in][B] (layer 1: X is [B][16])
    int fan_in, w_off, b_off, r;
    if (row < H) {
        r = row;
        delta = d1s + (long long)r * B;
        inp = nullptr;
        fan_in = NFEAT;
        w_off = P_W1 + r * NFEAT;
        b_off = P_B1 + r;
    } else if (row < 2 * H) {
        r = row - H;
        delta = d2s + (long long)r * B;
        inp = h1s;
        fan_in = H;
        w_off = P_W2 + r * H;
        b_off = P_B2 + r;
    } else {
        r = row - 2 * H;
        delta = d3s + (long long)r * B;
        inp = h2s;
        fan_in = H;
        w_off = P_W3 + r * H;
        b_off = P_B3 + r;
    }
    const float invB = 1.0f / (float)B;
    for (int j = -1; j < fan_in; ++j) {          // j = -1: the bias
        float acc = 0.0f;
        for (int b = threadIdx.x; b < B; b += blockDim.x) {
            float in = 1.0f;
            if (j >= 0) in = inp ? inp[(long long)j * B + b] : X[(long long)b * NFEAT + j];
            acc = fmaf(delta[b], in, acc);
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) grad[j < 0 ? b_off : w_off + j] = red[0] * invB;
        __syncthreads();
    }
}

__global__ void k_adam(float *__restrict__ params, const float *__restrict__ grad,
                       float *__restrict__ m, float *__restrict__ v, int count, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// s per sample: smallest class whose cumulative probability reaches conf.
__global__ void k_decode(const float *__restrict__ prob, int B, float conf, int *__restrict__ s) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float acc = 0.0f;
    int c = 0;
    for (; c < NCLS - 1; ++c) {
        acc += prob[(long long)b * NCLS + c];
        if (acc >= conf) break;
    }
    s[b] = 3 + c;
}

// ---------------------------------------------------------------- labels
// Per 256 x 256 tile: sum of squares of X_s - X_ref and of X_ref (FP64, fixed
// order); label = smallest s in [s_lo, s_hi] with rel. error <= tau.
__global__ __launch_bounds__(256) void k_tile_err(const double *__restrict__ Xs,
                                                  const double *__restrict__ Xr, long long ld,
                                                  int m, int n, int tiles_m,
                                                  double *__restrict__ err2,
                                                  double *__restrict__ ref2) {
    __shared__ double re[256], rr[256];
    const int I = blockIdx.x % tiles_m, J = blockIdx.x / tiles_m;
    const int i0 = I * FT, j0 = J * FT;
    double e = 0.0, r = 0.0;
    const int i = i0 + threadIdx.x;
    if (i < m)
        for (int j = j0; j < min(n, j0 + FT); ++j) {
            const double a = Xs[i + (long long)j * ld], c = Xr[i + (long long)j * ld];
            e += (a - c) * (a - c);
            r += c * c;
        }
    re[threadIdx.x] = e;
    rr[threadIdx.x] = r;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            re[threadIdx.x] += re[threadIdx.x + s];
            rr[threadIdx.x] += rr[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        err2[blockIdx.x] = re[0];
        ref2[blockIdx.x] = rr[0];
    }
}

__global__ void k_tile_label(const double *__restrict__ err2, const double *__restrict__ ref2,
                             int ntiles, int s, double tau, int *__restrict__ label) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ntiles) return;
    // walking s upward: the first s that passes keeps its label
    if (label[q] < 0 && sqrt(err2[q]) <= tau * sqrt(ref2[q])) label[q] = s;
}

// ------------------------------------------------------------- launchers
int learned_nparam() { return NPARAM; }

// Problem lists of the adaptive update, one per slice count, over the tiles
// of tile columns [jlo, jhi): wave s - 1 walks the tiles in order, 64 at a
// time; a ballot numbers the tiles of count s and a lane scan of their GEMM
// tile counts extends the running prefix.
static_assert(GROUPED_MAX_SLICES == 9, "one wave per slice count");
__global__ __launch_bounds__(9 * 64) void k_adaptive_lists(const int *__restrict__ smap, int nt,
                                                          int s_cap, AdaptiveTiles t, int jlo,
                                                          int jhi, GemmArgs *__restrict__ probs,
                                                          int *__restrict__ prefix,
                                                          int *__restrict__ counts) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, s = w + 1;
    GemmArgs *P = probs + (size_t)w * nt;
    int *pre = prefix + (size_t)w * (nt + 1);
    const int rows = gemm_tile_rows(s);
    int np = 0, tot = 0;
    if (lane == 0) pre[0] = 0;
    for (int q0 = 0; q0 < nt; q0 += 64) {
        const int q = q0 + lane;
        const int sq = q < nt ? min(smap[q], s_cap) : 0;
        const int Jq = q / t.tm;
        const bool match = q < nt && sq == s && Jq >= jlo && Jq < jhi;
        const unsigned long long mask = __ballot(match);
        const int pos = np + __popcll(mask & ((1ull << lane) - 1ull));
        int tc = 0;
        if (match) {
            const int I = q % t.tm, J = q / t.tm;
            GemmArgs a{};
            a.Ap = t.pa + (size_t)I * (FT / 32) * t.KB * FRAG_BYTES;
            a.Bp = t.pb + (size_t)J * (FT / 32) * t.KB * FRAG_BYTES;
            a.a_plane = t.a_plane;
            a.b_plane = t.b_plane;
            a.codeA = t.codeA + I * FT;
            a.codeB = t.codeB + J * FT;
            a.M = min(FT, t.M - I * FT);
            a.N = min(FT, t.N - J * FT);
            a.KB = t.KB;
            a.alpha = -1.0;
            a.beta = 1.0;
            a.C = t.C + I * FT + (long long)J * FT * t.ldc;
            a.ldc = t.ldc;
            a.tiles_m = (a.M + rows - 1) / rows;
            a.tiles_n = (a.N + GEMM_TILE_COLS - 1) / GEMM_TILE_COLS;
            tc = a.tiles_m * a.tiles_n;
            P[pos] = a;
        }
        int x = tc;                                   // inclusive scan over lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (match) pre[pos + 1] = tot + x;
        tot += __shfl(x, 63, 64);
        np += __popcll(mask);
    }
    if (lane == 0) {
        counts[2 * w] = np;
        counts[2 * w + 1] = tot;
    }
}

int launch_adaptive_lists(const int *smap, int nt, int s_cap, const AdaptiveTiles &t, int jlo,
                          int jhi, GemmArgs *probs, int *prefix, int *counts, hipStream_t st) {
    if (nt <= 0) return 0;
    hipLaunchKernelGGL(k_adaptive_lists, dim3(1), dim3(9 * 64), 0, st, smap, nt, s_cap, t, jlo,
                       jhi, probs, prefix, counts);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

size_t feat_stat_bytes(int lines) { return sizeof(Stat) * (size_t)((lines + FL - 1) / FL); }

int launch_feat_lines(const double *X, long long ldx, int lines, int k, int by_rows,
                      void *stats, hipStream_t st) {
    if (lines <= 0) return 0;
    hipLaunchKernelGGL(k_feat_lines, dim3((lines + FL - 1) / FL), dim3(FL * FQ), 0, st, X, ldx,
                       lines, k, by_rows, static_cast<Stat *>(stats));
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_feat_tiles(const void *row_stats, const void *col_stats, int m, int n, float *feat,
                      hipStream_t st) {
    const int nt = ((m + FT - 1) / FT) * ((n + FT - 1) / FT);
    if (nt <= 0) return 0;
    hipLaunchKernelGGL(k_feat_tiles, dim3((nt + 255) / 256), dim3(256), 0, st,
                       static_cast<const Stat *>(row_stats), static_cast<const Stat *>(col_stats),
                       m, n, feat);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_features(const double *L21, long long ldl, const double *U12, long long ldu, int m,
                    int n, int k, float *feat, void *stat_ws, hipStream_t st) {
    char *rs = static_cast<char *>(stat_ws);
    char *cs = rs + feat_stat_bytes(m);
    EMU_TRY(launch_feat_lines(L21, ldl, m, k, 1, rs, st));
    EMU_TRY(launch_feat_lines(U12, ldu, n, k, 0, cs, st));
    return launch_feat_tiles(rs, cs, m, n, feat, st);
}

size_t features_ws_bytes(int m, int n) { return feat_stat_bytes(m) + feat_stat_bytes(n); }

size_t mlp_train_ws_bytes(int B) {
    return sizeof(float) * (size_t)B * (4 * H + NCLS + NCLS + 1) + sizeof(float) * NPARAM;
}

int launch_mlp_train_step(float *params, const float *X, const int *label, int B, float *m,
                          float *v, int step, float lr, void *ws, float *loss_out,
                          hipStream_t st) {
    float *f = static_cast<float *>(ws);
    float *h1 = f, *h2 = h1 + (size_t)H * B, *d1 = h2 + (size_t)H * B, *d2 = d1 + (size_t)H * B;
    float *d3 = d2 + (size_t)H * B, *prob = d3 + (size_t)NCLS * B, *loss = prob + (size_t)NCLS * B;
    float *grad = loss + B;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((B + 255) / 256), dim3(256), 0, st, params, X, label,
                       B, h1, h2, d1, d2, d3, prob, loss);
    hipLaunchKernelGGL(k_mlp_grad, dim3(2 * H + NCLS), dim3(256), 0, st, X, h1, h2, d1, d2, d3,
                       B, grad);
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, params, grad, m, v,
                       NPARAM, lr, b1, b2, 1e-8f, c1, c2);
    if (loss_out) EMU_TRY_HIP(hipMemcpyAsync(loss_out, loss, sizeof(float) * B,
                                             hipMemcpyDeviceToDevice, st));
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_mlp_grad_only(const float *params, const float *X, const int *label, int B,
                         float *grad_out, void *ws, hipStream_t st) {
    float *f = static_cast<float *>(ws);
    float *h1 = f, *h2 = h1 + (size_t)H * B, *d1 = h2 + (size_t)H * B, *d2 = d1 + (size_t)H * B;
    float *d3 = d2 + (size_t)H * B, *prob = d3 + (size_t)NCLS * B, *loss = prob + (size_t)NCLS * B;
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((B + 255) / 256), dim3(256), 0, st, params, X, label,
                       B, h1, h2, d1, d2, d3, prob, loss);
    hipLaunchKernelGGL(k_mlp_grad, dim3(2 * H + NCLS), dim3(256), 0, st, X, h1, h2, d1, d2, d3,
                       B, grad_out);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_mlp_infer(const float *params, const float *X, int B, float *prob, int *s_out,
                     float conf, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((B + 255) / 256), dim3(256), 0, st, params, X,
                       (const int *)nullptr, B, (float *)nullptr, (float *)nullptr,
                       (float *)nullptr, (float *)nullptr, (float *)nullptr, prob,
                       (float *)nullptr);
    if (s_out)
        hipLaunchKernelGGL(k_decode, dim3((B + 255) / 256), dim3(256), 0, st, prob, B, conf,
                           s_out);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_tile_err(const double *Xs, const double *Xr, long long ld, int m, int n,
                    double *err2, double *ref2, hipStream_t st) {
    const int tm = (m + FT - 1) / FT, tn = (n + FT - 1) / FT;
    hipLaunchKernelGGL(k_tile_err, dim3(tm * tn), dim3(256), 0, st, Xs, Xr, ld, m, n, tm, err2,
                       ref2);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

int launch_tile_label(const double *err2, const double *ref2, int ntiles, int s, double tau,
                      int *label, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_label, dim3((ntiles + 255) / 256), dim3(256), 0, st, err2, ref2,
                       ntiles, s, tau, label);
    EMU_TRY_HIP(hipGetLastError());
    return 0;
}

}  // namespace emu
