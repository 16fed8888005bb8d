// Device helpers shared by the FP64 factorization kernels (panel.hip,
// batched.hip): pivot ordering and workgroup-wide pivot search.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>

namespace emu {

// Pivot order (partial pivoting): NaN ranks above every number, otherwise
// the larger magnitude wins, ties go to the smaller row.  It is evaluated
// branch-free on a key: the bit pattern of the magnitude as a signed 64-bit
// integer (monotone in the magnitude for non-negative doubles), every NaN
// mapped to one key above +inf, and -1 for "no candidate".
__device__ __forceinline__ long long pivot_key(double v) {
    const long long b = __double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFll;
    return b > 0x7FF0000000000000ll ? 0x7FF8000000000000ll : b;
}

__device__ __forceinline__ bool key_better(long long ka, int ia, long long kb, int ib) {
    return ka > kb || (ka == kb && ia < ib);
}

// One butterfly level through a DPP lane permutation (CTRL).
template <int CTRL>
__device__ __forceinline__ void key_dpp_step(long long &k, int &i) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)k, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(k >> 32), CTRL, 0xF, 0xF, false);
    const int oi = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
    const long long ok = (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    if (key_better(ok, oi, k, i)) {
        k = ok;
        i = oi;
    }
}

__device__ __forceinline__ void key_xor_step(long long &k, int &i, int off) {
    const long long ok = __shfl_xor(k, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (key_better(ok, oi, k, i)) {
        k = ok;
        i = oi;
    }
}

// Best (key, row) over each aligned group of W lanes (W = 16, 32 or 64);
// every lane of the group receives it.  The first four levels stay inside
// rows of 16 lanes and use DPP (lane ^ 1, lane ^ 2, then the mirrors within
// 8 and 16 lanes, which pair each half with the other once the halves are
// uniform); the levels across rows use lane shuffles.
template <int W>
__device__ __forceinline__ void key_best(long long &k, int &i) {
    key_dpp_step<0xB1>(k, i);                                // quad_perm [1, 0, 3, 2]
    if constexpr (W >= 4) key_dpp_step<0x4E>(k, i);          // quad_perm [2, 3, 0, 1]
    if constexpr (W >= 8) key_dpp_step<0x141>(k, i);         // row_half_mirror
    if constexpr (W >= 16) key_dpp_step<0x140>(k, i);        // row_mirror
    if constexpr (W >= 32) key_xor_step(k, i, 16);
    if constexpr (W >= 64) key_xor_step(k, i, 32);
}

// One level in which only the rows of ROWS (a 4-bit row mask) take a
// partner through the DPP control CTRL; the other rows keep their value.
template <int CTRL, int ROWS>
__device__ __forceinline__ void key_dpp_rows(long long &k, int &i) {
    const int lo = __builtin_amdgcn_update_dpp((int)k, (int)k, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(k >> 32), (int)(k >> 32), CTRL, ROWS, 0xF,
                                               false);
    const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, ROWS, 0xF, false);
    const long long ok = (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    if (key_better(ok, oi, k, i)) {
        k = ok;
        i = oi;
    }
}

// Best (key, row) of the whole wave, returned as wave-uniform values: the
// four levels inside rows of 16 lanes, then lane 15 of rows 0 and 2 joins
// rows 1 and 3 (row_bcast:15) and lane 31 joins rows 2 and 3
// (row_bcast:31), which leaves the wave's best in lane 63.  No lane
// shuffles through LDS.
__device__ __forceinline__ void key_best_wave(long long &k, int &i) {
    key_best<16>(k, i);
    key_dpp_rows<0x142, 0xA>(k, i);
    key_dpp_rows<0x143, 0xC>(k, i);
    const int lo = __builtin_amdgcn_readlane((int)k, 63);
    const int hi = __builtin_amdgcn_readlane((int)(k >> 32), 63);
    i = __builtin_amdgcn_readlane(i, 63);
    k = (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Best (key, row) over a workgroup of NWAVES waves (a power of two up to 16,
// all waves present); every thread gets the result.  One barrier: each wave
// then reduces the NWAVES wave results itself.  red_k / red_i: LDS arrays of
// NWAVES entries, which the caller must not rewrite before a later barrier.
template <int NWAVES>
__device__ __forceinline__ void block_key_best(long long &k, int &i, long long *red_k,
                                               int *red_i) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    key_best<64>(k, i);
    if (lane == 0) {
        red_k[wid] = k;
        red_i[wid] = i;
    }
    __syncthreads();
    k = red_k[lane & (NWAVES - 1)];
    i = red_i[lane & (NWAVES - 1)];
    key_best<NWAVES>(k, i);
}

// v of lane k (k wave-uniform) through two lane reads into scalar
// registers: a few cycles, where a shuffle (ds_bpermute) waits on LDS.
__device__ __forceinline__ double lane_read_f64(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// Composition of w <= 32 row interchanges k <-> p_k (k = 0..w-1 in order,
// p_k >= k; rows relative to the first) by one wave: lane k holds pk = p_k
// (any value for lanes >= w).  The rows they touch, at most 2w, get a lane
// ("slot") each: slots 0..w-1 are rows 0..w-1, the others the distinct
// pivot rows below them in order of first use.  The swaps are replayed on
// the slot contents with lane broadcasts.  Returns the slot count; lane x
// (x < count) gets srow, the row of slot x, and src, the row whose old
// contents end up there.
__device__ __forceinline__ int wave_compose32(int pk, int w, int &srow, int &src) {
    const int lane = threadIdx.x & 63;
    bool first = lane < w && pk >= w;            // first use of a row below the block
    for (int k2 = 0; k2 < w; ++k2) {
        const int pk2 = __builtin_amdgcn_readlane(pk, k2);
        if (k2 < lane && pk2 == pk) first = false;
    }
    const unsigned long long fm = __ballot(first);
    const int nslot = w + __popcll(fm);
    const int myslot = w + __popcll(fm & ((1ull << lane) - 1ull));
    int pslot = pk;                              // slot of row pk
    srow = lane < w ? lane : -1;
    for (int k2 = 0; k2 < w; ++k2) {
        if (!((fm >> k2) & 1ull)) continue;      // uniform
        const int r = __builtin_amdgcn_readlane(pk, k2);
        const int sl = __builtin_amdgcn_readlane(myslot, k2);
        if (lane < w && pk == r) pslot = sl;
        if (lane == sl) srow = r;
    }
    int content = srow;
    for (int k = 0; k < w; ++k) {
        const int b = __builtin_amdgcn_readlane(pslot, k);
        const int va = __builtin_amdgcn_readlane(content, k);
        const int vb = __builtin_amdgcn_readlane(content, b);
        if (lane == k) content = vb;
        if (lane == b) content = va;
    }
    src = content;
    return nslot;
}

}  // namespace emu
