// Device helpers shared by the FP64 factorization kernels (panel.hip,
// batched.hip): pivot ordering and workgroup-wide pivot search.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>

namespace emu {

// Pivot order: NaN ranks above every number; otherwise larger magnitude
// wins; ties go to the smaller row index.
__device__ __forceinline__ bool better(double va, int ia, double vb, int ib) {
    bool na = va != va, nb = vb != vb;
    if (na || nb) {
        if (na && nb) return ia < ib;
        return na;
    }
    if (va != vb) return va > vb;
    return ia < ib;
}

__device__ __forceinline__ void wave_best(double &v, int &i) {
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(v, off, 64);
        int oi = __shfl_xor(i, off, 64);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
}

// Best (value, row) over the workgroup; every thread gets the result.
// red_v/red_i: LDS arrays of at least nwaves + 1 entries.
template <int NWAVES>
__device__ __forceinline__ void block_best(double &v, int &i, double *red_v, int *red_i) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_best(v, i);
    if (lane == 0) {
        red_v[wid] = v;
        red_i[wid] = i;
    }
    __syncthreads();
    if (wid == 0) {
        double bv = lane < NWAVES ? red_v[lane] : -1.0;
        int bi = lane < NWAVES ? red_i[lane] : INT_MAX;
        wave_best(bv, bi);
        if (lane == 0) {
            red_v[NWAVES] = bv;
            red_i[NWAVES] = bi;
        }
    }
    __syncthreads();
    v = red_v[NWAVES];
    i = red_i[NWAVES];
}

}  // namespace emu
