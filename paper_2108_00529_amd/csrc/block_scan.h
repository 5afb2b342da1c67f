// Deterministic wavefront / workgroup scans shared by several kernels.
#pragma once
#include "common.h"

namespace bgv {

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive block scan of one value per thread; returns the exclusive prefix and
// the block total in *total.  blockDim.x must be a multiple of 64, <= 1024.  The
// combination order depends only on the thread index (deterministic for FP types).
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T *total) {
    __shared__ T wsum[17];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    T incl = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        T x = lane < nw ? wsum[lane] : T(0);
        T xi = wave_incl_scan(x);
        if (lane < nw) wsum[lane] = xi - x;
        if (lane == nw - 1) wsum[16] = xi;
    }
    __syncthreads();
    T res = (incl - v) + wsum[w];
    *total = wsum[16];
    __syncthreads();
    return res;
}

}  // namespace bgv
