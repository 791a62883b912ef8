// gf_reduce.hpp -- fixed-order block reductions of the 256-thread
// measurement and bookkeeping kernels (4 wavefronts of 64).
#pragma once

#include <hip/hip_runtime.h>

namespace gfd {

constexpr int MBLOCK = 256;

// sum over a 256-thread block, result valid in thread 0 (fixed order)
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

// maximum over a 256-thread block, result valid in thread 0
__device__ __forceinline__ double block_max(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    return r;
}

}  // namespace gfd
