// Deterministic block and grid reductions for wave64.
//
// A block reduces with a butterfly over the 64 lanes of each wavefront (every
// lane ends with the bitwise-identical total, since a+b == b+a) and then sums
// the wavefront totals in a fixed order.  A grid reduction writes one partial
// per block with a plain store; a separate one-block kernel sums the partials
// in index order.  No device-scope fence is executed per block: on a
// multi-XCD part such a fence writes back the XCD's L2, which costs more than
// the extra kernel launch.
#pragma once
#include <hip/hip_runtime.h>

namespace mifvm {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// blockDim.x == 256 assumed; lds needs 4 doubles.  Result valid in all threads.
__device__ inline double block_sum256(double v, double* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// blockDim.x in {64, 128, 256}; lds needs 4 doubles.  Result valid in all threads.
__device__ inline double block_sum_upto256(double v, double* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = lds[0];
    for (int k = 1; k < nw; ++k) s += lds[k];
    return s;
}

// blockDim.x == 1024 assumed; lds needs 16 doubles.  Result valid in all threads.
__device__ inline double block_sum1024(double v, double* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += lds[k];
    return s;
}

__device__ inline double block_min1024(double v, double* lds) {
    v = wave_min(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = lds[0];
#pragma unroll
    for (int k = 1; k < 16; ++k) s = fmin(s, lds[k]);
    return s;
}

// In a one-block kernel of 1024 threads: fixed-order sum of n partials.
__device__ inline double reduce_partials_sum(const double* partial, int64_t n, double* lds) {
    double s = 0.0;
    // batches of 8 independent loads, summed in index order
    for (int64_t b = threadIdx.x; b < n; b += 8 * 1024) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = b + j * 1024 < n ? partial[b + j * 1024] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    return block_sum1024(s, lds);
}

__device__ inline double reduce_partials_min(const double* partial, int64_t n, double* lds) {
    double s = __builtin_huge_val();
    for (int64_t i = threadIdx.x; i < n; i += 1024) s = fmin(s, partial[i]);
    return block_min1024(s, lds);
}

__device__ inline double block_min256(double v, double* lds) {
    v = wave_min(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    return fmin(fmin(lds[0], lds[1]), fmin(lds[2], lds[3]));
}

}  // namespace mifvm
