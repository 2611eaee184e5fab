// Deterministic block and grid reductions for wave64.
//
// A block reduces with a butterfly over the 64 lanes of each wavefront (every
// lane ends with the bitwise-identical total, since a+b == b+a) and then sums
// the 4 wavefront totals in a fixed order.  A grid reduction writes one
// partial per block; the last block to finish (device-scope counter) sums the
// partials in index order, so the result does not depend on block timing.
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

__device__ inline double block_min256(double v, double* lds) {
    v = wave_min(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    return fmin(fmin(lds[0], lds[1]), fmin(lds[2], lds[3]));
}

// Publish this block's partial(s) and report whether it is the last block.
// partial[k * nblocks + blockIdx.x] = vals[k] for k < K.
template <int K>
__device__ inline bool publish_partials(const double (&vals)[K], double* partial,
                                        unsigned int* counter) {
    __shared__ bool last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) partial[k * gridDim.x + blockIdx.x] = vals[k];
        __threadfence();
        unsigned int t = atomicAdd(counter, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// In the last block: fixed-order sum of partial[k*nblocks ...].
__device__ inline double sum_partials(const double* partial, int k, double* lds) {
    double s = 0.0;
    for (unsigned int i = threadIdx.x; i < gridDim.x; i += blockDim.x)
        s += __builtin_nontemporal_load(&partial[k * gridDim.x + i]);
    return block_sum256(s, lds);
}

__device__ inline double min_partials(const double* partial, int k, double* lds) {
    double s = __builtin_huge_val();
    for (unsigned int i = threadIdx.x; i < gridDim.x; i += blockDim.x)
        s = fmin(s, __builtin_nontemporal_load(&partial[k * gridDim.x + i]));
    return block_min256(s, lds);
}

}  // namespace mifvm
