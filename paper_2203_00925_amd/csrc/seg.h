// Per-mesh (segmented) reductions for a batch of independent meshes stored
// one after the other in the internal cell numbering.  Every mesh of a batch
// has at least 256 cells, so a block of at most 256 consecutive rows touches
// at most two meshes: the block writes one partial sum for the mesh of its
// first row and one for the mesh of its last row, and a finalize kernel with
// one block per mesh adds its mesh's partials in block order.  With a single
// mesh this is the plain deterministic grid reduction.
#pragma once
#include "reduce.h"
#include "state.h"

namespace mifvm {

__device__ inline int mesh_of(const Dev& d, int64_t row) {
    if (d.nm == 1) return 0;
    int lo = 0, hi = d.nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.mesh_start[mid] <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline double* msc(const Dev& d, int m) { return d.scal + int64_t(m) * SC_COUNT_; }

// Meshes of the rows [r0, r0 + B) of one block: rows below `split` belong
// to m0, the others to m1.
struct BlockSeg {
    int m0, m1;
    int64_t split;
};

__device__ inline BlockSeg block_seg(const Dev& d, int64_t r0, int64_t B) {
    BlockSeg g;
    const int64_t last = (r0 + B < d.nc ? r0 + B : d.nc) - 1;
    g.m0 = mesh_of(d, r0);
    g.m1 = mesh_of(d, last);
    g.split = g.m1 != g.m0 ? d.mesh_start[g.m1] : r0 + B;
    return g;
}

__device__ inline int row_mesh(const BlockSeg& g, int64_t row) { return row < g.split ? g.m0 : g.m1; }

// True when every mesh this block touches has finished its solve.
__device__ inline bool block_done(const Dev& d, const BlockSeg& g) {
    return msc(d, g.m0)[SC_DONE] != 0.0 && msc(d, g.m1)[SC_DONE] != 0.0;
}

// Publish K sums of this block split by mesh: partial[(2k + j) * nblk + b],
// j = 0 for rows of m0 and 1 for rows of m1.  `second` says which side the
// calling thread's row is on.  blockDim.x in {64, 128, 256}.
template <int K>
__device__ inline void seg_publish(const Dev& d, const BlockSeg& g, const double (&v)[K], bool second,
                                   double* lds) {
    const bool two = g.m1 != g.m0;            // uniform over the block
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s0 = block_sum_upto256(second ? 0.0 : v[k], lds);
        const double s1 = two ? block_sum_upto256(second ? v[k] : 0.0, lds) : 0.0;
        if (threadIdx.x == 0) {
            d.partial[(2 * k) * int64_t(gridDim.x) + blockIdx.x] = s0;
            d.partial[(2 * k + 1) * int64_t(gridDim.x) + blockIdx.x] = s1;
        }
    }
}

// As seg_publish, for a block that works on logical block `lb` of `nblk`
// (a kernel whose block order is permuted).
template <int K>
__device__ inline void seg_publish_at(const Dev& d, const BlockSeg& g, const double (&v)[K], bool second,
                                      double* lds, int64_t lb, int64_t nblk) {
    const bool two = g.m1 != g.m0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s0 = block_sum_upto256(second ? 0.0 : v[k], lds);
        const double s1 = two ? block_sum_upto256(second ? v[k] : 0.0, lds) : 0.0;
        if (threadIdx.x == 0) {
            d.partial[(2 * k) * nblk + lb] = s0;
            d.partial[(2 * k + 1) * nblk + lb] = s1;
        }
    }
}

// In the finalize kernel (one 1024-thread block per mesh, blockIdx.x = m):
// the sums of partials k0 .. k0+K-1 of mesh m, produced by a kernel of nblk
// blocks of B rows, each added in block order, in one pass over the
// partials (a thread keeps 16 loads in flight: the finalize is a chain of
// load latencies).  Thread t adds the blocks t, t + 1024, ... in increasing
// order, whatever the batch width, so the sums do not depend on it.
template <int K>
__device__ inline void seg_sums(const Dev& d, int k0, int m, int64_t nblk, int64_t B, double* lds,
                                double (&out)[K]) {
    constexpr int J = K == 1 ? 16 : 8;
    const int64_t lo = d.mesh_start[m], hi = d.mesh_start[m + 1];
    const int64_t first = lo / B, last = (hi - 1) / B;
    double s[K];
#pragma unroll
    for (int q = 0; q < K; ++q) s[q] = 0.0;
    for (int64_t b0 = first + threadIdx.x; b0 <= last; b0 += J * 1024) {
        double v[K][J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t b = b0 + int64_t(j) * 1024;
            const bool in = b <= last;
            const int64_t bb = in ? b : first;
            // a block that starts before the mesh holds it in its second slot
            const int side = bb * B >= lo ? 0 : 1;
#pragma unroll
            for (int q = 0; q < K; ++q) v[q][j] = in ? d.partial[(2 * (k0 + q) + side) * nblk + bb] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int j = 0; j < J; ++j) s[q] += v[q][j];
    }
#pragma unroll
    for (int q = 0; q < K; ++q) out[q] = block_sum1024(s[q], lds);
}

__device__ inline double seg_sum(const Dev& d, int k, int m, int64_t nblk, int64_t B, double* lds) {
    double s[1];
    seg_sums<1>(d, k, m, nblk, B, lds, s);
    return s[0];
}

}  // namespace mifvm
