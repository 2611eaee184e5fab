// Staging of one vector's values over a tile's halo in LDS, for the
// stored-matrix products (one block per tile of d.tile_rows rows; the
// tile's halo lists every cell and ghost its rows reference, ghosts taking
// the value 0).  Eight index loads per thread go out together, then eight
// value loads, then the LDS writes: two memory latencies per 8T entries
// instead of two per entry.  Slots past the halo read entry 0 and are not
// stored; a ghost reads x[0] and stores 0.
#pragma once

#include "state.h"

namespace mifvm {

template <class V>
__device__ inline void stage_halo_values(const Dev& d, int64_t t, const V* __restrict__ x, V* sp) {
    const int T = blockDim.x;
    const int64_t h0 = d.h_off[t];
    const int hn = int(d.h_off[t + 1] - h0);
    const int64_t nc = d.nc;
    for (int hb = 0; hb < hn; hb += 8 * T) {
        int e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int h = hb + j * T + int(threadIdx.x);
            e[j] = d.h_idx[h0 + (h < hn ? h : 0)];
        }
        V v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = x[e[j] < nc ? e[j] : 0];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int h = hb + j * T + int(threadIdx.x);
            if (h < hn) sp[h] = e[j] < nc ? v[j] : V(0);
        }
    }
}

}  // namespace mifvm
