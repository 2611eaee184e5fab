// Scalar steps of a CG iteration, shared by the FP64 and FP32-inner solvers:
// one 1024-thread block per mesh reduces that mesh's partial sums (in block
// order) and updates its device-resident scalars.  Templates so that every
// translation unit instantiates its own copy.
#pragma once
#include "seg.h"
#include "state.h"

namespace mifvm {

// alpha = rz / (p . q)
template <int Unused>
__global__ __launch_bounds__(1024) void k_cg_alpha(Dev d, int64_t nparts, int64_t rows_per_block) {
    __shared__ double lds[16];
    const int m = blockIdx.x;
    double* sc = msc(d, m);
    if (sc[SC_DONE] != 0.0) return;
    const double pq = seg_sum(d, 0, m, nparts, rows_per_block, lds);
    if (threadIdx.x == 0) {
        sc[SC_PQ] = pq;
        sc[SC_ALPHA] = sc[SC_RZ] / pq;
    }
}

// beta = rz_new / rz; count; convergence (1), iteration limit (2) or a
// scheduled restart (3) ends this mesh's part of the enqueued chunk.
template <int Unused>
__global__ __launch_bounds__(1024) void k_cg_beta(Dev d, int64_t nparts, int64_t rows_per_block) {
    __shared__ double lds[16];
    const int m = blockIdx.x;
    double* sc = msc(d, m);
    if (sc[SC_DONE] != 0.0) return;
    double t[2];
    seg_sums<2>(d, 0, m, nparts, rows_per_block, lds, t);
    const double trz = t[0], trr = t[1];
    if (threadIdx.x == 0) {
        sc[SC_BETA] = trz / sc[SC_RZ];
        sc[SC_RZ] = trz;
        sc[SC_RR] = trr;
        sc[SC_IT] = sc[SC_IT] + 1.0;
        sc[SC_SINCE] = sc[SC_SINCE] + 1.0;
        if (trr <= sc[SC_TOL2BB]) sc[SC_DONE] = 1.0;
        else if (sc[SC_IT] >= sc[SC_MAXIT]) sc[SC_DONE] = 2.0;
        else if (sc[SC_RESTART] > 0.0 && sc[SC_SINCE] >= sc[SC_RESTART]) sc[SC_DONE] = 3.0;
    }
}

}  // namespace mifvm
