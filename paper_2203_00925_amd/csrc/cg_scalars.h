// Scalar steps of a CG iteration, shared by the FP64 and FP32-inner solvers:
// one-block kernels that reduce the per-block partials (in index order) and
// update the device-resident scalars.  Templates so that every translation
// unit instantiates its own copy.
#pragma once
#include "reduce.h"
#include "state.h"

namespace mifvm {

// alpha = rz / (p . q)
template <int Unused>
__global__ __launch_bounds__(1024) void k_cg_alpha(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    if (d.scal[SC_DONE] != 0.0) return;
    const double pq = reduce_partials_sum(d.partial, nparts, lds);
    if (threadIdx.x == 0) {
        d.scal[SC_PQ] = pq;
        d.scal[SC_ALPHA] = d.scal[SC_RZ] / pq;
    }
}

// beta = rz_new / rz; count; convergence (1), iteration limit (2) or a
// scheduled restart (3) ends the enqueued chunk.
template <int Unused>
__global__ __launch_bounds__(1024) void k_cg_beta(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    if (d.scal[SC_DONE] != 0.0) return;
    const double trz = reduce_partials_sum(d.partial, nparts, lds);
    const double trr = reduce_partials_sum(d.partial + nparts, nparts, lds);
    if (threadIdx.x == 0) {
        double* sc = d.scal;
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
