// Device form of the aggregation multigrid hierarchy (amg.h) and the
// launchers of its cycle and flexible CG (amg_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

#include "amg.h"
#include "state.h"

namespace mifvm {

struct AmgLevelDev {
    int64_t n = 0;
    // level >= 1: off-diagonal entries in 64-row slices, diagonal, inverse diagonal
    int64_t* off = nullptr;
    int32_t* w = nullptr;
    int32_t* idx = nullptr;
    double* val = nullptr;
    double* diag = nullptr;
    double* dinv = nullptr;
    // every level but the coarsest: row -> aggregate, and the members of each
    // aggregate (CSR over the next level's rows)
    int32_t* agg = nullptr;
    int64_t* mptr = nullptr;
    int32_t* midx = nullptr;
    // level >= 1: right-hand side, iterate, product; the W-cycle's second
    // visit: its right-hand side (residual) and correction
    double *b = nullptr, *x = nullptr, *t = nullptr, *r = nullptr, *e = nullptr;
};

struct AmgDev {
    int nl = 0;
    double omega = 2.0 / 3.0;
    int gamma = 1;                    // coarse visits per level: 1 V-cycle, 2 W-cycle
    AmgLevelDev lv[kAmgMaxLevels];
    double* cinv = nullptr;           // dense inverse of the coarsest matrix, row-major
    double* r_old = nullptr;          // flexible CG [nc]
    double *s0 = nullptr, *s1 = nullptr;   // finest-level scratch of a learned smoother [nc]
};

// out = M(in) on the finest level: a learned smoother replacing the Jacobi
// sweeps there (null: Jacobi)
using AmgSmoother = std::function<hipError_t(const double* in, double* out, hipStream_t s)>;

// x0 = V(b0) on the state's system (level 0: K's diagonal and the
// matrix-free product with the potential's conditions); flag: skip when set
hipError_t launch_amg_cycle(const Dev& d, const BcTable& bc_pot, const AmgDev& a, const double* b0, double* x0,
                            const double* flag, hipStream_t s, const AmgSmoother* fine = nullptr);
// open (or reopen) the flexible CG: r = b - K x, the convergence tests,
// z = V(r), p = z, rz
hipError_t launch_amg_open(const Dev& d, const BcTable& bc_pot, const AmgDev& a, double tol, int maxit,
                           int restart, bool fresh, hipStream_t s, const AmgSmoother* fine = nullptr);
// one iteration: q = K p (matrix-free or stored), x, r, the tests, z = V(r),
// Polak-Ribiere beta, p = z + beta p
hipError_t launch_amg_iteration(const Dev& d, const BcTable& bc_pot, const AmgDev& a, bool matrix_free,
                                hipStream_t s, const AmgSmoother* fine = nullptr);

}  // namespace mifvm
