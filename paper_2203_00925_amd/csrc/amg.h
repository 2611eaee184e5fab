// Aggregation algebraic multigrid for the Poisson system of Sec. 2.2 (eqs.
// (7), (laplace)): the analogue of the paper's fastest solver configuration
// (PETSc GAMG, Sec. 3.4.2), built here as plain (unsmoothed) aggregation.
//
// Setup (host, amg.cpp), per level from the finest:
//   strength  j != i is a strong neighbour of row i when
//             |a_ij| >= theta * max_{k != i} |a_ik|;
//   aggregates three passes in row order: (1) a row whose strong neighbours
//             are all free seeds an aggregate with them; (2) a free row joins
//             the aggregate of its strongest aggregated strong neighbour
//             (smallest index on ties); (3) a row still free seeds an
//             aggregate with its free strong neighbours (or alone);
//   coarse    A_c = P^T A P with the piecewise-constant prolongator P
//             (row i of P is the unit vector of its aggregate);
// until a level has at most coarse_max rows, whose inverse is formed densely
// (LU with partial pivoting).
// The cycle (device, amg_kernels.hip) is a V(1,1) cycle with damped Jacobi
// smoothing from a zero initial guess:
//   x = w D^-1 b;  b_c = P^T (b - A x);  x += P V(b_c);  x += w D^-1 (b - A x),
// with the dense inverse on the coarsest level.
#pragma once
#include <algorithm>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "mesh.h"

namespace mifvm {

// Host threads for the setup's row-parallel passes: up to 16 for n rows of
// at least 65,536, else 1.
inline int setup_threads(int64_t n) {
    const unsigned h = std::thread::hardware_concurrency();
    return n < 65536 ? 1 : int(std::min<unsigned>(16, h ? h : 1));
}

// f(k, lo, hi) for the nt contiguous chunks [lo, hi) of [0, n), chunk k on
// its own thread (chunk 0 on the caller's); every row is handled by exactly
// one call, so results do not depend on nt.
template <class F>
void for_chunks(int64_t n, int nt, F&& f) {
    std::vector<std::thread> th;
    for (int k = 1; k < nt; ++k)
        th.emplace_back([&f, n, nt, k] { f(k, n * k / nt, n * (k + 1) / nt); });
    f(0, 0, n / nt);
    for (auto& t : th) t.join();
}

constexpr int kAmgMaxLevels = 16;

struct AmgCsr {                          // square matrix, diagonal included
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

struct AmgLevel {
    AmgCsr A;
    std::vector<int32_t> agg;             // row -> aggregate (coarse row); empty on the coarsest level
    int64_t ncoarse = 0;
};

struct AmgHierarchy {
    std::vector<AmgLevel> lv;             // lv[0] is the input matrix
    std::vector<double> cinv;             // dense inverse of the coarsest matrix, row-major
    double theta = 0.25, omega = 2.0 / 3.0;
    int gamma = 1;                        // cycle of the device (1 V, 2 W)
    int max_levels = 10;
    int64_t coarse_max = 1024;
};

// Builds the hierarchy of A (moved into lv[0]).  Returns 0 or a negative
// mifvm status; err receives a message.
int amg_build(AmgCsr&& A, double theta, int max_levels, int64_t coarse_max, double omega, AmgHierarchy& H,
              std::string& err);

// 64-row slices of a level's off-diagonal entries (pad: the row itself with
// value 0) and its diagonal, as the device stores them.
void amg_pack(const AmgCsr& A, Sell64& off, std::vector<double>& diag);

}  // namespace mifvm
