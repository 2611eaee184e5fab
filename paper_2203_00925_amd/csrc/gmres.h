// Restarted flexible GMRES(m) with the Jacobi preconditioner: the Krylov
// method of the paper's solver runs (Sec. 3.4.2, PETSc FGMRES with Jacobi),
// on one GPU.  Classical Gram-Schmidt (all dot products of a step against
// the same vector, PETSc's default orthogonalisation), Givens rotations,
// every scalar in device memory.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "state.h"

namespace mifvm {

constexpr int kGmMaxM = 64;
constexpr int kGmGrid = 1024;             // blocks of the grid-stride reduction kernels

struct GmDev {
    int m;
    double* V;          // [m + 1][nc] Arnoldi vectors (V[j + 1] holds w during step j)
    double* Z;          // [m][nc] preconditioned vectors z_j = D^-1 v_j
    double* H;          // [m + 1][m] Hessenberg, rotated in place (column-major: H[j * (m + 1) + i])
    double* cs;         // [m] rotations
    double* sn;
    double* g;          // [m + 1] rotated right-hand side
    double* y;          // [m] least-squares coefficients of the cycle
    double* sc;         // [4] beta, steps done this cycle, 1/h_{j+1,j}, -
    double* partial;    // [m + 1][kGmGrid]
};
enum GmScal { GM_BETA = 0, GM_K = 1, GM_INVH = 2 };

size_t gm_layout(int64_t nc, int m, char* base, GmDev& g);

// r = b - K x (into V[0]) from y_kx = K x (CSR when y_kx is null); opens a
// cycle: beta, g = beta e0, the convergence and limit tests (fresh: also the
// tolerance and limits), then v0 = r / beta, z0 = D^-1 v0
hipError_t launch_gm_open(const Dev& d, const GmDev& g, const double* y_kx, double tol, int maxit, bool fresh,
                          hipStream_t s);
// w = K z_j into V[j + 1] (stored matrix; the matrix-free product is
// launched by the caller), then the orthogonalisation and the rotation
hipError_t launch_gm_spmv(const Dev& d, const GmDev& g, int j, hipStream_t s);
hipError_t launch_gm_orth(const Dev& d, const GmDev& g, int j, hipStream_t s);
// end of cycle: H y = g, x += Z y
hipError_t launch_gm_close(const Dev& d, const GmDev& g, hipStream_t s);

}  // namespace mifvm
