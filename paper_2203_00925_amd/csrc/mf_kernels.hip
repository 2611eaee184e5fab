// Matrix-free application of the Poisson operator of Sec. 2.2 (eqs. (7),
// (laplace)): y = K x evaluated from the discretisation itself instead of
// the stored matrix.  Row i of K is minus the sum over the faces of i of
// s_if dF_f/dP, where on interior and Dirichlet faces
//     F_f = kAC (x_A - x_C) + kBC (x_B - x_C) + kRL (x_R - x_L)     (eq. (diamond))
// with vertex values x_v = sum alpha_{v,e} x_e (Algorithm 2) and a ghost
// entity e = nc + g standing for s_g x_owner (s_g = -1 Dirichlet, +1 else:
// the homogeneous part of the ghost value; its constant goes into c).
// Neumann and zero-flux faces carry a fixed flux, which is constant in x and
// so absent from K.  Three kernels: vertex values (one thread per vertex,
// 64-row slices of the vertex lists), face fluxes (one thread per face), and
// the per-cell gather through the cell->face table, which also writes the
// partial p.q of the conjugate gradient.  About 210 bytes per row move
// against about 730 for the stored 64-row-sliced matrix.
#include "cg_scalars.h"
#include "reduce.h"
#include "seg.h"
#include "state.h"
#include "xcd.h"

namespace mifvm {
namespace {

// ghost values of x (homogeneous part): xg[g] = s_g x_owner
__global__ __launch_bounds__(kBlock) void k_mf_ghost(Dev d, BcTable bc, const double* __restrict__ x,
                                                     double* __restrict__ xg, const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= d.nb) return;
    const double sg = bc.kind[d.gtag[g]] == kDirichlet ? -1.0 : 1.0;
    xg[g] = sg * x[d.gowner[g]];
}

// x_v = sum alpha x_e over the vertex list; a cell reads x, a ghost xg.  The
// entries go in batches of 8: the weight and index loads of a batch first,
// then its gathers, so 8 gathers are in flight per thread.
__global__ __launch_bounds__(kBlock) void k_mf_vertex(Dev d, const double* __restrict__ x,
                                                      const double* __restrict__ xg, double* __restrict__ xv,
                                                      const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t v = gtid_m();
    if (v >= d.nv) return;
    const int64_t sl = v >> 6;
    const int64_t base = d.n_off[sl] + (v & 63);
    const int w = d.n_w[sl];
    const int nc = int(d.nc);
    double s = 0.0;
    for (int k0 = 0; k0 < w; k0 += 8) {
        int e[8];
        double al[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool in = k0 + j < w;
            const int64_t at = base + int64_t(k0 + j) * 64;
            e[j] = in ? d.n_idx[at] : 0;                 // padding entries carry weight 0
            al[j] = in ? d.n_alpha[at] : 0.0;
        }
        double xe[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) xe[j] = e[j] < nc ? x[e[j]] : xg[e[j] - nc];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += al[j] * xe[j];
    }
    xv[v] = s;
}

__global__ __launch_bounds__(kBlock) void k_mf_face(Dev d, BcTable bc, const double* __restrict__ x,
                                                    const double* __restrict__ xv, double* __restrict__ F,
                                                    const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t f = gtid_m();
    if (f >= d.nf) return;
    const int L = d.fL[f];
    double xr;
    if (f >= d.nfi) {
        if (bc.kind[d.gtag[f - d.nfi]] != kDirichlet) {
            F[f] = 0.0;
            return;
        }
        xr = -x[L];
    } else {
        xr = x[d.fR[f]];
    }
    const double xc = xv[d.fC[f]];
    F[f] = d.kAC[f] * (xv[d.fA[f]] - xc) + d.kBC[f] * (xv[d.fB[f]] - xc) + d.kRL[f] * (xr - x[L]);
}

// y_i = -sum_f s_if F_f
__device__ inline double gather_row(const Dev& d, const double* __restrict__ F, int64_t i) {
    double y = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int code = d.c2f[k * d.nc + i];
        y += code >= 0 ? -F[code] : F[~code];
    }
    return y;
}

__global__ __launch_bounds__(kBlock) void k_mf_gather(Dev d, const double* __restrict__ F, double* y,
                                                      const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t i = gtid_m();
    if (i < d.nc) y[i] = gather_row(d, F, i);
}

// q = K p through F, and the partial p.q (the matrix-free counterpart of
// k_cg_spmv; rows of finished meshes are left untouched)
// (partial slots by logical block; padding blocks past the rows return)
__global__ __launch_bounds__(kBlock) void k_mf_cg_gather(Dev d, const double* __restrict__ F, int64_t nblk) {
    __shared__ double lds[4];
    const int64_t lb = xcd_block();
    if (lb >= nblk) return;
    const BlockSeg g = block_seg(d, lb * kBlock, kBlock);
    if (block_done(d, g)) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < d.nc && msc(d, row_mesh(g, i))[SC_DONE] == 0.0) {
        const double y = gather_row(d, F, i);
        d.q[i] = y;
        v[0] = d.p[i] * y;
    }
    seg_publish_at<1>(d, g, v, i >= g.split, lds, lb, nblk);
}

}  // namespace

hipError_t launch_mf_apply(const Dev& d, const BcTable& bc, const double* x, double* y, hipStream_t s,
                           const double* skip) {
    hipLaunchKernelGGL(k_mf_ghost, dim3(unsigned((d.nb + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d, bc, x,
                       d.mf_xg, skip);
    hipLaunchKernelGGL(k_mf_vertex, dim3(rows_m(d.nv, kBlock)), dim3(kBlock), 0, s, d, x, d.mf_xg, d.mf_xv, skip);
    hipLaunchKernelGGL(k_mf_face, dim3(rows_m(d.nf, kBlock)), dim3(kBlock), 0, s, d, bc, x, d.mf_xv, d.mf_flux, skip);
    hipLaunchKernelGGL(k_mf_gather, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, d.mf_flux, y, skip);
    return hipGetLastError();
}

hipError_t launch_mf_cg_part(const Dev& d, const BcTable& bc, int part, hipStream_t s) {
    const double* none = nullptr;
    if (part == 0) {
        hipLaunchKernelGGL(k_mf_ghost, dim3(unsigned((d.nb + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d, bc, d.p,
                           d.mf_xg, none);
        hipLaunchKernelGGL(k_mf_vertex, dim3(rows_m(d.nv, kBlock)), dim3(kBlock), 0, s, d, d.p, d.mf_xg, d.mf_xv, none);
    } else if (part == 1) {
        hipLaunchKernelGGL(k_mf_face, dim3(rows_m(d.nf, kBlock)), dim3(kBlock), 0, s, d, bc, d.p, d.mf_xv, d.mf_flux, none);
    } else {
        const int64_t nblk = (d.nc + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_mf_cg_gather, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, d.mf_flux, nblk);
        hipLaunchKernelGGL(k_cg_alpha<1>, dim3(d.nm), dim3(1024), 0, s, d, nblk, int64_t(kBlock));
    }
    return hipGetLastError();
}

hipError_t launch_mf_cg_spmv(const Dev& d, const BcTable& bc, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int part = 0; part < 3 && e == hipSuccess; ++part) e = launch_mf_cg_part(d, bc, part, s);
    return e;
}

}  // namespace mifvm
