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

namespace mifvm {
namespace {

// Blocks are dealt to the 8 XCDs in turn, and each XCD has its own L2.  The
// grid is padded to a multiple of 8 and block b works on logical block
// (b % 8) * (grid / 8) + b / 8, so each XCD takes one contiguous eighth of
// the rows: the neighbour data that consecutive blocks share (vertex lists
// reading nearby cells, faces reading nearby vertices) then stays in one L2.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block() {
    const int64_t per = gridDim.x / kXcds;
    return int64_t(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}
__device__ inline int64_t gtid_m() { return xcd_block() * blockDim.x + threadIdx.x; }
inline unsigned rows_m(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return unsigned((b + kXcds - 1) / kXcds * kXcds);
}

// x of a cell, or of a ghost entity (homogeneous ghost value)
__device__ inline double xval(const Dev& d, const BcTable& bc, const double* __restrict__ x, int e) {
    if (e < d.nc) return x[e];
    const int g = e - int(d.nc);
    const double s = bc.kind[d.gtag[g]] == kDirichlet ? -1.0 : 1.0;
    return s * x[d.gowner[g]];
}

__global__ __launch_bounds__(kBlock) void k_mf_vertex(Dev d, BcTable bc, const double* __restrict__ x,
                                                      double* __restrict__ xv, const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t v = gtid_m();
    if (v >= d.nv) return;
    const int64_t sl = v >> 6;
    const int64_t base = d.n_off[sl] + (v & 63);
    const int w = d.n_w[sl];
    double s = 0.0;
    for (int k = 0; k < w; ++k) {
        const int64_t at = base + int64_t(k) * 64;
        const double al = d.n_alpha[at];             // padding entries carry 0
        if (al != 0.0) s += al * xval(d, bc, x, d.n_idx[at]);
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
    hipLaunchKernelGGL(k_mf_vertex, dim3(rows_m(d.nv)), dim3(kBlock), 0, s, d, bc, x, d.mf_xv, skip);
    hipLaunchKernelGGL(k_mf_face, dim3(rows_m(d.nf)), dim3(kBlock), 0, s, d, bc, x, d.mf_xv, d.mf_flux, skip);
    hipLaunchKernelGGL(k_mf_gather, dim3(rows_m(d.nc)), dim3(kBlock), 0, s, d, d.mf_flux, y, skip);
    return hipGetLastError();
}

hipError_t launch_mf_cg_part(const Dev& d, const BcTable& bc, int part, hipStream_t s) {
    const double* none = nullptr;
    if (part == 0) {
        hipLaunchKernelGGL(k_mf_vertex, dim3(rows_m(d.nv)), dim3(kBlock), 0, s, d, bc, d.p, d.mf_xv, none);
    } else if (part == 1) {
        hipLaunchKernelGGL(k_mf_face, dim3(rows_m(d.nf)), dim3(kBlock), 0, s, d, bc, d.p, d.mf_xv, d.mf_flux, none);
    } else {
        const int64_t nblk = (d.nc + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_mf_cg_gather, dim3(rows_m(d.nc)), dim3(kBlock), 0, s, d, d.mf_flux, nblk);
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
