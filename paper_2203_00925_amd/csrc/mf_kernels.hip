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
#include <type_traits>

#include "cg_scalars.h"
#include "mf_cell.h"
#include "reduce.h"
#include "seg.h"
#include "state.h"
#include "xcd.h"

namespace mifvm {
namespace {

// The vertex weights of one precision: FP64, or the FP32 copies the
// reduced-precision forms read (the inner CG of the refined solve).
template <class R> struct MfCoef;
template <> struct MfCoef<double> {
    __device__ static const double* alpha(const Dev& d) { return d.n_alpha; }
};
template <> struct MfCoef<float> {
    __device__ static const float* alpha(const Dev& d) { return d.n_alpha32; }
};

// The vertex lists for the operator: each ghost entry folded onto its owner
// (the homogeneous ghost value is s_g x_owner, s_g = -1 behind a Dirichlet
// face, +1 otherwise; stored as ~owner for -1), so the vertex pass gathers
// cells only.  Built with the per-cell tables, once per potential
// boundary-kind set.
__global__ __launch_bounds__(kBlock) void k_mf_nidx_setup(Dev d, BcTable bc) {
    const int64_t p = gtid_m();
    if (p >= d.n_entries) return;
    const int e = d.n_idx[p];
    int out = e;
    if (e >= d.nc) {
        const int64_t g = e - d.nc;
        const int o = d.gowner[g];
        out = bc.kind[d.gtag[g]] == kDirichlet ? ~o : o;
    }
    d.mf_nidx[p] = out;
}

// x_v = sum alpha x_e over the vertex list, a ghost entry as +-x of its
// owner (mf_nidx).  The entries go in batches of 24: the weight and index
// loads of a batch first, then its gathers, so 24 gathers are in flight per
// thread.
template <class R>
__global__ __launch_bounds__(kBlock) void k_mf_vertex(Dev d, const R* __restrict__ x, R* __restrict__ xv,
                                                      const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t v = gtid_m();
    if (v >= d.nv) return;
    const R* __restrict__ alpha = MfCoef<R>::alpha(d);
    const int64_t sl = v >> 6;
    const int64_t base = d.n_off[sl] + (v & 63);
    const int w = d.n_w[sl];
    R s = R(0);
    // batches of 24 (an interior vertex of the 6-tetrahedra cube has 24
    // cells): the next batch's indices and weights are in flight while this
    // batch's values are gathered (one load per entry: a cell's x, negated
    // for a ghost stored as ~owner)
    int e[24];
    R al[24];
    auto batch = [&](int k0, int* eo, R* ao) {
#pragma unroll
        for (int j = 0; j < 24; ++j) {
            const bool in = k0 + j < w;
            const int64_t at = base + int64_t(k0 + j) * 64;
            eo[j] = in ? d.mf_nidx[at] : 0;              // padding entries carry weight 0
            ao[j] = in ? alpha[at] : R(0);
        }
    };
    batch(0, e, al);
    for (int k0 = 0; k0 < w; k0 += 24) {
        R xe[24];
#pragma unroll
        for (int j = 0; j < 24; ++j) {
            const R xo = x[e[j] >= 0 ? e[j] : ~e[j]];
            xe[j] = e[j] >= 0 ? xo : -xo;
        }
        int en[24];
        R an[24];
        batch(k0 + 24, en, an);
#pragma unroll
        for (int j = 0; j < 24; ++j) s += al[j] * xe[j];
#pragma unroll
        for (int j = 0; j < 24; ++j) {
            e[j] = en[j];
            al[j] = an[j];
        }
    }
    xv[v] = s;
}

// ---- the product per cell ----------------------------------------------------
// gather_row's y_i = -sum_f s_if F_f regrouped per cell: each face of a
// tetrahedron holds three of its four vertices, so the vertex terms of its
// faces add up to one weight per vertex, w_k = sum over the cell's faces f
// holding vertex k of s_if times that vertex's coefficient in F_f (kAC, kBC
// or -(kAC + kBC)); the kRL term s_if kRL (x_R - x_L) is kRL (x_n - x_i)
// on an interior face (n the cell across it) and -2 kRL x_i on a Dirichlet
// face (its ghost is -x_i in the homogeneous part).  Faces of other kinds are
// not part of K.  So
//     (K x)_i = -(sum_k w_k x_v[vid_k] + sum_k r_k t_k)
// with r_k = kRL and t_k = x[n_k] - x_i on interior faces, r_k = -2 kRL and
// t_k = x_i on Dirichlet faces (r_k = 0 on the others).  Built once per
// potential boundary-kind set; in the product a cell streams 4 vertex ids,
// 4 face neighbours and 8 coefficients instead of its faces' indices and
// coefficients, and no face flux goes through memory.
__global__ __launch_bounds__(kBlock) void k_mf_cell_setup(Dev d, BcTable bc) {
    const int64_t i = gtid_m();
    if (i >= d.nc) return;
    const int64_t nc = d.nc;
    int vid[4] = {-1, -1, -1, -1};
    double w[4] = {0.0, 0.0, 0.0, 0.0}, r[4] = {0.0, 0.0, 0.0, 0.0};
    auto add = [&](int v, double c) {                 // the vertex's slot (first seen, first slot)
        bool done = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool hit = !done && (vid[q] == v || vid[q] < 0);
            if (hit) {
                vid[q] = v;
                w[q] += c;
            }
            done = done || hit;
        }
    };
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int code = d.c2f[k * nc + i];
        const int f = code >= 0 ? code : ~code;
        const double sg = code >= 0 ? 1.0 : -1.0;
        const bool bnd = f >= d.nfi;
        if (bnd && bc.kind[d.gtag[f - d.nfi]] != kDirichlet) continue;
        const double kac = d.kAC[f], kbc = d.kBC[f], krl = d.kRL[f];
        add(d.fA[f], sg * kac);
        add(d.fB[f], sg * kbc);
        add(d.fC[f], sg * (-(kac + kbc)));
        r[k] = bnd ? -2.0 * krl : krl;
    }
    // unused slots (a cell none of whose faces is in K) point at a used
    // vertex, or vertex 0, with weight 0
    const int v0 = vid[0] >= 0 ? vid[0] : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        d.mfc_vid[q * nc + i] = vid[q] >= 0 ? vid[q] : v0;
        d.mfc_w[q * nc + i] = w[q];
        d.mfc_r[q * nc + i] = r[q];
        d.mfc_w32[q * nc + i] = float(w[q]);
        d.mfc_r32[q * nc + i] = float(r[q]);
    }
}

__global__ __launch_bounds__(kBlock) void k_mf_cell(Dev d, const double* __restrict__ x,
                                                    const double* __restrict__ xv, double* y, const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t i = gtid_m();
    if (i < d.nc) y[i] = cell_row(d, x, xv, i);
}

// q = K p from the tables, and the partial p.q (the matrix-free counterpart
// of k_cg_spmv; rows of finished meshes are left untouched; partial slots by
// logical block, padding blocks past the rows return).  FP32: q32 = K p32
// with the FP32 tables and the partial in FP64 (as k_cg32_spmv).
template <class R>
__global__ __launch_bounds__(kBlock) void k_mf_cg_cell(Dev d, int64_t nblk) {
    __shared__ double lds[4];
    const int64_t lb = xcd_block();
    if (lb >= nblk) return;
    const BlockSeg g = block_seg(d, lb * kBlock, kBlock);
    if (block_done(d, g)) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    const R* __restrict__ p = std::is_same<R, double>::value ? reinterpret_cast<const R*>(d.p)
                                                              : reinterpret_cast<const R*>(d.p32);
    const R* __restrict__ xv = reinterpret_cast<const R*>(d.mf_xv);
    double v[1] = {0.0};
    if (i < d.nc) {
        // the row's loads go out before the mesh's done flag is read (a
        // finished mesh's row is read and dropped)
        const R y = cell_row(d, p, xv, i);
        const double pi = double(p[i]);
        if (msc(d, row_mesh(g, i))[SC_DONE] == 0.0) {
            if constexpr (std::is_same<R, double>::value) d.q[i] = y;
            else d.q32[i] = y;
            v[0] = pi * double(y);
        }
    }
    seg_publish_at<1>(d, g, v, i >= g.split, lds, lb, nblk);
}

}  // namespace

hipError_t launch_mf_apply(const Dev& d, const BcTable& bc, const double* x, double* y, hipStream_t s,
                           const double* skip) {
    (void)bc;                                  // its kinds are in the tables
    hipLaunchKernelGGL(k_mf_vertex<double>, dim3(rows_m(d.nv, kBlock)), dim3(kBlock), 0, s, d, x, d.mf_xv, skip);
    hipLaunchKernelGGL(k_mf_cell, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, x, d.mf_xv, y, skip);
    return hipGetLastError();
}

hipError_t launch_mf_cell_setup(const Dev& d, const BcTable& bc_pot, hipStream_t s) {
    hipLaunchKernelGGL(k_mf_cell_setup, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, bc_pot);
    if (d.n_entries > 0)
        hipLaunchKernelGGL(k_mf_nidx_setup, dim3(rows_m(d.n_entries, kBlock)), dim3(kBlock), 0, s, d, bc_pot);
    return hipGetLastError();
}

namespace {
// one part of q = K p (FP64 p, or FP32 p32 into the same scratch arrays
// taken as floats): 0 the vertex values, 1 the per-cell product with the
// p.q partials, 2 alpha
template <class R>
void mf_cg_part(const Dev& d, const BcTable& bc, int part, const R* p, hipStream_t s) {
    (void)bc;                                  // its kinds are in the tables
    const double* none = nullptr;
    R* xv = reinterpret_cast<R*>(d.mf_xv);
    if (part == 0) {
        hipLaunchKernelGGL(k_mf_vertex<R>, dim3(rows_m(d.nv, kBlock)), dim3(kBlock), 0, s, d, p, xv, none);
    } else if (part == 1) {
        const int64_t nblk = (d.nc + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_mf_cg_cell<R>, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, nblk);
    } else {
        const int64_t nblk = (d.nc + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_cg_alpha<1>, dim3(d.nm), dim3(1024), 0, s, d, nblk, int64_t(kBlock));
    }
}
}  // namespace

hipError_t launch_mf_cg_part(const Dev& d, const BcTable& bc, int part, hipStream_t s) {
    mf_cg_part<double>(d, bc, part, d.p, s);
    return hipGetLastError();
}

hipError_t launch_mf_cg_spmv(const Dev& d, const BcTable& bc, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int part = 0; part < kMfParts && e == hipSuccess; ++part) e = launch_mf_cg_part(d, bc, part, s);
    return e;
}

hipError_t launch_mf_cg32_part(const Dev& d, const BcTable& bc, int part, hipStream_t s) {
    mf_cg_part<float>(d, bc, part, d.p32, s);
    return hipGetLastError();
}

hipError_t launch_mf_cg32_spmv(const Dev& d, const BcTable& bc, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int part = 0; part < kMfParts && e == hipSuccess; ++part) e = launch_mf_cg32_part(d, bc, part, s);
    return e;
}

}  // namespace mifvm
