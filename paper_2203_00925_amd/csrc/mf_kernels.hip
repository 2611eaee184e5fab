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
#include "reduce.h"
#include "seg.h"
#include "state.h"
#include "xcd.h"

namespace mifvm {
namespace {

// The coefficient arrays of one precision: FP64, or the FP32 copies the
// reduced-precision forms read (the inner CG of the refined solve).
template <class R> struct MfCoef;
template <> struct MfCoef<double> {
    __device__ static const double* alpha(const Dev& d) { return d.n_alpha; }
    __device__ static const double* kac(const Dev& d) { return d.kAC; }
    __device__ static const double* kbc(const Dev& d) { return d.kBC; }
    __device__ static const double* krl(const Dev& d) { return d.kRL; }
};
template <> struct MfCoef<float> {
    __device__ static const float* alpha(const Dev& d) { return d.n_alpha32; }
    __device__ static const float* kac(const Dev& d) { return d.kAC32; }
    __device__ static const float* kbc(const Dev& d) { return d.kBC32; }
    __device__ static const float* krl(const Dev& d) { return d.kRL32; }
};

// ghost values of x (homogeneous part): xg[g] = s_g x_owner
template <class R>
__global__ __launch_bounds__(kBlock) void k_mf_ghost(Dev d, BcTable bc, const R* __restrict__ x,
                                                     R* __restrict__ xg, const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= d.nb) return;
    const R sg = bc.kind[d.gtag[g]] == kDirichlet ? R(-1) : R(1);
    xg[g] = sg * x[d.gowner[g]];
}

// x_v = sum alpha x_e over the vertex list; a cell reads x, a ghost xg.  The
// entries go in batches of 24: the weight and index loads of a batch first,
// then its gathers, so 24 gathers are in flight per thread.
template <class R>
__global__ __launch_bounds__(kBlock) void k_mf_vertex(Dev d, const R* __restrict__ x, const R* __restrict__ xg,
                                                      R* __restrict__ xv, const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t v = gtid_m();
    if (v >= d.nv) return;
    const R* __restrict__ alpha = MfCoef<R>::alpha(d);
    const int64_t sl = v >> 6;
    const int64_t base = d.n_off[sl] + (v & 63);
    const int w = d.n_w[sl];
    const int nc = int(d.nc);
    R s = R(0);
    // batches of 24 (an interior vertex of the 6-tetrahedra cube has 24
    // cells): the next batch's indices and weights are in flight while this
    // batch's values are gathered (one load per entry: a cell's x or a
    // ghost's xg, by pointer)
    int e[24];
    R al[24];
    auto batch = [&](int k0, int* eo, R* ao) {
#pragma unroll
        for (int j = 0; j < 24; ++j) {
            const bool in = k0 + j < w;
            const int64_t at = base + int64_t(k0 + j) * 64;
            eo[j] = in ? d.n_idx[at] : 0;                // padding entries carry weight 0
            ao[j] = in ? alpha[at] : R(0);
        }
    };
    batch(0, e, al);
    for (int k0 = 0; k0 < w; k0 += 24) {
        R xe[24];
#pragma unroll
        for (int j = 0; j < 24; ++j) xe[j] = *(e[j] < nc ? x + e[j] : xg + (e[j] - nc));
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

// FPT faces per thread (blocks of kBlock threads take kBlock * FPT
// consecutive faces, thread t faces t, t + kBlock, ...): every face's index
// and coefficient loads go out before any of its gathers, with no branch
// between them.  A face's arithmetic does not depend on FPT.  At 10.4M cells
// one face per thread measured fastest (0.230 ms; 2 and 4: 0.234, 0.238; the
// form that returned early on non-Dirichlet boundary faces: 0.245).
constexpr int kMfFacesPerThread = 1;
template <class R, int FPT>
__global__ __launch_bounds__(kBlock) void k_mf_face(Dev d, BcTable bc, const R* __restrict__ x,
                                                    const R* __restrict__ xv, R* __restrict__ F,
                                                    const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t f0 = xcd_block() * (int64_t(kBlock) * FPT) + threadIdx.x;
    const R* __restrict__ kac = MfCoef<R>::kac(d);
    const R* __restrict__ kbc = MfCoef<R>::kbc(d);
    const R* __restrict__ krl = MfCoef<R>::krl(d);
    int L[FPT], Rr[FPT], A[FPT], Bv[FPT], C[FPT];
    bool act[FPT], bnd[FPT];
    R ca[FPT], cb[FPT], cr[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
        const int64_t f = f0 + int64_t(j) * kBlock;
        const int64_t fi = f < d.nf ? f : d.nf - 1;      // past the faces: a valid face, not stored
        bnd[j] = fi >= d.nfi;
        act[j] = f < d.nf && (!bnd[j] || bc.kind[d.gtag[fi - d.nfi]] == kDirichlet);
        L[j] = d.fL[fi];
        Rr[j] = d.fR[fi];
        A[j] = d.fA[fi];
        Bv[j] = d.fB[fi];
        C[j] = d.fC[fi];
        ca[j] = kac[fi];
        cb[j] = kbc[fi];
        cr[j] = krl[fi];
    }
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
        const int64_t f = f0 + int64_t(j) * kBlock;
        if (f >= d.nf) continue;
        if (!act[j]) {                                    // Neumann / zero flux: no part in K
            F[f] = R(0);
            continue;
        }
        const R xl = x[L[j]];
        const R xr = bnd[j] ? -xl : x[Rr[j]];
        const R xc = xv[C[j]];
        F[f] = ca[j] * (xv[A[j]] - xc) + cb[j] * (xv[Bv[j]] - xc) + cr[j] * (xr - xl);
    }
}

// y_i = -sum_f s_if F_f
template <class R>
__device__ inline R gather_row(const Dev& d, const R* __restrict__ F, int64_t i) {
    // the four face codes, then the four fluxes, each set in flight together
    int code[4];
    R fl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) code[k] = d.c2f[k * d.nc + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) fl[k] = F[code[k] >= 0 ? code[k] : ~code[k]];
    R y = R(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) y += code[k] >= 0 ? -fl[k] : fl[k];
    return y;
}

__global__ __launch_bounds__(kBlock) void k_mf_gather(Dev d, const double* __restrict__ F, double* y,
                                                      const double* skip) {
    if (skip && *skip != 0.0) return;
    const int64_t i = gtid_m();
    if (i < d.nc) y[i] = gather_row(d, F, i);
}

// q = K p through F, and the partial p.q (the matrix-free counterpart of
// k_cg_spmv; rows of finished meshes are left untouched; partial slots by
// logical block, padding blocks past the rows return).  FP32: q32 = K p32
// with the FP32 coefficients and the partial in FP64 (as k_cg32_spmv).
template <class R>
__global__ __launch_bounds__(kBlock) void k_mf_cg_gather(Dev d, const R* __restrict__ F, int64_t nblk) {
    __shared__ double lds[4];
    const int64_t lb = xcd_block();
    if (lb >= nblk) return;
    const BlockSeg g = block_seg(d, lb * kBlock, kBlock);
    if (block_done(d, g)) return;
    const int64_t i = lb * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < d.nc) {
        // the row's loads go out before the mesh's done flag is read (a
        // finished mesh's row is read and dropped)
        const R y = gather_row(d, F, i);
        const double pi = std::is_same<R, double>::value ? d.p[i] : double(d.p32[i]);
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
    if (d.nb > 0)
        hipLaunchKernelGGL(k_mf_ghost<double>, dim3(unsigned((d.nb + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           d, bc, x, d.mf_xg, skip);
    hipLaunchKernelGGL(k_mf_vertex<double>, dim3(rows_m(d.nv, kBlock)), dim3(kBlock), 0, s, d, x, d.mf_xg,
                       d.mf_xv, skip);
    hipLaunchKernelGGL((k_mf_face<double, kMfFacesPerThread>), dim3(rows_m(d.nf, kBlock * kMfFacesPerThread)),
                       dim3(kBlock), 0, s, d, bc, x, d.mf_xv,
                       d.mf_flux, skip);
    hipLaunchKernelGGL(k_mf_gather, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, d.mf_flux, y, skip);
    return hipGetLastError();
}

namespace {
// one part of q = K p (FP64 p, or FP32 p32 into the same scratch arrays
// taken as floats)
template <class R>
void mf_cg_part(const Dev& d, const BcTable& bc, int part, const R* p, hipStream_t s) {
    const double* none = nullptr;
    R* xg = reinterpret_cast<R*>(d.mf_xg);
    R* xv = reinterpret_cast<R*>(d.mf_xv);
    R* F = reinterpret_cast<R*>(d.mf_flux);
    if (part == 0) {
        if (d.nb > 0)
            hipLaunchKernelGGL(k_mf_ghost<R>, dim3(unsigned((d.nb + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d,
                               bc, p, xg, none);
        hipLaunchKernelGGL(k_mf_vertex<R>, dim3(rows_m(d.nv, kBlock)), dim3(kBlock), 0, s, d, p, xg, xv, none);
    } else if (part == 1) {
        hipLaunchKernelGGL((k_mf_face<R, kMfFacesPerThread>), dim3(rows_m(d.nf, kBlock * kMfFacesPerThread)),
                           dim3(kBlock), 0, s, d, bc, p, xv, F, none);
    } else {
        const int64_t nblk = (d.nc + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_mf_cg_gather<R>, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, F, nblk);
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
    for (int part = 0; part < 3 && e == hipSuccess; ++part) e = launch_mf_cg_part(d, bc, part, s);
    return e;
}

hipError_t launch_mf_cg32_part(const Dev& d, const BcTable& bc, int part, hipStream_t s) {
    mf_cg_part<float>(d, bc, part, d.p32, s);
    return hipGetLastError();
}

hipError_t launch_mf_cg32_spmv(const Dev& d, const BcTable& bc, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int part = 0; part < 3 && e == hipSuccess; ++part) e = launch_mf_cg32_part(d, bc, part, s);
    return e;
}

}  // namespace mifvm
