// Coupled streamer-type loop (Sec. 4, eq. (10)): the per-step kernels that
// tie the Poisson solve to the transport step of the electron density n_e.
//   k_streamer_rhs     f = kappa (n_e - n_p), the right-hand side of
//                      Delta P = f (the paper's Laplacian of the potential
//                      equals -e/eps (n_p - n_e));
//   k_streamer_fields  per cell: g = least-squares gradient of P over the
//                      node-neighbour stencil (Algorithm 1), ghost values of
//                      P from the potential's boundary conditions; E = -g,
//                      v_e = -mu E, S_e = alpha(|E|) |v_e| n_e with
//                      alpha(|E|) = a exp(-b / |E|) (0 when E = 0);
//   k_ion_update       n_p += dt S_e with the cell's mesh's step.
// Also here: the discrete L2 norm of mifvm_norm_l2 (cell-centre quadrature,
// the annex's error report), a deterministic two-pass reduction.
// The stencil is read from the 64-row slices of global indices (padding is
// the cell itself, which adds exact zeros).  This runs once per coupled
// step, beside a Poisson solve of some thousand products, so it stays a
// plain gather kernel.
#include <algorithm>

#include "reduce.h"
#include "seg.h"
#include "state.h"

namespace mifvm {
namespace {

__device__ inline int64_t tid_s() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
inline unsigned grid_s(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_streamer_rhs(Dev d, double kappa, double* __restrict__ f) {
    const int64_t i = tid_s();
    if (i < d.nc) f[i] = kappa * (d.u[i] - d.np_ion[i]);
}

// value of P at a stencil entity (cell, or ghost from the potential's BCs)
__device__ inline double pot_at(const Dev& d, const BcTable& bc, int e) {
    if (e < d.nc) return d.x[e];
    const int64_t g = e - d.nc;
    const int t = d.gtag[g];
    const double po = d.x[d.gowner[g]];
    const int kind = bc.kind[t];
    if (kind == kDirichlet) return 2.0 * bc.val[g] - po;
    if (kind == kNeumann) return po + bc.val[g] * d.gdist[g];
    return po;
}

__global__ __launch_bounds__(kBlock) void k_streamer_fields(Dev d, BcTable bc, double mu, double a, double b) {
    const int64_t i = tid_s();
    const int64_t nc = d.nc;
    if (i >= nc) return;
    const double4 me = d.xyz4[i];
    const double pi = d.x[i];
    const int64_t s = i >> 6;
    const int32_t* __restrict__ idx = d.s_idx + d.s_off[s] + (i & 63);
    const int w = d.s_w[s];
    double jx = 0.0, jy = 0.0, jz = 0.0;
    for (int k0 = 0; k0 < w; k0 += 8) {
        int e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = k0 + j < w ? idx[int64_t(k0 + j) * 64] : int(i);
        double4 pe[8];
        double ve[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            pe[j] = d.xyz4[e[j]];
            ve[j] = pot_at(d, bc, e[j]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double dv = ve[j] - pi;
            jx += (pe[j].x - me.x) * dv;
            jy += (pe[j].y - me.y) * dv;
            jz += (pe[j].z - me.z) * dv;
        }
    }
    const double* __restrict__ m = d.minv;
    const double m0 = m[i], m1 = m[nc + i], m2 = m[2 * nc + i];
    const double m3 = m[3 * nc + i], m4 = m[4 * nc + i], m5 = m[5 * nc + i];
    const double ex = -(m0 * jx + m1 * jy + m2 * jz);
    const double ey = -(m1 * jx + m3 * jy + m4 * jz);
    const double ez = -(m2 * jx + m4 * jy + m5 * jz);
    d.efield[i] = ex;
    d.efield[nc + i] = ey;
    d.efield[2 * nc + i] = ez;
    d.vel[i] = -mu * ex;
    d.vel[nc + i] = -mu * ey;
    d.vel[2 * nc + i] = -mu * ez;
    const double en = sqrt(ex * ex + ey * ey + ez * ez);
    const double alpha = en > 0.0 ? a * exp(-b / en) : 0.0;
    d.src[i] = alpha * (mu * en) * d.u[i];
}

__global__ __launch_bounds__(kBlock) void k_ion_update(Dev d) {
    const int64_t i = tid_s();
    if (i < d.nc) d.np_ion[i] = d.np_ion[i] + d.mesh_dt[mesh_of(d, i)] * d.src[i];
}

// partials of sum mu_i (a_i - e_i)^2: a grid-stride sum per block, then one
// block adds the partials in block order (deterministic)
__global__ __launch_bounds__(kBlock) void k_norm_part(Dev d, const double* __restrict__ a,
                                                      const double* __restrict__ e) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int64_t i = tid_s(); i < d.nc; i += int64_t(gridDim.x) * kBlock) {
        const double v = a[i] - (e ? e[i] : 0.0);
        s += d.vol[i] * v * v;
    }
    s = block_sum256(s, lds);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_norm_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    const double s = reduce_partials_sum(d.partial, nparts, lds);
    if (threadIdx.x == 0) d.scal[SC_NORM] = s;
}

}  // namespace

hipError_t launch_norm_l2(const Dev& d, const double* a, const double* e, hipStream_t s) {
    const int64_t nb = std::min<int64_t>(1024, std::max<int64_t>(1, (d.nc + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_norm_part, dim3(unsigned(nb)), dim3(kBlock), 0, s, d, a, e);
    hipLaunchKernelGGL(k_norm_fin, dim3(1), dim3(1024), 0, s, d, nb);
    return hipGetLastError();
}

hipError_t launch_streamer_rhs(const Dev& d, double kappa, double* f, hipStream_t s) {
    hipLaunchKernelGGL(k_streamer_rhs, dim3(grid_s(d.nc)), dim3(kBlock), 0, s, d, kappa, f);
    return hipGetLastError();
}

hipError_t launch_streamer_fields(const Dev& d, const BcTable& bc_pot, double mu, double a, double b,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_streamer_fields, dim3(grid_s(d.nc)), dim3(kBlock), 0, s, d, bc_pot, mu, a, b);
    return hipGetLastError();
}

hipError_t launch_ion_update(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_ion_update, dim3(grid_s(d.nc)), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

}  // namespace mifvm
