// Row i of the matrix-free Poisson operator from the per-cell tables that
// k_mf_cell_setup (mf_kernels.hip) builds:
//     (K x)_i = -(sum_k w_k x_v[vid_k] + sum_k r_k t_k)
// over the cell's 4 vertices (vertex values x_v of the current x) and its 4
// faces: t_k = x[n_k] - x_i across an interior face (n_k from c2n), t_k = x_i
// on a boundary face (r_k = -2 kRL on a Dirichlet face, 0 on the others).
// Shared by the per-launch product and the persistent batch solver.
#pragma once
#include "state.h"

namespace mifvm {

template <class R> struct MfCell;
template <> struct MfCell<double> {
    __device__ static const double* w(const Dev& d) { return d.mfc_w; }
    __device__ static const double* r(const Dev& d) { return d.mfc_r; }
};
template <> struct MfCell<float> {
    __device__ static const float* w(const Dev& d) { return d.mfc_w32; }
    __device__ static const float* r(const Dev& d) { return d.mfc_r32; }
};

// (K x)_i from the tables: the row's table loads go out together, then its
// 4 vertex values and 4 neighbour values (a boundary face reads x_i)
template <class R>
__device__ inline R cell_row(const Dev& d, const R* __restrict__ x, const R* __restrict__ xv, int64_t i) {
    const int64_t nc = d.nc;
    const R* __restrict__ W = MfCell<R>::w(d);
    const R* __restrict__ Rk = MfCell<R>::r(d);
    int vid[4], nb[4];
    R w[4], r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        vid[k] = d.mfc_vid[k * nc + i];
        nb[k] = d.c2n[k * nc + i];
        w[k] = W[k * nc + i];
        r[k] = Rk[k * nc + i];
    }
    const R xi = x[i];
    R xvv[4], xn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        xvv[k] = xv[vid[k]];
        xn[k] = x[nb[k] < nc ? nb[k] : i];
    }
    R acc = R(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += w[k] * xvv[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += r[k] * (nb[k] < nc ? xn[k] - xi : xn[k]);
    return -acc;
}

}  // namespace mifvm
