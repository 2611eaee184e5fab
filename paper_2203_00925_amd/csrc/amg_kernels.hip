// Aggregation multigrid V(1,1) cycle and the flexible CG around it (the
// setup and the cycle's definition are in amg.h).  Level 0 is the state's
// system: its product is the matrix-free one, its diagonal K's; coarser
// levels store their off-diagonal entries in 64-row slices beside the
// diagonal.  Every kernel takes the solve's done flag and returns at once
// when it is set (a captured chunk of iterations then runs to its end
// without work).
#include "amg_dev.h"
#include "reduce.h"
#include "seg.h"
#include "state.h"

namespace mifvm {
namespace {

__device__ inline int64_t tid_a() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
inline unsigned grid_a(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }
__device__ inline bool done(const double* flag) { return flag && *flag != 0.0; }

// x = w D^-1 b
__global__ __launch_bounds__(kBlock) void k_amg_smooth0(int64_t n, double w, const double* __restrict__ dinv,
                                                        const double* __restrict__ b, double* __restrict__ x,
                                                        const double* flag) {
    if (done(flag)) return;
    const int64_t i = tid_a();
    if (i < n) x[i] = w * dinv[i] * b[i];
}

// x += w D^-1 (b - t)
__global__ __launch_bounds__(kBlock) void k_amg_smooth1(int64_t n, double w, const double* __restrict__ dinv,
                                                        const double* __restrict__ b, const double* __restrict__ t,
                                                        double* __restrict__ x, const double* flag) {
    if (done(flag)) return;
    const int64_t i = tid_a();
    if (i < n) x[i] = x[i] + w * dinv[i] * (b[i] - t[i]);
}

// t = A x on a coarse level (diagonal + sliced off-diagonal entries)
__global__ __launch_bounds__(kBlock) void k_amg_spmv(AmgLevelDev L, const double* __restrict__ x,
                                                     double* __restrict__ t, const double* flag) {
    if (done(flag)) return;
    const int64_t i = tid_a();
    if (i >= L.n) return;
    const int64_t base = L.off[i >> 6] + (i & 63);
    const int w = L.w[i >> 6];
    double y = L.diag[i] * x[i];
    // batches of 8: the next batch's columns and values are in flight while
    // this batch's x values are gathered
    int c[8];
    double a[8];
    auto batch = [&](int k0, int* co, double* ao) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool in = k0 + j < w;
            const int64_t at = base + int64_t(k0 + j) * 64;
            co[j] = in ? L.idx[at] : int(i);
            ao[j] = in ? L.val[at] : 0.0;
        }
    };
    batch(0, c, a);
    for (int k0 = 0; k0 < w; k0 += 8) {
        double xe[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) xe[j] = x[c[j]];
        int cn[8];
        double an[8];
        batch(k0 + 8, cn, an);
#pragma unroll
        for (int j = 0; j < 8; ++j) y += a[j] * xe[j];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            c[j] = cn[j];
            a[j] = an[j];
        }
    }
    t[i] = y;
}

// b_c[I] = sum over the members i of aggregate I of (b[i] - t[i])
__global__ __launch_bounds__(kBlock) void k_amg_restrict(int64_t nco, const int64_t* __restrict__ mptr,
                                                         const int32_t* __restrict__ midx,
                                                         const double* __restrict__ b, const double* __restrict__ t,
                                                         double* __restrict__ bc, const double* flag) {
    if (done(flag)) return;
    const int64_t I = tid_a();
    if (I >= nco) return;
    // members in batches of 8: their indices in flight together, then their
    // values, then the sums in member order (a slot past the aggregate
    // re-reads its first member and is not added; aggregates are non-empty)
    const int64_t m0 = mptr[I], cnt = mptr[I + 1] - m0;
    double s = 0.0;
    for (int64_t k0 = 0; k0 < cnt; k0 += 8) {
        int id[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) id[j] = midx[m0 + (k0 + j < cnt ? k0 + j : 0)];
        double bv[8], tv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            bv[j] = b[id[j]];
            tv[j] = t[id[j]];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (k0 + j < cnt) s += bv[j] - tv[j];
    }
    bc[I] = s;
}

// r = b - t
__global__ __launch_bounds__(kBlock) void k_amg_sub(int64_t n, const double* __restrict__ b,
                                                    const double* __restrict__ t, double* __restrict__ r,
                                                    const double* flag) {
    if (done(flag)) return;
    const int64_t i = tid_a();
    if (i < n) r[i] = b[i] - t[i];
}

// x += y
__global__ __launch_bounds__(kBlock) void k_amg_add(int64_t n, const double* __restrict__ y, double* __restrict__ x,
                                                    const double* flag) {
    if (done(flag)) return;
    const int64_t i = tid_a();
    if (i < n) x[i] = x[i] + y[i];
}

// x[i] += x_c[agg[i]]
__global__ __launch_bounds__(kBlock) void k_amg_prolong(int64_t n, const int32_t* __restrict__ agg,
                                                        const double* __restrict__ xc, double* __restrict__ x,
                                                        const double* flag) {
    if (done(flag)) return;
    const int64_t i = tid_a();
    if (i < n) x[i] = x[i] + xc[agg[i]];
}

// x = C^-1 b on the coarsest level: one block per row
__global__ __launch_bounds__(256) void k_amg_dense(int64_t n, const double* __restrict__ cinv,
                                                   const double* __restrict__ b, double* __restrict__ x,
                                                   const double* flag) {
    __shared__ double lds[4];
    if (done(flag)) return;
    const int64_t r = blockIdx.x;
    double s = 0.0;
    for (int64_t c = threadIdx.x; c < n; c += 256) s += cinv[r * n + c] * b[c];
    s = block_sum256(s, lds);
    if (threadIdx.x == 0) x[r] = s;
}

// ---- flexible CG (one mesh) -------------------------------------------------------
// r = b - t (t = K x); partial rr, bb
__global__ __launch_bounds__(kBlock) void k_amg_open(Dev d, const double* __restrict__ t) {
    __shared__ double lds[4];
    const int64_t i = tid_a();
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    double v[2] = {0.0, 0.0};
    if (i < d.nc) {
        const double bi = d.b[i];
        const double ri = bi - t[i];
        d.r[i] = ri;
        v[0] = ri * ri;
        v[1] = bi * bi;
    }
    seg_publish<2>(d, g, v, i >= g.split, lds);
}

__global__ __launch_bounds__(1024) void k_amg_open_fin(Dev d, int64_t nparts, double tol, int maxit, int restart,
                                                       int fresh) {
    __shared__ double lds[16];
    double t[2];
    seg_sums<2>(d, 0, 0, nparts, kBlock, lds, t);
    const double rr = t[0], bb = t[1];
    if (threadIdx.x == 0) {
        double* sc = d.scal;
        sc[SC_RR] = rr;
        sc[SC_TRUE_RR] = rr;
        sc[SC_BB] = bb;
        if (fresh) {
            sc[SC_TOL2BB] = tol * tol * bb;
            sc[SC_MAXIT] = double(maxit);
            sc[SC_RESTART] = double(restart);
            sc[SC_IT] = 0.0;
        }
        sc[SC_SINCE] = 0.0;
        sc[SC_DONE] = (rr <= sc[SC_TOL2BB] || bb == 0.0) ? 1.0 : (sc[SC_IT] >= sc[SC_MAXIT] ? 2.0 : 0.0);
    }
}

// after the cycle of the opening: p = z, partial z.r
__global__ __launch_bounds__(kBlock) void k_amg_p0(Dev d) {
    __shared__ double lds[4];
    if (d.scal[SC_DONE] != 0.0) return;
    const int64_t i = tid_a();
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    double v[1] = {0.0};
    if (i < d.nc) {
        const double zi = d.z[i];
        d.p[i] = zi;
        v[0] = zi * d.r[i];
    }
    seg_publish<1>(d, g, v, i >= g.split, lds);
}

__global__ __launch_bounds__(1024) void k_amg_rz_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    if (d.scal[SC_DONE] != 0.0) return;
    const double zr = seg_sum(d, 0, 0, nparts, kBlock, lds);
    if (threadIdx.x == 0) d.scal[SC_RZ] = zr;
}

// x += alpha p; r_old = r; r -= alpha q; partial rr
__global__ __launch_bounds__(kBlock) void k_amg_axpy(Dev d, double* __restrict__ r_old) {
    __shared__ double lds[4];
    if (d.scal[SC_DONE] != 0.0) return;
    const int64_t i = tid_a();
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    double v[1] = {0.0};
    if (i < d.nc) {
        const double alpha = d.scal[SC_ALPHA];
        d.x[i] = d.x[i] + alpha * d.p[i];
        const double ro = d.r[i];
        const double ri = ro - alpha * d.q[i];
        r_old[i] = ro;
        d.r[i] = ri;
        v[0] = ri * ri;
    }
    seg_publish<1>(d, g, v, i >= g.split, lds);
}

// count; convergence (1), limit (2) or a scheduled restart (3)
__global__ __launch_bounds__(1024) void k_amg_rr_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    double* sc = d.scal;
    if (sc[SC_DONE] != 0.0) return;
    const double rr = seg_sum(d, 0, 0, nparts, kBlock, lds);
    if (threadIdx.x == 0) {
        sc[SC_RR] = rr;
        sc[SC_IT] = sc[SC_IT] + 1.0;
        sc[SC_SINCE] = sc[SC_SINCE] + 1.0;
        if (rr <= sc[SC_TOL2BB]) sc[SC_DONE] = 1.0;
        else if (sc[SC_IT] >= sc[SC_MAXIT]) sc[SC_DONE] = 2.0;
        else if (sc[SC_RESTART] > 0.0 && sc[SC_SINCE] >= sc[SC_RESTART]) sc[SC_DONE] = 3.0;
    }
}

// partial z.r and z.r_old
__global__ __launch_bounds__(kBlock) void k_amg_zdots(Dev d, const double* __restrict__ r_old) {
    __shared__ double lds[4];
    if (d.scal[SC_DONE] != 0.0) return;
    const int64_t i = tid_a();
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    double v[2] = {0.0, 0.0};
    if (i < d.nc) {
        const double zi = d.z[i];
        v[0] = zi * d.r[i];
        v[1] = zi * r_old[i];
    }
    seg_publish<2>(d, g, v, i >= g.split, lds);
}

// flexible (Polak-Ribiere) beta = z_new . (r_new - r_old) / (z_old . r_old)
__global__ __launch_bounds__(1024) void k_amg_beta_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    double* sc = d.scal;
    if (sc[SC_DONE] != 0.0) return;
    double t[2];
    seg_sums<2>(d, 0, 0, nparts, kBlock, lds, t);
    const double zr = t[0], zro = t[1];
    if (threadIdx.x == 0) {
        sc[SC_BETA] = (zr - zro) / sc[SC_RZ];
        sc[SC_RZ] = zr;
    }
}

}  // namespace

namespace {

hipError_t coarse_correction(const AmgDev& a, int l, const double* flag, hipStream_t s);

// x = cycle of coarse level l (>= 1) on the right-hand side b
hipError_t coarse_cycle(const AmgDev& a, int l, const double* b, double* x, const double* flag, hipStream_t s) {
    const double w = a.omega;
    const AmgLevelDev& L = a.lv[l];
    if (l == a.nl - 1) {               // the coarsest level: its dense inverse
        hipLaunchKernelGGL(k_amg_dense, dim3(unsigned(L.n)), dim3(256), 0, s, L.n, a.cinv, b, x, flag);
        return hipGetLastError();
    }
    const AmgLevelDev& N = a.lv[l + 1];
    hipLaunchKernelGGL(k_amg_smooth0, dim3(grid_a(L.n)), dim3(kBlock), 0, s, L.n, w, L.dinv, b, x, flag);
    hipLaunchKernelGGL(k_amg_spmv, dim3(grid_a(L.n)), dim3(kBlock), 0, s, L, x, L.t, flag);
    hipLaunchKernelGGL(k_amg_restrict, dim3(grid_a(N.n)), dim3(kBlock), 0, s, N.n, L.mptr, L.midx, b, L.t, N.b,
                       flag);
    hipError_t e = coarse_correction(a, l + 1, flag, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amg_prolong, dim3(grid_a(L.n)), dim3(kBlock), 0, s, L.n, L.agg, N.x, x, flag);
    hipLaunchKernelGGL(k_amg_spmv, dim3(grid_a(L.n)), dim3(kBlock), 0, s, L, x, L.t, flag);
    hipLaunchKernelGGL(k_amg_smooth1, dim3(grid_a(L.n)), dim3(kBlock), 0, s, L.n, w, L.dinv, b, L.t, x, flag);
    return hipGetLastError();
}

// level l's x from its b (the restricted residual of level l - 1): one
// cycle, and for a W-cycle a second one on the remaining residual, unless
// level l is solved exactly
hipError_t coarse_correction(const AmgDev& a, int l, const double* flag, hipStream_t s) {
    const AmgLevelDev& N = a.lv[l];
    hipError_t e = coarse_cycle(a, l, N.b, N.x, flag, s);
    for (int k = 1; e == hipSuccess && k < a.gamma && l < a.nl - 1; ++k) {
        hipLaunchKernelGGL(k_amg_spmv, dim3(grid_a(N.n)), dim3(kBlock), 0, s, N, N.x, N.t, flag);
        hipLaunchKernelGGL(k_amg_sub, dim3(grid_a(N.n)), dim3(kBlock), 0, s, N.n, N.b, N.t, N.r, flag);
        e = coarse_cycle(a, l, N.r, N.e, flag, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_amg_add, dim3(grid_a(N.n)), dim3(kBlock), 0, s, N.n, N.e, N.x, flag);
            e = hipGetLastError();
        }
    }
    return e;
}

}  // namespace

hipError_t launch_amg_cycle(const Dev& d, const BcTable& bc_pot, const AmgDev& a, const double* b0, double* x0,
                            const double* flag, hipStream_t s, const AmgSmoother* fine) {
    const int nl = a.nl;
    const double w = a.omega;
    if (nl == 1) {                 // the system is small enough to invert densely
        hipLaunchKernelGGL(k_amg_dense, dim3(unsigned(d.nc)), dim3(256), 0, s, d.nc, a.cinv, b0, x0, flag);
        return hipGetLastError();
    }
    // level 0: smoothing with the matrix-free product (into tmp), then the
    // coarse levels
    hipError_t e = hipSuccess;
    if (fine) {
        e = (*fine)(b0, x0, s);                    // x = M(b)
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_amg_smooth0, dim3(grid_a(d.nc)), dim3(kBlock), 0, s, d.nc, w, d.k_dinv, b0, x0,
                           flag);
    }
    e = launch_mf_apply(d, bc_pot, x0, d.tmp, s, flag);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amg_restrict, dim3(grid_a(a.lv[1].n)), dim3(kBlock), 0, s, a.lv[1].n, a.lv[0].mptr,
                       a.lv[0].midx, b0, d.tmp, a.lv[1].b, flag);
    e = coarse_correction(a, 1, flag, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amg_prolong, dim3(grid_a(d.nc)), dim3(kBlock), 0, s, d.nc, a.lv[0].agg, a.lv[1].x, x0,
                       flag);
    e = launch_mf_apply(d, bc_pot, x0, d.tmp, s, flag);
    if (e != hipSuccess) return e;
    if (fine) {                                    // x += M(b - K x)
        hipLaunchKernelGGL(k_amg_sub, dim3(grid_a(d.nc)), dim3(kBlock), 0, s, d.nc, b0, d.tmp, a.s0, flag);
        e = (*fine)(a.s0, a.s1, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_amg_add, dim3(grid_a(d.nc)), dim3(kBlock), 0, s, d.nc, a.s1, x0, flag);
    } else {
        hipLaunchKernelGGL(k_amg_smooth1, dim3(grid_a(d.nc)), dim3(kBlock), 0, s, d.nc, w, d.k_dinv, b0, d.tmp,
                           x0, flag);
    }
    return hipGetLastError();
}

hipError_t launch_amg_open(const Dev& d, const BcTable& bc_pot, const AmgDev& a, double tol, int maxit,
                           int restart, bool fresh, hipStream_t s, const AmgSmoother* fine) {
    const int64_t nb = grid_a(d.nc);
    hipError_t e = launch_mf_apply(d, bc_pot, d.x, d.tmp, s);            // t = K x
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amg_open, dim3(unsigned(nb)), dim3(kBlock), 0, s, d, d.tmp);
    hipLaunchKernelGGL(k_amg_open_fin, dim3(1), dim3(1024), 0, s, d, nb, tol, maxit, restart, fresh ? 1 : 0);
    e = launch_amg_cycle(d, bc_pot, a, d.r, d.z, d.scal + SC_DONE, s, fine);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amg_p0, dim3(unsigned(nb)), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL(k_amg_rz_fin, dim3(1), dim3(1024), 0, s, d, nb);
    return hipGetLastError();
}

hipError_t launch_amg_iteration(const Dev& d, const BcTable& bc_pot, const AmgDev& a, bool matrix_free,
                                hipStream_t s, const AmgSmoother* fine) {
    const int64_t nb = grid_a(d.nc);
    hipError_t e = matrix_free ? launch_mf_cg_spmv(d, bc_pot, s) : launch_cg_spmv(d, s);   // q = K p, alpha
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amg_axpy, dim3(unsigned(nb)), dim3(kBlock), 0, s, d, a.r_old);
    hipLaunchKernelGGL(k_amg_rr_fin, dim3(1), dim3(1024), 0, s, d, nb);
    e = launch_amg_cycle(d, bc_pot, a, d.r, d.z, d.scal + SC_DONE, s, fine);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amg_zdots, dim3(unsigned(nb)), dim3(kBlock), 0, s, d, a.r_old);
    hipLaunchKernelGGL(k_amg_beta_fin, dim3(1), dim3(1024), 0, s, d, nb);
    return launch_cg_dir(d, s);                                           // p = z + beta p
}

}  // namespace mifvm
