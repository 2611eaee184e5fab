// Mixed-precision Poisson solve: iterative refinement whose correction
// equation K d = r is solved approximately by Jacobi-CG in FP32 (FP32 matrix
// copy and vectors, FP64 accumulation of every dot product), while the true
// residual r = b - K x and the update x += d stay in FP64.  The FP64 outer
// residual also serves as the restart of the inner CG.
#include "cg_scalars.h"
#include "reduce.h"
#include "seg.h"
#include "state.h"
#include "halo_stage.h"

namespace mifvm {

namespace {
__device__ inline int64_t tid_g() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
inline int rows_grid(int64_t n) { return int((n + kBlock - 1) / kBlock); }
}  // namespace

__global__ __launch_bounds__(kBlock) void k_cast_matrix(Dev d, int64_t padded) {
    const int64_t i = tid_g();
    if (i < padded) d.k_val32[i] = float(d.k_val[i]);
    if (i < d.nc) {
        d.k_diag32[i] = float(d.k_diag[i]);
        d.k_dinv32[i] = float(d.k_dinv[i]);
    }
}

// Outer step: r = b - K x (FP64, same entries and order as the plain SpMV);
// inner start d = 0, r32 = r, z32 = D^-1 r32, p32 = z32.  Partials: true
// rr (FP64), inner rz and rr (FP64 sums of FP32 values), bb.
// kx non-null: K x was formed by the matrix-free product.
__global__ __launch_bounds__(kBlock) void k_ir_residual(Dev d, const double* __restrict__ kx) {
    __shared__ double lds[4];
    const int64_t i = tid_g();
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < d.nc) {
        double y;
        if (kx) {
            y = kx[i];
        } else {
            const int64_t s = i >> 6;
            const int64_t base = d.k_off[s] + (i & 63);
            const int w = d.k_w[s];
            y = d.k_diag[i] * d.x[i];
            for (int k = 0; k < w; ++k) {
                const int64_t at = base + int64_t(k) * 64;
                y += d.k_val[at] * d.x[d.k_col[at]];
            }
        }
        const double bi = d.b[i];
        const double ri = bi - y;
        const float r32 = float(ri);
        const float z32 = d.k_dinv32[i] * r32;
        d.r32[i] = r32;
        d.z32[i] = z32;
        d.p32[i] = z32;
        d.d32[i] = 0.0f;
        v[0] = ri * ri;
        v[1] = double(r32) * double(z32);
        v[2] = double(r32) * double(r32);
        v[3] = bi * bi;
    }
    seg_publish<4>(d, g, v, i >= g.split, lds);
}

// One block per mesh.  fresh: a new solve (sets the outer tolerance, limits
// and count).  The inner solve runs until ||r32|| <= max(tol_in ||r32_0||,
// tol ||b|| / 2), the iteration limit, or a restart; the outer loop ends
// when the FP64 true residual meets tol.
__global__ __launch_bounds__(1024) void k_ir_residual_fin(Dev d, int64_t nparts, double tol, double tol_in,
                                                          int maxit, int restart, int fresh) {
    __shared__ double lds[16];
    const int m = blockIdx.x;
    double t[4];
    seg_sums<4>(d, 0, m, nparts, kBlock, lds, t);
    const double trr = t[0], trz = t[1], trr32 = t[2], tbb = t[3];
    if (threadIdx.x == 0) {
        double* sc = msc(d, m);
        sc[SC_TRUE_RR] = trr;
        sc[SC_BB] = tbb;
        sc[SC_RZ] = trz;
        sc[SC_RR] = trr32;
        if (fresh) {
            sc[SC_TOL2BB_OUT] = tol * tol * tbb;
            sc[SC_MAXIT] = double(maxit);
            sc[SC_RESTART] = double(restart);
            sc[SC_IT] = 0.0;
        }
        // inner target: the asked reduction of this step's residual, but no
        // further than half the outer tolerance (the last step stops early)
        sc[SC_TOL2BB] = fmax(tol_in * tol_in * trr32, 0.25 * sc[SC_TOL2BB_OUT]);
        sc[SC_SINCE] = 0.0;
        sc[SC_DONE] = (trr <= sc[SC_TOL2BB_OUT] || tbb == 0.0) ? 1.0 : (sc[SC_IT] >= sc[SC_MAXIT] ? 2.0 : 0.0);
    }
}

// q32 = K32 p32 with the tile's halo of p32 in LDS; partial p.q in FP64
__global__ __launch_bounds__(kBlock) void k_cg32_spmv(Dev d) {
    extern __shared__ float sp32[];
    __shared__ double lds[4];
    const int64_t nc = d.nc;
    const int64_t t = blockIdx.x;
    const int T = blockDim.x;
    const BlockSeg g = block_seg(d, t * T, T);
    if (block_done(d, g)) return;
    stage_halo_values(d, t, d.p32, sp32);
    __syncthreads();
    const int64_t i = t * T + threadIdx.x;
    double v[1] = {0.0};
    if (i < nc && msc(d, row_mesh(g, i))[SC_DONE] == 0.0) {
        const float pi = sp32[d.h_self[t] + threadIdx.x];
        const int64_t s = i >> 6;
        const int64_t base = d.k_off[s] + (i & 63);
        const int w = d.k_w[s];
        float y = d.k_diag32[i] * pi;
        for (int k0 = 0; k0 < w; k0 += 16) {
            uint16_t l[16];
            float a[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const bool in = k0 + j < w;
                const int64_t at = base + int64_t(k0 + j) * 64;
                l[j] = in ? d.k_lidx[at] : 0;
                a[j] = in ? d.k_val32[at] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) y += a[j] * sp32[l[j]];
        }
        d.q32[i] = y;
        v[0] = double(pi) * double(y);
    }
    seg_publish<1>(d, g, v, i >= g.split, lds);
}

// d += alpha p; r -= alpha q; z = D^-1 r (FP32); partial rz, rr (FP64).
// The row's loads go out before the meshes' scalars are read (they do not
// depend on them; a row past the mesh reads a valid row and is dropped), so
// a block pays one memory latency, not three, before its stores.
__global__ __launch_bounds__(kBlock) void k_cg32_axpy(Dev d) {
    __shared__ double lds[4];
    const int64_t i = tid_g();
    const int64_t j = i < d.nc ? i : d.nc - 1;
    const float di = d.d32[j], pi = d.p32[j], r0 = d.r32[j], qi = d.q32[j], dv = d.k_dinv32[j];
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    if (block_done(d, g)) return;
    const double* sc = msc(d, row_mesh(g, i));
    double v[2] = {0.0, 0.0};
    if (i < d.nc && sc[SC_DONE] == 0.0) {
        const float alpha = float(sc[SC_ALPHA]);
        d.d32[i] = di + alpha * pi;
        const float ri = r0 - alpha * qi;
        const float zi = dv * ri;
        d.r32[i] = ri;
        d.z32[i] = zi;
        v[0] = double(ri) * double(zi);
        v[1] = double(ri) * double(ri);
    }
    seg_publish<2>(d, g, v, i >= g.split, lds);
}

// p = z + beta p (FP32), the row's loads first as above
__global__ __launch_bounds__(kBlock) void k_cg32_dir(Dev d) {
    const int64_t i = tid_g();
    const int64_t j = i < d.nc ? i : d.nc - 1;
    const float zi = d.z32[j], pi = d.p32[j];
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    if (block_done(d, g)) return;
    if (i >= d.nc) return;
    const double* sc = msc(d, row_mesh(g, i));
    if (sc[SC_DONE] != 0.0) return;
    d.p32[i] = zi + float(sc[SC_BETA]) * pi;
}

// x += d (FP64).  d is zero on meshes that ran no inner solve this step.
__global__ __launch_bounds__(kBlock) void k_ir_update(Dev d) {
    const int64_t i = tid_g();
    if (i >= d.nc) return;
    d.x[i] = d.x[i] + double(d.d32[i]);
}

hipError_t launch_cast_matrix(const Dev& d, int64_t padded, hipStream_t s) {
    const int64_t n = padded > d.nc ? padded : d.nc;
    hipLaunchKernelGGL(k_cast_matrix, dim3(rows_grid(n)), dim3(kBlock), 0, s, d, padded);
    return hipGetLastError();
}

hipError_t launch_ir_residual(const Dev& d, double tol, double tol_in, int maxit, int restart, bool fresh,
                              const double* kx, hipStream_t s) {
    const int nb = rows_grid(d.nc);
    hipLaunchKernelGGL(k_ir_residual, dim3(nb), dim3(kBlock), 0, s, d, kx);
    hipLaunchKernelGGL(k_ir_residual_fin, dim3(d.nm), dim3(1024), 0, s, d, int64_t(nb), tol, tol_in, maxit,
                       restart, fresh ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_cg32_spmv(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_cg32_spmv, dim3(unsigned(d.ntiles)), dim3(d.tile_rows),
                       size_t(d.halo_max) * sizeof(float), s, d);
    hipLaunchKernelGGL(k_cg_alpha<0>, dim3(d.nm), dim3(1024), 0, s, d, d.ntiles, int64_t(d.tile_rows));
    return hipGetLastError();
}

hipError_t launch_cg32_axpy(const Dev& d, hipStream_t s) {
    const int nb = rows_grid(d.nc);
    hipLaunchKernelGGL(k_cg32_axpy, dim3(nb), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL(k_cg_beta<0>, dim3(d.nm), dim3(1024), 0, s, d, int64_t(nb), int64_t(kBlock));
    return hipGetLastError();
}

hipError_t launch_cg32_dir(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_cg32_dir, dim3(rows_grid(d.nc)), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_ir_update(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_ir_update, dim3(rows_grid(d.nc)), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

}  // namespace mifvm
