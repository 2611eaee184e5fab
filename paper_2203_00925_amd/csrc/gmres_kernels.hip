// Kernels of the restarted flexible GMRES(m) (gmres.h).  Every kernel of a
// step returns at once when the solve has finished (SC_DONE != 0), so a
// captured cycle replays cheaply past convergence.  Reductions are per-block
// partial sums of a fixed grid, added in block order by one block
// (deterministic).
#include "gmres.h"
#include "halo_stage.h"
#include "reduce.h"

namespace mifvm {
namespace {

inline unsigned grid_red(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return unsigned(b < kGmGrid ? (b < 1 ? 1 : b) : kGmGrid);
}
__device__ inline bool finished(const Dev& d) { return d.scal[SC_DONE] != 0.0; }

// r = b - (K x); partial rr, bb
__global__ __launch_bounds__(256) void k_gm_residual(Dev d, GmDev g, const double* kx) {
    __shared__ double lds[4];
    double a = 0.0, c = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < d.nc; i += int64_t(gridDim.x) * 256) {
        double y;
        if (kx) {
            y = kx[i];
        } else {
            const int64_t s = i >> 6;
            const int64_t base = d.k_off[s] + (i & 63);
            y = d.k_diag[i] * d.x[i];
            for (int k = 0; k < d.k_w[s]; ++k) {
                const int64_t at = base + int64_t(k) * 64;
                y += d.k_val[at] * d.x[d.k_col[at]];
            }
        }
        const double bi = d.b[i], ri = bi - y;
        g.V[i] = ri;
        a += ri * ri;
        c += bi * bi;
    }
    const double s0 = block_sum256(a, lds), s1 = block_sum256(c, lds);
    if (threadIdx.x == 0) {
        g.partial[blockIdx.x] = s0;
        g.partial[kGmGrid + blockIdx.x] = s1;
    }
}

__global__ __launch_bounds__(1024) void k_gm_open_fin(Dev d, GmDev g, int nparts, double tol, int maxit,
                                                      int fresh) {
    __shared__ double lds[16];
    const double rr = reduce_partials_sum(g.partial, nparts, lds);
    const double bb = reduce_partials_sum(g.partial + kGmGrid, nparts, lds);
    if (threadIdx.x == 0) {
        double* sc = d.scal;
        sc[SC_RR] = rr;
        sc[SC_TRUE_RR] = rr;
        sc[SC_BB] = bb;
        if (fresh) {
            sc[SC_TOL2BB] = tol * tol * bb;
            sc[SC_MAXIT] = double(maxit);
            sc[SC_IT] = 0.0;
        }
        sc[SC_DONE] = (rr <= sc[SC_TOL2BB] || bb == 0.0) ? 1.0 : (sc[SC_IT] >= sc[SC_MAXIT] ? 2.0 : 0.0);
        const double beta = sqrt(rr);
        g.sc[GM_BETA] = beta;
        g.sc[GM_K] = 0.0;
        g.sc[GM_INVH] = beta > 0.0 ? 1.0 / beta : 0.0;
        for (int i = 0; i <= g.m; ++i) g.g[i] = 0.0;
        g.g[0] = beta;
    }
}

// v_j = w / h (in place in V[j]); z_j = D^-1 v_j
__global__ __launch_bounds__(256) void k_gm_next(Dev d, GmDev g, int j) {
    if (finished(d)) return;
    const double ih = g.sc[GM_INVH];
    double* v = g.V + int64_t(j) * d.nc;
    double* z = g.Z + int64_t(j) * d.nc;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < d.nc; i += int64_t(gridDim.x) * 256) {
        const double vi = v[i] * ih;
        v[i] = vi;
        z[i] = d.k_dinv[i] * vi;
    }
}

// w = K z_j into V[j + 1]: one block per LDS tile as the CG's product
__global__ __launch_bounds__(256) void k_gm_spmv(Dev d, GmDev g, int j) {
    extern __shared__ double sp[];
    if (finished(d)) return;
    const int64_t nc = d.nc;
    const int64_t t = blockIdx.x;
    const int T = blockDim.x;
    const double* __restrict__ z = g.Z + int64_t(j) * nc;
    double* w = g.V + int64_t(j + 1) * nc;
    stage_halo_values(d, t, z, sp);
    __syncthreads();
    const int64_t i = t * T + threadIdx.x;
    if (i >= nc) return;
    const int64_t s = i >> 6;
    const int64_t base = d.k_off[s] + (i & 63);
    const int wd = d.k_w[s];
    double y = d.k_diag[i] * sp[d.h_self[t] + threadIdx.x];
    for (int k0 = 0; k0 < wd; k0 += 16) {
        uint16_t l[16];
        double a[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const bool in = k0 + jj < wd;
            const int64_t at = base + int64_t(k0 + jj) * 64;
            l[jj] = in ? d.k_lidx[at] : uint16_t(0);
            a[jj] = in ? d.k_val[at] : 0.0;
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            if (k0 + jj < wd) y += a[jj] * sp[l[jj]];
    }
    w[i] = y;
}

// partial h_i = v_i . w for i in [i0, i0 + cnt), cnt <= kGmDots, w = V[j + 1]:
// one pass over w for up to kGmDots basis vectors
constexpr int kGmDots = 32;
__global__ __launch_bounds__(256) void k_gm_dots(Dev d, GmDev g, int j, int i0, int cnt) {
    __shared__ double lds[4];
    if (finished(d)) return;
    const double* __restrict__ w = g.V + int64_t(j + 1) * d.nc;
    double acc[kGmDots];
#pragma unroll
    for (int q = 0; q < kGmDots; ++q) acc[q] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < d.nc; i += int64_t(gridDim.x) * 256) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < kGmDots; ++q)
            if (q < cnt) acc[q] += g.V[int64_t(i0 + q) * d.nc + i] * wi;
    }
#pragma unroll
    for (int q = 0; q < kGmDots; ++q) {
        if (q < cnt) {                         // cnt is the same for the whole block
            const double s = block_sum256(acc[q], lds);
            if (threadIdx.x == 0) g.partial[int64_t(i0 + q) * kGmGrid + blockIdx.x] = s;
        }
    }
}

// column j of H from the partials: block i sums those of h_ij
__global__ __launch_bounds__(1024) void k_gm_hcol(Dev d, GmDev g, int j, int nparts) {
    __shared__ double lds[16];
    if (finished(d)) return;
    const int i = blockIdx.x;
    const double h = reduce_partials_sum(g.partial + int64_t(i) * kGmGrid, nparts, lds);
    if (threadIdx.x == 0) g.H[int64_t(j) * (g.m + 1) + i] = h;
}

// w -= sum_{i <= j} h_ij v_i; partial |w|^2
__global__ __launch_bounds__(256) void k_gm_orth(Dev d, GmDev g, int j) {
    __shared__ double lds[4];
    if (finished(d)) return;
    double* w = g.V + int64_t(j + 1) * d.nc;
    const double* hc = g.H + int64_t(j) * (g.m + 1);
    double a = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < d.nc; i += int64_t(gridDim.x) * 256) {
        double wi = w[i];
        for (int q = 0; q <= j; ++q) wi -= hc[q] * g.V[int64_t(q) * d.nc + i];
        w[i] = wi;
        a += wi * wi;
    }
    const double s = block_sum256(a, lds);
    if (threadIdx.x == 0) g.partial[blockIdx.x] = s;
}

// h_{j+1,j} = |w|; rotations; residual estimate; convergence and limit tests
__global__ __launch_bounds__(1024) void k_gm_givens(Dev d, GmDev g, int j, int nparts) {
    __shared__ double lds[16];
    if (finished(d)) return;
    const double ww = reduce_partials_sum(g.partial, nparts, lds);
    if (threadIdx.x != 0) return;
    double* sc = d.scal;
    const int ld = g.m + 1;
    double* h = g.H + int64_t(j) * ld;
    const double hn = sqrt(ww);
    for (int i = 0; i < j; ++i) {
        const double a = h[i], b = h[i + 1];
        h[i] = g.cs[i] * a + g.sn[i] * b;
        h[i + 1] = -g.sn[i] * a + g.cs[i] * b;
    }
    const double den = hypot(h[j], hn);
    const double c = den > 0.0 ? h[j] / den : 1.0, sn = den > 0.0 ? hn / den : 0.0;
    g.cs[j] = c;
    g.sn[j] = sn;
    h[j] = den;
    h[j + 1] = 0.0;
    g.g[j + 1] = -sn * g.g[j];
    g.g[j] = c * g.g[j];
    g.sc[GM_K] = double(j + 1);
    g.sc[GM_INVH] = hn > 0.0 ? 1.0 / hn : 0.0;
    const double est = g.g[j + 1] * g.g[j + 1];
    sc[SC_RR] = est;
    sc[SC_IT] = sc[SC_IT] + 1.0;
    if (est <= sc[SC_TOL2BB] || hn == 0.0) sc[SC_DONE] = 1.0;      // hn = 0: exact in this space
    else if (sc[SC_IT] >= sc[SC_MAXIT]) sc[SC_DONE] = 2.0;
}

// H y = g (k steps of this cycle), then x += Z y
__global__ __launch_bounds__(64) void k_gm_solve(GmDev g) {
    if (threadIdx.x != 0) return;
    const int k = int(g.sc[GM_K]);
    const int ld = g.m + 1;
    for (int i = k - 1; i >= 0; --i) {
        double s = g.g[i];
        for (int q = i + 1; q < k; ++q) s -= g.H[int64_t(q) * ld + i] * g.y[q];
        g.y[i] = s / g.H[int64_t(i) * ld + i];
    }
}

__global__ __launch_bounds__(256) void k_gm_update(Dev d, GmDev g) {
    const int k = int(g.sc[GM_K]);
    if (k == 0) return;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < d.nc; i += int64_t(gridDim.x) * 256) {
        double xi = d.x[i];
        for (int q = 0; q < k; ++q) xi += g.y[q] * g.Z[int64_t(q) * d.nc + i];
        d.x[i] = xi;
    }
}

}  // namespace

size_t gm_layout(int64_t nc, int m, char* base, GmDev& g) {
    size_t off = 0;
    auto carve = [&](size_t count) -> double* {
        off = (off + 255) & ~size_t(255);
        double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
        off += count * sizeof(double);
        return p;
    };
    g.m = m;
    g.V = carve(size_t(m + 1) * nc);
    g.Z = carve(size_t(m) * nc);
    g.H = carve(size_t(m + 1) * m);
    g.cs = carve(m);
    g.sn = carve(m);
    g.g = carve(m + 1);
    g.y = carve(m);
    g.sc = carve(4);
    g.partial = carve(size_t(m + 1) * kGmGrid);
    return (off + 255) & ~size_t(255);
}

hipError_t launch_gm_open(const Dev& d, const GmDev& g, const double* y_kx, double tol, int maxit, bool fresh,
                          hipStream_t s) {
    const unsigned nb = grid_red(d.nc);
    hipLaunchKernelGGL(k_gm_residual, dim3(nb), dim3(256), 0, s, d, g, y_kx);
    hipLaunchKernelGGL(k_gm_open_fin, dim3(1), dim3(1024), 0, s, d, g, int(nb), tol, maxit, fresh ? 1 : 0);
    hipLaunchKernelGGL(k_gm_next, dim3(grid_red(d.nc)), dim3(256), 0, s, d, g, 0);
    return hipGetLastError();
}

hipError_t launch_gm_spmv(const Dev& d, const GmDev& g, int j, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_spmv, dim3(unsigned(d.ntiles)), dim3(d.tile_rows), size_t(d.halo_max) * sizeof(double),
                       s, d, g, j);
    return hipGetLastError();
}

hipError_t launch_gm_orth(const Dev& d, const GmDev& g, int j, hipStream_t s) {
    const unsigned nb = grid_red(d.nc);
    for (int i0 = 0; i0 <= j; i0 += kGmDots) {
        const int cnt = j + 1 - i0 < kGmDots ? j + 1 - i0 : kGmDots;
        hipLaunchKernelGGL(k_gm_dots, dim3(nb), dim3(256), 0, s, d, g, j, i0, cnt);
    }
    hipLaunchKernelGGL(k_gm_hcol, dim3(unsigned(j + 1)), dim3(1024), 0, s, d, g, j, int(nb));
    hipLaunchKernelGGL(k_gm_orth, dim3(nb), dim3(256), 0, s, d, g, j);
    hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(1024), 0, s, d, g, j, int(nb));
    if (j + 1 < g.m) hipLaunchKernelGGL(k_gm_next, dim3(nb), dim3(256), 0, s, d, g, j + 1);
    return hipGetLastError();
}

hipError_t launch_gm_close(const Dev& d, const GmDev& g, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, s, g);
    hipLaunchKernelGGL(k_gm_update, dim3(grid_red(d.nc)), dim3(256), 0, s, d, g);
    return hipGetLastError();
}

}  // namespace mifvm
