// Kernels of the explicit finite-volume residual (eq. (4) of the paper) and
// its Runge-Kutta update (eq. (6)), for CDNA4 wave64.
//
// One residual evaluation is three gather kernels, each owner-computes and
// free of atomics:
//   k_grad_limiter  per cell: least-squares gradient over the node-neighbour
//                   stencil (Algorithm 1), then the Barth-Jespersen limiter
//                   over the 4 face neighbours;
//                   the same kernel computes the vertex values of the
//                   least-squares interpolation (Algorithm 2);
//   k_face_flux     per face: MUSCL upwind convective flux (eq. (15)) minus
//                   the diamond diffusive flux (eq. (diamond)), written once;
//   k_update        per cell: gathers its 4 face fluxes with their signs.
// Ghost values (behind boundary faces) are materialised after every update
// by k_ghost_fill, so every gather is a plain indexed load.
//
// Per-row lists (stencil, vertex lists) are stored in 64-row slices with the
// entry index as the slow dimension, so the index/weight loads of a
// wavefront are one contiguous 256/512-byte segment.
#include "reduce.h"
#include "state.h"

namespace mifvm {

__device__ inline int64_t gtid() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }

inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_ghost_fill(int64_t nc, int64_t nb,
                                                        const int32_t* __restrict__ gowner,
                                                        const int32_t* __restrict__ gtag,
                                                        const double* __restrict__ gdist,
                                                        BcTable bc, double* u) {
    const int64_t g = gtid();
    if (g >= nb) return;
    const int t = gtag[g];
    const int kind = bc.kind[t];
    const double val = bc.value[t];
    const double uo = u[gowner[g]];
    double ug;
    if (kind == kDirichlet) ug = 2.0 * val - uo;
    else if (kind == kNeumann) ug = uo + val * gdist[g];
    else ug = uo;
    u[nc + g] = ug;
}

// One block per tile of d.tile_rows cells.  The tile's halo (every cell and
// ghost its stencils reference) is staged in LDS as (x, y, z, u) records, so
// the ~70 neighbour reads per cell are LDS reads addressed by 16-bit local
// indices; global memory sees one gather per halo entity and the streamed
// local index list.  The same halo holds the cell/ghost list of every vertex
// owned by the tile, so the vertex values of Algorithm 2 are computed here
// too (u_v = sum alpha u_c, entries in the same order as the vertex list).
__global__ __launch_bounds__(kBlock) void k_grad_limiter(Dev d) {
    extern __shared__ double4 sm[];                  // [halo] x, y, z, u
    const int64_t nc = d.nc, NX = d.nc + d.nb, nf = d.nf;
    const int64_t t = blockIdx.x;
    const int T = blockDim.x;
    const int64_t h0 = d.h_off[t];
    const int hn = int(d.h_off[t + 1] - h0);
    const double* __restrict__ X = d.xc;
    const double* __restrict__ Y = d.xc + NX;
    const double* __restrict__ Z = d.xc + 2 * NX;
    const double* __restrict__ u = d.u;
    for (int h = threadIdx.x; h < hn; h += T) {
        const int e = d.h_idx[h0 + h];
        sm[h] = make_double4(X[e], Y[e], Z[e], u[e]);
    }
    __syncthreads();
    for (int64_t v = d.v_off[t] + threadIdx.x; v < d.v_off[t + 1]; v += T) {
        const int64_t vb = d.n_off[v >> 6] + (v & 63);
        const int vw = d.n_w[v >> 6];
        double acc = 0.0;
        for (int k = 0; k < vw; ++k) {
            const int64_t at = vb + int64_t(k) * 64;
            acc += d.n_alpha[at] * sm[d.n_lidx[at]].w;
        }
        d.unode[v] = acc;
    }
    const int64_t i = t * T + threadIdx.x;
    if (i >= nc) return;
    const double4 me = sm[d.h_self[t] + threadIdx.x];
    const double xi = me.x, yi = me.y, zi = me.z, ui = me.w;
    const int64_t s = i >> 6;
    const uint16_t* __restrict__ idx = d.s_lidx + d.s_off[s] + (i & 63);
    const int w = d.s_w[s];
    double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll 4
    for (int k = 0; k < w; ++k) {
        const double4 o = sm[idx[int64_t(k) * 64]];
        const double du = o.w - ui;
        jx += (o.x - xi) * du;
        jy += (o.y - yi) * du;
        jz += (o.z - zi) * du;
    }
    const double* __restrict__ m = d.minv;
    const double m0 = m[i], m1 = m[nc + i], m2 = m[2 * nc + i];
    const double m3 = m[3 * nc + i], m4 = m[4 * nc + i], m5 = m[5 * nc + i];
    const double gx = m0 * jx + m1 * jy + m2 * jz;
    const double gy = m1 * jx + m3 * jy + m4 * jz;
    const double gz = m2 * jx + m4 * jy + m5 * jz;
    d.grad[i] = gx;
    d.grad[nc + i] = gy;
    d.grad[2 * nc + i] = gz;

    // Barth-Jespersen: bounds over the cell and its face neighbours
    double umax = ui, umin = ui;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = sm[d.c2n_l[k * nc + i]].w;
        umax = fmax(umax, v);
        umin = fmin(umin, v);
    }
    double psi = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int f = d.c2f[k * nc + i];
        f = f < 0 ? ~f : f;
        const double dl = gx * (d.fx[f] - xi) + gy * (d.fx[nf + f] - yi) + gz * (d.fx[2 * nf + f] - zi);
        double ph = 1.0;
        if (dl > 0.0) ph = fmin(1.0, (umax - ui) / dl);
        else if (dl < 0.0) ph = fmin(1.0, (umin - ui) / dl);
        psi = fmin(psi, ph);
    }
    d.psi[i] = psi;
}

__global__ __launch_bounds__(kBlock) void k_face_flux(Dev d, BcTable bc, double D) {
    const int64_t f = gtid();
    if (f >= d.nf) return;
    const int64_t nc = d.nc, NX = d.nc + d.nb, nf = d.nf;
    const double* __restrict__ u = d.u;
    int kind = kDirichlet;
    double val = 0.0;
    if (f >= d.nfi) {
        const int t = d.gtag[f - d.nfi];
        kind = bc.kind[t];
        val = bc.value[t];
    }
    if (kind == kZeroFlux) {
        d.flux[f] = 0.0;
        return;
    }
    const int L = d.fL[f], R = d.fR[f];
    const double ph = d.phi[f];
    const int up = ph >= 0.0 ? L : R;
    double uup = u[up];
    if (up < nc) {   // MUSCL reconstruction at the face centroid (ghost side: first order)
        const double rx = d.fx[f] - d.xc[up];
        const double ry = d.fx[nf + f] - d.xc[NX + up];
        const double rz = d.fx[2 * nf + f] - d.xc[2 * NX + up];
        const double gr = d.grad[up] * rx + d.grad[nc + up] * ry + d.grad[2 * nc + up] * rz;
        uup = uup + d.psi[up] * gr;
    }
    double diff;
    if (kind == kNeumann) {
        diff = val * d.area[f];
    } else {
        const double uA = d.unode[d.fA[f]], uB = d.unode[d.fB[f]], uC = d.unode[d.fC[f]];
        diff = d.kAC[f] * (uA - uC) + d.kBC[f] * (uB - uC) + d.kRL[f] * (u[R] - u[L]);
    }
    d.flux[f] = uup * ph - D * diff;
}

// u^(k) = u^n + a dt Res(u^(k-1)); the first stage also saves u^n.
__global__ __launch_bounds__(kBlock) void k_update(Dev d, double a_dt, int first) {
    const int64_t i = gtid();
    if (i >= d.nc) return;
    const int64_t nc = d.nc;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = d.c2f[k * nc + i];
        if (c >= 0) acc += d.flux[c];
        else acc -= d.flux[~c];
    }
    const double res = -acc / d.vol[i] + d.src[i];
    double base;
    if (first) {
        base = d.u[i];
        d.un[i] = base;
    } else {
        base = d.un[i];
    }
    d.u[i] = base + a_dt * res;
}

__global__ __launch_bounds__(kBlock) void k_residual_out(Dev d, double* res) {
    const int64_t i = gtid();
    if (i >= d.nc) return;
    const int64_t nc = d.nc;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = d.c2f[k * nc + i];
        if (c >= 0) acc += d.flux[c];
        else acc -= d.flux[~c];
    }
    res[i] = -acc / d.vol[i] + d.src[i];
}

// phi_f = 1/2 (V_L + V_R) . S_f  (V_L . S_f on the boundary)
__global__ __launch_bounds__(kBlock) void k_face_phi(Dev d) {
    const int64_t f = gtid();
    if (f >= d.nf) return;
    const int64_t nc = d.nc, nf = d.nf;
    const int L = d.fL[f];
    const int R = f < d.nfi ? d.fR[f] : L;
    const double vx = 0.5 * (d.vel[L] + d.vel[R]);
    const double vy = 0.5 * (d.vel[nc + L] + d.vel[nc + R]);
    const double vz = 0.5 * (d.vel[2 * nc + L] + d.vel[2 * nc + R]);
    d.phi[f] = vx * d.S[f] + vy * d.S[nf + f] + vz * d.S[2 * nf + f];
}

__global__ __launch_bounds__(kBlock) void k_to_internal(const int32_t* __restrict__ perm, int64_t n,
                                                         int64_t sin, int64_t sout, int comps,
                                                         const double* __restrict__ src, double* dst) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int64_t o = perm[i];
    for (int c = 0; c < comps; ++c) dst[c * sout + i] = src[c * sin + o];
}

__global__ __launch_bounds__(kBlock) void k_to_user(const int32_t* __restrict__ perm, int64_t n,
                                                     int64_t sin, int64_t sout, int comps,
                                                     const double* __restrict__ src, double* dst) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int64_t o = perm[i];
    for (int c = 0; c < comps; ++c) dst[c * sout + o] = src[c * sin + i];
}

// dt bound: min_i mu_i / sum_{active faces} (|phi_f| + D kRL_f), per block
__global__ __launch_bounds__(kBlock) void k_cfl(Dev d, BcTable bc, double D) {
    __shared__ double lds[4];
    const int64_t nc = d.nc;
    double best = __builtin_huge_val();
    for (int64_t i = gtid(); i < nc; i += int64_t(gridDim.x) * blockDim.x) {
        double rate = 0.0;
        for (int k = 0; k < 4; ++k) {
            int f = d.c2f[k * nc + i];
            f = f < 0 ? ~f : f;
            if (f >= d.nfi && bc.kind[d.gtag[f - d.nfi]] == kZeroFlux) continue;
            rate += fabs(d.phi[f]) + D * d.kRL[f];
        }
        best = fmin(best, d.vol[i] / rate);
    }
    best = block_min256(best, lds);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = best;
}

__global__ __launch_bounds__(kBlock) void k_conservation(Dev d) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int64_t i = gtid(); i < d.nc; i += int64_t(gridDim.x) * blockDim.x) s += d.vol[i] * d.u[i];
    s = block_sum256(s, lds);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = s;
}

// one block: reduce n partials into scal[slot] (op 0 = sum, 1 = min)
__global__ __launch_bounds__(1024) void k_finalize(Dev d, int64_t n, int slot, int op) {
    __shared__ double lds[16];
    const double v = op == 0 ? reduce_partials_sum(d.partial, n, lds) : reduce_partials_min(d.partial, n, lds);
    if (threadIdx.x == 0) d.scal[slot] = v;
}

// ---- launchers ---------------------------------------------------------------
hipError_t launch_ghost_fill(const Dev& d, double* u, const BcTable& bc, hipStream_t s) {
    if (d.nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_fill, dim3(grid_for(d.nb)), dim3(kBlock), 0, s, d.nc, d.nb, d.gowner,
                       d.gtag, d.gdist, bc, u);
    return hipGetLastError();
}

hipError_t launch_grad_limiter(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_limiter, dim3(unsigned(d.ntiles)), dim3(d.tile_rows),
                       size_t(d.halo_max) * sizeof(double4), s, d);
    return hipGetLastError();
}

hipError_t launch_face_flux(const Dev& d, const BcTable& bc, double D, hipStream_t s) {
    hipLaunchKernelGGL(k_face_flux, dim3(grid_for(d.nf)), dim3(kBlock), 0, s, d, bc, D);
    return hipGetLastError();
}

hipError_t launch_update(const Dev& d, double a_dt, bool first_stage, hipStream_t s) {
    hipLaunchKernelGGL(k_update, dim3(grid_for(d.nc)), dim3(kBlock), 0, s, d, a_dt, first_stage ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_residual_out(const Dev& d, double* res, hipStream_t s) {
    hipLaunchKernelGGL(k_residual_out, dim3(grid_for(d.nc)), dim3(kBlock), 0, s, d, res);
    return hipGetLastError();
}

hipError_t launch_face_phi(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_face_phi, dim3(grid_for(d.nf)), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_to_internal(const int32_t* perm, int64_t n, int64_t sin, int64_t sout, int comps,
                              const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_to_internal, dim3(grid_for(n)), dim3(kBlock), 0, s, perm, n, sin, sout, comps,
                       src, dst);
    return hipGetLastError();
}

hipError_t launch_to_user(const int32_t* perm, int64_t n, int64_t sin, int64_t sout, int comps,
                          const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_to_user, dim3(grid_for(n)), dim3(kBlock), 0, s, perm, n, sin, sout, comps, src,
                       dst);
    return hipGetLastError();
}

hipError_t launch_cfl(const Dev& d, const BcTable& bc, double D, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_cfl, dim3(nblk), dim3(kBlock), 0, s, d, bc, D);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, d, int64_t(nblk), int(SC_DT_INV), 1);
    return hipGetLastError();
}

hipError_t launch_conservation(const Dev& d, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_conservation, dim3(nblk), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, d, int64_t(nblk), int(SC_CONS), 0);
    return hipGetLastError();
}

}  // namespace mifvm
