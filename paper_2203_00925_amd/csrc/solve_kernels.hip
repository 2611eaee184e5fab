// Poisson system of the discretisation (Sec. 2.2, eqs. (7), (laplace)):
// on-device assembly into 64-row slices, the sparse product, and the
// Jacobi-preconditioned conjugate-gradient iteration with every scalar kept
// in device memory (alpha, beta and the convergence test are computed by the
// last block of the kernel that produces their partial sums; later kernels
// of an enqueued chunk return at once when the solve has finished).
#include "cg_scalars.h"
#include "reduce.h"
#include "seg.h"
#include "state.h"
#include "halo_stage.h"
#include "xcd.h"

namespace mifvm {

__device__ inline int64_t gtid_s() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
inline int grid_rows(int64_t n) { return int((n + kBlock - 1) / kBlock); }

// Row i of K = -(sum_f s_if dF_f/dP), c_i = sum_f s_if (constant part of F_f),
// where F_f = kAC (P_A - P_C) + kBC (P_B - P_C) + kRL (P_R - P_L) on interior
// and Dirichlet faces, P_v = sum alpha_{v,e} P_e over the vertex list, and a
// ghost value is s_g P_owner + t_g.  Neumann / zero-flux faces carry a fixed
// flux that only enters c.  No atomics: each row is summed by one wavefront.
// FULL = false computes only the diagonal, D^-1 and c (the same sums in the
// same order, the off-diagonal coefficients dropped): what the matrix-free
// solves need, without the stored pattern.
//
// One wavefront per row (four rows per 256-thread block).  All
// of a row's loads go out together: its four faces' data, then the entries of
// its twelve vertex lists, one entry per lane and list.  The row's entries
// are summed in LDS ([row_cap] per wave, columns staged beside them for the
// binary search of a column's slot).  The faces go in order; a vertex list's
// cells are distinct, so their contributions are added by all lanes at once,
// then its ghost entries (mapped to their owners, which may repeat a column)
// one lane after the other in list order, then R and L.  Every sum is in a
// fixed order (deterministic).
__device__ inline double lane_read(double x, int c) {
    const int64_t b = __double_as_longlong(x);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b)), c));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(uint64_t(b) >> 32)), c));
    return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

template <bool FULL>
__global__ __launch_bounds__(256) void k_assemble_rows(Dev d, BcTable bc, int row_cap) {
    extern __shared__ __align__(8) unsigned char asm_raw[];
    constexpr int NONE = -1, DIAG = -2, OFF = -3;         // OFF: off-diagonal, constant part only
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    // XCD-contiguous block order: the 16 blocks of a 64-row slice share one
    // L2, which merges their 8-byte stores into whole lines of the slice
    const int64_t i = xcd_block() * 4 + wv;
    const int64_t nc = d.nc;
    if (i >= nc) return;
    const int64_t s = i >> 6;
    double* acc = reinterpret_cast<double*>(asm_raw) + size_t(wv) * row_cap;
    int32_t* cols = reinterpret_cast<int32_t*>(reinterpret_cast<double*>(asm_raw) + size_t(4) * row_cap) +
                    size_t(wv) * row_cap;
    const int len = FULL ? d.k_len[i] : 0;
    const int w = FULL ? d.k_w[s] : 0;
    if (FULL) {
        const int32_t* __restrict__ kc = d.k_col + d.k_off[s] + (i & 63);
        for (int j = lane; j < len; j += 64) {
            cols[j] = kc[int64_t(j) * 64];
            acc[j] = 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the row's faces: sign, kind, and for diamond faces the three vertices,
    // their weights and R, L (the same on every lane)
    int fcode[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) fcode[k] = d.c2f[k * nc + i];
    int fkind[4], vtx[12], fr[4], fl[4];
    double fsg[4], wts[12], krl[4], nconst[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int f = fcode[k] >= 0 ? fcode[k] : ~fcode[k];
        fsg[k] = fcode[k] >= 0 ? 1.0 : -1.0;
        fkind[k] = f >= d.nfi ? bc.kind[d.gtag[f - d.nfi]] : kDirichlet;
        nconst[k] = fkind[k] == kNeumann ? fsg[k] * (bc.val[f - d.nfi] * d.area[f]) : 0.0;
        const double kac = d.kAC[f], kbc = d.kBC[f];
        krl[k] = d.kRL[f];
        vtx[3 * k] = d.fA[f];
        vtx[3 * k + 1] = d.fB[f];
        vtx[3 * k + 2] = d.fC[f];
        wts[3 * k] = fsg[k] * kac;
        wts[3 * k + 1] = fsg[k] * kbc;
        wts[3 * k + 2] = fsg[k] * (-(kac + kbc));
        fr[k] = d.fR[f];
        fl[k] = d.fL[f];
    }
    // first 64 entries of every list, one per lane, all loads in flight
    int64_t lbase[12];
    int lw[12], le[12];
    double la[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const int v = vtx[q];
        lbase[q] = d.n_off[v >> 6] + (v & 63);
        lw[q] = d.n_w[v >> 6];
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const bool in = lane < lw[q] && fkind[q / 3] == kDirichlet;
        const int64_t at = lbase[q] + int64_t(in ? lane : 0) * 64;
        le[q] = d.n_idx[at];
        la[q] = in ? d.n_alpha[at] : 0.0;
    }
    auto slot_of = [&](int e) -> int {                     // sorted prefix of the row
        int lo = 0, hi = len - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cols[mid] < e) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    double diag = 0.0, cconst = 0.0;                       // the same on every lane
    auto ghost_map = [&](int& e, double& coef, double& cp) {
        const int g = e - int(nc);
        const int kind = bc.kind[d.gtag[g]];
        const double val = bc.val[g];
        const double sg = kind == kDirichlet ? -1.0 : 1.0;
        const double tg = kind == kDirichlet ? 2.0 * val : (kind == kNeumann ? val * d.gdist[g] : 0.0);
        cp = tg * coef;
        coef = sg * coef;
        e = d.gowner[g];
    };
    // one batch of list entries (entry e, weight al on each lane; al = 0: none)
    auto batch = [&](int e, double al, double wq) {
        double coef = wq * al, cp = 0.0;
        bool gh = false;
        int sl = NONE;
        if (al != 0.0) {
            if (e >= nc) {
                ghost_map(e, coef, cp);
                gh = true;
            }
            sl = e == i ? DIAG : (FULL ? slot_of(e) : OFF);
        }
        if (FULL && !gh && sl >= 0) acc[sl] += coef;       // distinct cells: distinct entries
        const uint64_t dm = __ballot(!gh && sl == DIAG);   // the row's own cell
        if (dm) diag += lane_read(coef, __builtin_ctzll(dm));
        uint64_t gm = __ballot(gh);
        while (gm) {
            const int c = __builtin_ctzll(gm);
            gm &= gm - 1;
            const int sc = __builtin_amdgcn_readlane(sl, c);
            const double vc = lane_read(coef, c);
            cconst += lane_read(cp, c);
            if (sc == DIAG) diag += vc;
            else if (FULL && sc >= 0 && lane == 0) acc[sc] += vc;
        }
    };
    auto single = [&](int e, double coef) {                // R or L of a face
        double cp = 0.0;
        if (e >= nc) {
            ghost_map(e, coef, cp);
            cconst += cp;
        }
        if (e == i) diag += coef;
        else if (FULL) {
            const int sl = slot_of(e);
            if (lane == 0) acc[sl] += coef;
        }
    };
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (fkind[k] != kDirichlet) {                      // Neumann / zero flux: a fixed flux
            cconst += nconst[k];
            continue;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int q = 3 * k + a;
            batch(le[q], la[q], wts[q]);
            for (int k0 = 64; k0 < lw[q]; k0 += 64) {      // lists longer than a wavefront
                const bool in = k0 + lane < lw[q];
                const int64_t at = lbase[q] + int64_t(in ? k0 + lane : 0) * 64;
                batch(d.n_idx[at], in ? d.n_alpha[at] : 0.0, wts[q]);
            }
        }
        single(fr[k], fsg[k] * krl[k]);
        single(fl[k], -fsg[k] * krl[k]);
    }
    if (FULL) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double* __restrict__ vals = d.k_val + d.k_off[s] + (i & 63);
        for (int k = lane; k < w; k += 64) vals[int64_t(k) * 64] = k < len ? -acc[k] : 0.0;
    }
    if (lane == 0) {
        d.k_diag[i] = -diag;
        d.k_dinv[i] = 1.0 / (-diag);
        d.k_c[i] = cconst;
    }
}

__device__ inline double spmv_row(const Dev& d, const double* __restrict__ x, int64_t i) {
    const int64_t s = i >> 6;
    const int64_t base = d.k_off[s] + (i & 63);
    const int w = d.k_w[s];
    double y = d.k_diag[i] * x[i];
    for (int k = 0; k < w; ++k) {
        const int64_t at = base + int64_t(k) * 64;
        y += d.k_val[at] * x[d.k_col[at]];
    }
    return y;
}

__global__ __launch_bounds__(kBlock) void k_spmv(Dev d, const double* __restrict__ x, double* y) {
    const int64_t i = gtid_s();
    if (i >= d.nc) return;
    y[i] = spmv_row(d, x, i);
}

// b = -mu f + c
__global__ __launch_bounds__(kBlock) void k_rhs(Dev d, const double* __restrict__ f) {
    const int64_t i = gtid_s();
    if (i >= d.nc) return;
    d.b[i] = -d.vol[i] * f[i] + d.k_c[i];
}

// Every CG quantity is per mesh (a batch holds independent meshes): a row
// reads the scalars of its own mesh, rows of a mesh whose solve has finished
// (SC_DONE != 0) are left untouched, and a block whose meshes have all
// finished returns at once, so a chunk of enqueued iterations past
// convergence costs only launches.

// r = b - K x; z = D^-1 r; p = z; partial rz, rr, bb.  (Re)opens the loop.
// kx: K x already computed (matrix-free), or null for the stored K.
__global__ __launch_bounds__(kBlock) void k_cg_setup(Dev d, const double* __restrict__ kx) {
    __shared__ double lds[4];
    const int64_t i = gtid_s();
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    double v[3] = {0.0, 0.0, 0.0};
    if (i < d.nc) {
        const double bi = d.b[i];
        const double ri = bi - (kx ? kx[i] : spmv_row(d, d.x, i));
        const double zi = d.k_dinv[i] * ri;
        d.r[i] = ri;
        d.z[i] = zi;
        d.p[i] = zi;
        v[0] = ri * zi;
        v[1] = ri * ri;
        v[2] = bi * bi;
    }
    seg_publish<3>(d, g, v, i >= g.split, lds);
}

// One block per mesh.  fresh != 0: a new solve (sets tolerance, limits,
// count); otherwise a reopen after a true-residual check or a restart keeps
// them.
__global__ __launch_bounds__(1024) void k_cg_setup_fin(Dev d, int64_t nparts, double tol, int maxit,
                                                       int restart, int fresh) {
    __shared__ double lds[16];
    const int m = blockIdx.x;
    const double trz = seg_sum(d, 0, m, nparts, kBlock, lds);
    const double trr = seg_sum(d, 1, m, nparts, kBlock, lds);
    const double tbb = seg_sum(d, 2, m, nparts, kBlock, lds);
    if (threadIdx.x == 0) {
        double* sc = msc(d, m);
        sc[SC_RZ] = trz;
        sc[SC_RR] = trr;
        sc[SC_TRUE_RR] = trr;
        sc[SC_BB] = tbb;
        if (fresh) {
            sc[SC_TOL2BB] = tol * tol * tbb;
            sc[SC_MAXIT] = double(maxit);
            sc[SC_RESTART] = double(restart);
            sc[SC_IT] = 0.0;
        }
        sc[SC_SINCE] = 0.0;
        sc[SC_DONE] = (trr <= sc[SC_TOL2BB] || tbb == 0.0) ? 1.0 : (sc[SC_IT] >= sc[SC_MAXIT] ? 2.0 : 0.0);
    }
}

// q = K p; partial p . q.  One block per cell tile: the tile's halo of p is
// staged in LDS (ghost halo entries are not unknowns and read as 0) and the
// rows address it with 16-bit local indices; the same entries in the same
// order as spmv_row, so the result is bitwise the same.
__global__ __launch_bounds__(kBlock) void k_cg_spmv(Dev d) {
    extern __shared__ double sp[];                   // [halo] p
    __shared__ double lds[4];
    const int64_t nc = d.nc;
    const int64_t t = blockIdx.x;
    const int T = blockDim.x;
    const BlockSeg g = block_seg(d, t * T, T);
    if (block_done(d, g)) return;
    stage_halo_values(d, t, d.p, sp);
    __syncthreads();
    const int64_t i = t * T + threadIdx.x;
    const int m = row_mesh(g, i);
    double v[1] = {0.0};
    if (i < nc && msc(d, m)[SC_DONE] == 0.0) {
        const double pi = sp[d.h_self[t] + threadIdx.x];
        const int64_t s = i >> 6;
        const int64_t base = d.k_off[s] + (i & 63);
        const int w = d.k_w[s];
        double y = d.k_diag[i] * pi;
        // 16 entries' loads in flight, then their sums in row order
        for (int k0 = 0; k0 < w; k0 += 16) {
            uint16_t l[16];
            double a[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const bool in = k0 + j < w;
                const int64_t at = base + int64_t(k0 + j) * 64;
                l[j] = in ? d.k_lidx[at] : uint16_t(0);
                a[j] = in ? d.k_val[at] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (k0 + j < w) y += a[j] * sp[l[j]];   // w is one slice's: uniform over the wave
        }
        d.q[i] = y;
        v[0] = pi * y;
    }
    seg_publish<1>(d, g, v, i >= g.split, lds);
}

// x += alpha p; r -= alpha q; z = D^-1 r; partial rz, rr
__global__ __launch_bounds__(kBlock) void k_cg_axpy(Dev d) {
    __shared__ double lds[4];
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    if (block_done(d, g)) return;
    const int64_t i = gtid_s();
    const int m = row_mesh(g, i);
    const double* sc = msc(d, m);
    double v[2] = {0.0, 0.0};
    if (i < d.nc && sc[SC_DONE] == 0.0) {
        const double alpha = sc[SC_ALPHA];
        d.x[i] = d.x[i] + alpha * d.p[i];
        const double ri = d.r[i] - alpha * d.q[i];
        const double zi = d.k_dinv[i] * ri;
        d.r[i] = ri;
        d.z[i] = zi;
        v[0] = ri * zi;
        v[1] = ri * ri;
    }
    seg_publish<2>(d, g, v, i >= g.split, lds);
}

// p = z + beta p
__global__ __launch_bounds__(kBlock) void k_cg_dir(Dev d) {
    const BlockSeg g = block_seg(d, int64_t(blockIdx.x) * kBlock, kBlock);
    if (block_done(d, g)) return;
    const int64_t i = gtid_s();
    if (i >= d.nc) return;
    const double* sc = msc(d, row_mesh(g, i));
    if (sc[SC_DONE] != 0.0) return;
    d.p[i] = d.z[i] + sc[SC_BETA] * d.p[i];
}

// ---- launchers ---------------------------------------------------------------
hipError_t launch_assemble(const Dev& d, const BcTable& bc, int row_max, hipStream_t s) {
    const int cap = row_max > 0 ? row_max : 1;
    if (size_t(4) * cap * (sizeof(double) + sizeof(int32_t)) > 65536) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_assemble_rows<true>, dim3(rows_m(d.nc, 4)), dim3(256),
                       size_t(4) * cap * (sizeof(double) + sizeof(int32_t)), s, d, bc, cap);
    return hipGetLastError();
}

hipError_t launch_assemble_consts(const Dev& d, const BcTable& bc, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble_rows<false>, dim3(rows_m(d.nc, 4)), dim3(256), 0, s, d, bc, 1);
    return hipGetLastError();
}

hipError_t launch_spmv_plain(const Dev& d, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_spmv, dim3(grid_rows(d.nc)), dim3(kBlock), 0, s, d, x, y);
    return hipGetLastError();
}

hipError_t launch_rhs(const Dev& d, const double* f, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, dim3(grid_rows(d.nc)), dim3(kBlock), 0, s, d, f);
    return hipGetLastError();
}

hipError_t launch_cg_setup(const Dev& d, double tol, int maxit, int restart, bool fresh, hipStream_t s,
                           const double* kx) {
    const int nb = grid_rows(d.nc);
    hipLaunchKernelGGL(k_cg_setup, dim3(nb), dim3(kBlock), 0, s, d, kx);
    hipLaunchKernelGGL(k_cg_setup_fin, dim3(d.nm), dim3(1024), 0, s, d, int64_t(nb), tol, maxit, restart,
                       fresh ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_cg_spmv(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_spmv, dim3(unsigned(d.ntiles)), dim3(d.tile_rows),
                       size_t(d.halo_max) * sizeof(double), s, d);
    hipLaunchKernelGGL(k_cg_alpha<0>, dim3(d.nm), dim3(1024), 0, s, d, d.ntiles, int64_t(d.tile_rows));
    return hipGetLastError();
}

hipError_t launch_cg_axpy(const Dev& d, hipStream_t s) {
    const int nb = grid_rows(d.nc);
    hipLaunchKernelGGL(k_cg_axpy, dim3(nb), dim3(kBlock), 0, s, d);
    hipLaunchKernelGGL(k_cg_beta<0>, dim3(d.nm), dim3(1024), 0, s, d, int64_t(nb), int64_t(kBlock));
    return hipGetLastError();
}

hipError_t launch_cg_dir(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dir, dim3(grid_rows(d.nc)), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

}  // namespace mifvm
