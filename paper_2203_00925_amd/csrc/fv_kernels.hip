// Kernels of the explicit finite-volume residual (eq. (4) of the paper) and
// its Runge-Kutta update (eq. (6)), for CDNA4 wave64.
//
// A Runge-Kutta stage is two gather kernels, each owner-computes and free
// of atomics:
//   k_grad_moments  per tile of cells: least-squares gradient (Algorithm 1,
//                   in star-moment form), then the Barth-Jespersen limiter
//                   over the 4 face neighbours and the MUSCL values at the
//                   cell's face centroids; the same kernel computes the
//                   vertex values of the least-squares interpolation
//                   (Algorithm 2);
//   k_cell_step     per cell: the upwind convective fluxes (eq. (15)) minus
//                   the diamond diffusive fluxes (eq. (diamond)) of its four
//                   faces, summed, and the stage update.
// The residual evaluation that returns the face fluxes runs the face kernel
// k_face_flux (one thread per face) after the gradient kernel instead.
// Ghost values (behind boundary faces) are materialised by k_ghost_fill
// before a run of steps and by k_cell_step after every stage, so every
// gather is a plain indexed load.
//
// Every kernel is instantiated for FP64 (the method as stated) and FP32 (the
// reduced-precision form: state, gradients, fluxes and geometry copies in
// FP32; in LDS the FP32 form keeps positions relative to the tile's first
// cell, computed in FP64, so differences of nearby positions keep their
// digits).  Sums that must stay FP64 (conservation, the CFL bound) read the
// FP64 geometry.
//
// Per-row lists (stencil, vertex lists) are stored in 64-row slices with the
// entry index as the slow dimension, so the index/weight loads of a
// wavefront are one contiguous 128/256/512-byte segment.
#include <type_traits>

#include "reduce.h"
#include "seg.h"
#include "state.h"
#include "xcd.h"

namespace mifvm {

__device__ inline int64_t gtid() { return int64_t(blockIdx.x) * blockDim.x + threadIdx.x; }

inline int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

template <class R> struct Vec4T;
template <> struct Vec4T<double> { using T = double4; };
template <> struct Vec4T<float> { using T = float4; };
template <class R> struct Vec2T;
template <> struct Vec2T<double> { using T = double2; };
template <> struct Vec2T<float> { using T = float2; };

__device__ inline double4 mk4(double x, double y, double z, double w) { return make_double4(x, y, z, w); }
__device__ inline float4 mk4(float x, float y, float z, float w) { return make_float4(x, y, z, w); }
__device__ inline double2 mk2(double x, double y) { return make_double2(x, y); }
__device__ inline float2 mk2(float x, float y) { return make_float2(x, y); }

template <class R>
__global__ __launch_bounds__(kBlock) void k_ghost_fill(int64_t nc, int64_t nb,
                                                        const int32_t* __restrict__ gowner,
                                                        const int32_t* __restrict__ gtag,
                                                        const R* __restrict__ gdist, BcTable bc, R* u) {
    const int64_t g = gtid();
    if (g >= nb) return;
    const int t = gtag[g];
    const int kind = bc.kind[t];
    const R val = bc_value<R>(bc, g);
    const R uo = u[gowner[g]];
    R ug;
    if (kind == kDirichlet) ug = R(2) * val - uo;
    else if (kind == kNeumann) ug = uo + val * gdist[g];
    else ug = uo;
    u[nc + g] = ug;
}

// Stage tile t's halo in LDS (positions relative to `ref`) as two 16-byte
// arrays, (x, y) and (z, u): random reads of 16-byte items spread over twice
// as many LDS bank groups as the halves of 32-byte records would.  Each
// thread's 8 index loads go out together, then its 8 gathers, then the LDS
// stores; `from` skips the part already staged.
template <class R>
struct HaloSoA {
    using V2 = typename Vec2T<R>::T;
    using V4 = typename Vec4T<R>::T;
    V2* xy;
    V2* zu;
    __device__ V4 operator[](int l) const {
        const V2 a = xy[l], b = zu[l];
        return mk4(a.x, a.y, b.x, b.y);
    }
};

template <class R>
__device__ inline void stage_halo_soa(const Dev& d, const R* __restrict__ u, HaloSoA<R> sm, int64_t t, double4 ref,
                                      int from = 0) {
    const int T = blockDim.x;
    const int64_t h0 = d.h_off[t];
    const int hn = int(d.h_off[t + 1] - h0);
    const double4* __restrict__ P = d.xyz4;
    for (int hb = from; hb < hn; hb += 8 * T) {
        int e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int h = hb + j * T + threadIdx.x;
            e[j] = d.h_idx[h0 + (h < hn ? h : 0)];
        }
        double4 r[8];
        R ue[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            r[j] = P[e[j]];
            ue[j] = u[e[j]];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int h = hb + j * T + threadIdx.x;
            if (h < hn) {
                sm.xy[h] = mk2(R(r[j].x - ref.x), R(r[j].y - ref.y));
                sm.zu[h] = mk2(R(r[j].z - ref.z), ue[j]);
            }
        }
    }
}

// ---- gradient in star-moment form ------------------------------------------
// The sum of Algorithm 1, J_i = sum_{j in N(i)} (x_j - x_i)(u_j - u_i) over
// the node-neighbour stencil N(i) (every cell and ghost sharing a vertex
// with i), rewritten exactly.  An entity sharing m vertices with i lies in m
// of i's 4 vertex lists, so with T_L(i) = sum_{j in L} (x_j - x_i)(u_j - u_i)
//   J_i = sum_{v of i} T_{L(v)}(i) - sum_{j sharing only an edge} (.) - 2 sum_{face nbrs} (.)
// (i itself adds zeros).  For a list L of n entities with mean position xb,
// mean value ub and centred moment C = sum (x_j - xb)(u_j - ub),
//   T_L(i) = C + n (xb - x_i)(ub - u_i).
// Each list is summed once per vertex instead of once per cell of its ~24
// cells, and a cell reads 4 vertex records, its 4 face neighbours and ~13
// edge neighbours instead of ~70 stencil entries.  Every term is a product
// of differences of nearby values, so no large value cancels.
//
// One block per tile of d.tile_rows cells.  The tile's halo (every cell and
// ghost the tile's stencils reference) is staged in LDS and addressed by
// 16-bit local indices, so global memory sees one gather per halo entity and
// streamed index lists.  Every vertex the tile's cells touch (its own, then the foreign ones, whose lists
// lie in the same halo) gets its record (xb, n), (C, ub) in LDS, from sums
// shifted by the list's first entry (pad entries repeat it and add zeros):
//   s = sum (x_j - x_0), q = sum (u_j - u_0), c = sum (x_j - x_0)(u_j - u_0),
//   xb = x_0 + s/n, ub = u_0 + q/n, C = c - s q/n;
// own vertices also store u_v = sum alpha u_j (Algorithm 2).
template <class R, bool PARTS>
__global__ __launch_bounds__(kBlock) void k_grad_moments(Dev d, FvArrays<R> a) {
    using V2 = typename Vec2T<R>::T;
    using V4 = typename Vec4T<R>::T;
    extern __shared__ __align__(16) unsigned char sm_raw[];
    // [halo] (x, y), [halo] (z, u), then the touched vertices' records as
    // four 16-byte arrays (xb_x, xb_y), (xb_z, n), (C_x, C_y), (C_z, ub): a
    // random vertex's first 16 bytes then fall in any of 8 bank groups, not 2
    const int hcap = (d.halo_max + 1) & ~1;
    const HaloSoA<R> sm{reinterpret_cast<V2*>(sm_raw), reinterpret_cast<V2*>(sm_raw) + hcap};
    const int tvc = d.tv_max;
    V2* va = sm.zu + hcap;
    V2* vb = va + tvc;
    V2* vc = vb + tvc;
    V2* vd = vc + tvc;
    constexpr bool rel = std::is_same<R, float>::value;
    const int64_t nc = d.nc;
    const int64_t t = xcd_block();
    if (t >= d.ntiles) return;
    const int T = blockDim.x;
    const int64_t i = t * T + threadIdx.x;
    const bool cell = i < nc;
    const int lself = d.h_self[t] + threadIdx.x;

    // Global loads are issued in two waves before the first barrier, so the
    // tile pays about two memory latencies before its LDS work: first every
    // load that depends on no other (the first 8T halo indices, the cell's
    // tables, the slice headers of its edge-neighbour list and of the vertex
    // list it will sum), then the loads addressed by those (the halo
    // gathers, the first batches of both lists).  Out-of-range slots read a
    // valid address and are discarded, so no load sits under a branch.
    const int64_t h0 = d.h_off[t];
    const int hn = int(d.h_off[t + 1] - h0);
    int he[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int h = j * T + threadIdx.x;
        he[j] = d.h_idx[h0 + (h < hn ? h : 0)];
    }
    const int64_t ic = cell ? i : nc - 1;
    uint16_t nl[4], lv[4];
    int fc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        fc[k] = d.c2f[k * nc + ic];
        nl[k] = d.c2n_l[k * nc + ic];
        lv[k] = d.c2v_l[k * nc + ic];
    }
    const int64_t eoff = d.e_off[ic >> 6];
    const int ew = cell ? d.e_w[ic >> 6] : 0;

    const int64_t v0 = d.v_off[t], f0 = d.fv_off[t];
    const int own = int(d.v_off[t + 1] - v0), nfor = int(d.fv_off[t + 1] - f0);
    int r = threadIdx.x;
    bool mine = true;
    int64_t row = 0, vbase = 0;
    int vw = 0, vn = 1;
    const uint16_t* __restrict__ li = d.n_lidx;
    constexpr int VB = 8;               // vertex-list entries per batch
    uint16_t vl[VB];
    R val[VB];
    // row meta of vertex row r (threads past the rows read row 0 of the
    // tile-owned lists and sum nothing)
    auto vmeta = [&]() {
        const bool act = r < own + nfor;
        mine = !act || r < own;
        row = !act ? 0 : (mine ? v0 + r : f0 + (r - own));
        const int64_t sl = row >> 6;
        const int64_t* __restrict__ op = mine ? d.n_off : d.f_off;
        const int32_t* __restrict__ wp = mine ? d.n_w : d.f_w;
        const int32_t* __restrict__ np = mine ? d.n_len : d.fv_len;
        vbase = op[sl] + (row & 63);
        vw = act ? wp[sl] : 0;
        vn = np[row];
        li = mine ? d.n_lidx : d.f_lidx;
    };
    auto vbatch = [&]() {
#pragma unroll
        for (int j = 0; j < VB; ++j) {
            const bool in = j < vw;
            vl[j] = in ? li[vbase + int64_t(j) * 64] : uint16_t(0);
            val[j] = (mine && in) ? a.n_alpha[vbase + int64_t(j) * 64] : R(0);
        }
    };
    vmeta();

    const double4* __restrict__ P = d.xyz4;
    double4 hp[8];
    R hu[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        hp[j] = P[he[j]];
        hu[j] = a.u[he[j]];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) fc[k] = fc[k] < 0 ? ~fc[k] : fc[k];
    const uint16_t* __restrict__ eidx = d.e_lidx + (cell ? eoff + (i & 63) : 0);
    constexpr int EB = 16;              // edge-only neighbours per batch
    uint16_t el[EB];
#pragma unroll
    for (int j = 0; j < EB; ++j) el[j] = j < ew ? eidx[int64_t(j) * 64] : uint16_t(lself);
    vbatch();

    const double4 ref = rel ? d.xyz4[t * T] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int h = j * T + threadIdx.x;
        if (h < hn) {
            sm.xy[h] = mk2(R(hp[j].x - ref.x), R(hp[j].y - ref.y));
            sm.zu[h] = mk2(R(hp[j].z - ref.z), hu[j]);
        }
    }
    if (hn > 8 * T) stage_halo_soa<R>(d, a.u, sm, t, ref, 8 * T);
    __syncthreads();

    for (; r < own + nfor; r += T) {
        if (r != int(threadIdx.x)) {
            vmeta();
            vbatch();
        }
        const uint16_t l0 = vl[0];
        const V4 q0 = sm[l0];
        R un = R(0), sx = R(0), sy = R(0), sz = R(0), su = R(0), cx = R(0), cy = R(0), cz = R(0);
        for (int k0 = 0; k0 < vw; k0 += VB) {
            // next batch in flight while this one is summed (pad = first entry)
            uint16_t nlx[VB];
            R nal[VB];
#pragma unroll
            for (int j = 0; j < VB; ++j) {
                const bool in = k0 + VB + j < vw;
                const int64_t at = vbase + int64_t(k0 + VB + j) * 64;
                nlx[j] = in ? li[at] : l0;
                nal[j] = (mine && in) ? a.n_alpha[at] : R(0);
            }
#pragma unroll
            for (int j = 0; j < VB; ++j) {
                const V4 q = sm[k0 + j < vw ? vl[j] : l0];
                const R dx = q.x - q0.x, dy = q.y - q0.y, dz = q.z - q0.z, du = q.w - q0.w;
                un += val[j] * q.w;
                sx += dx; sy += dy; sz += dz; su += du;
                cx += dx * du; cy += dy * du; cz += dz * du;
            }
#pragma unroll
            for (int j = 0; j < VB; ++j) {
                vl[j] = nlx[j];
                val[j] = nal[j];
            }
        }
        const R inv = R(1) / R(vn);
        const R mu = su * inv;
        va[r] = mk2(q0.x + sx * inv, q0.y + sy * inv);
        vb[r] = mk2(q0.z + sz * inv, R(vn));
        vc[r] = mk2(cx - sx * mu, cy - sy * mu);
        vd[r] = mk2(cz - sz * mu, q0.w + mu);
        if (mine) a.unode[row] = un;
    }
    // loads used at the end (limiter, M^-1) go out before the barrier
    double4 xf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) xf[k] = d.fx4[fc[k]];
    const R* __restrict__ m = a.minv;
    const R m0 = m[ic], m1 = m[nc + ic], m2 = m[2 * nc + ic];
    const R m3 = m[3 * nc + ic], m4 = m[4 * nc + ic], m5 = m[5 * nc + ic];
    __syncthreads();
    if (!cell) return;

    const V4 me = sm[lself];
    const R xi = me.x, yi = me.y, zi = me.z, ui = me.w;
    R jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const V2 pa = va[lv[k]], pb = vb[lv[k]], pc = vc[lv[k]], pd = vd[lv[k]];
        const V4 vs = mk4(pa.x, pa.y, pb.x, pb.y), vm = mk4(pc.x, pc.y, pd.x, pd.y);
        const R nd = vs.w * (vm.w - ui);
        jx += vm.x + (vs.x - xi) * nd;
        jy += vm.y + (vs.y - yi) * nd;
        jz += vm.z + (vs.z - zi) * nd;
    }
    R umax = ui, umin = ui;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const V4 o = sm[nl[k]];
        const R du2 = R(2) * (o.w - ui);
        jx -= (o.x - xi) * du2;
        jy -= (o.y - yi) * du2;
        jz -= (o.z - zi) * du2;
        umax = fmax(umax, o.w);
        umin = fmin(umin, o.w);
    }
    // edge-only neighbours (slice padding = the cell itself, which adds zeros)
    for (int k0 = 0; k0 < ew; k0 += EB) {
        uint16_t nx[EB];
#pragma unroll
        for (int j = 0; j < EB; ++j)
            nx[j] = k0 + EB + j < ew ? eidx[int64_t(k0 + EB + j) * 64] : uint16_t(lself);
#pragma unroll
        for (int j = 0; j < EB; ++j) {
            if (k0 + j < ew) {          // uniform over the wave (one slice)
                const V4 o = sm[el[j]];
                const R du = o.w - ui;
                jx -= (o.x - xi) * du;
                jy -= (o.y - yi) * du;
                jz -= (o.z - zi) * du;
            }
        }
#pragma unroll
        for (int j = 0; j < EB; ++j) el[j] = nx[j];
    }
    const R gx = m0 * jx + m1 * jy + m2 * jz;
    const R gy = m1 * jx + m3 * jy + m4 * jz;
    const R gz = m2 * jx + m4 * jy + m5 * jz;
    R psi = R(1), dl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dl[k] = gx * (R(xf[k].x - ref.x) - xi) + gy * (R(xf[k].y - ref.y) - yi) + gz * (R(xf[k].z - ref.z) - zi);
        R ph = R(1);
        if (dl[k] > R(0)) ph = fmin(R(1), (umax - ui) / dl[k]);
        else if (dl[k] < R(0)) ph = fmin(R(1), (umin - ui) / dl[k]);
        psi = fmin(psi, ph);
    }
    // The step: the MUSCL value u + psi g.(x_f - x_i) at each of the cell's
    // face centroids (in c2f order), which the cell step reads for both sides
    // of a face.  With parts: the gradient and limiter arrays, which the face
    // kernel reads.
    if constexpr (!PARTS) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.uf[k * nc + i] = ui + psi * dl[k];
    } else {
        a.grad[i] = gx;
        a.grad[nc + i] = gy;
        a.grad[2 * nc + i] = gz;
        a.psi[i] = psi;
    }
}

// One thread per face (the residual evaluation; it reads
// the gradient and limiter arrays).  Every load of the face goes out before
// its first branch (boundary faces read a valid dummy where they need no
// data); the arithmetic of each kind of face is unchanged by that.
template <class R>
__global__ __launch_bounds__(kBlock) void k_face_flux(Dev d, FvArrays<R> a, BcTable bc) {
    const int64_t f = gtid();
    if (f >= d.nf) return;
    const int64_t nc = d.nc, NX = d.nc + d.nb, nf = d.nf;
    const R* __restrict__ u = a.u;
    const bool bnd = f >= d.nfi;
    const int64_t g = bnd ? f - d.nfi : 0;
    const int kind = bnd ? bc.kind[d.gtag[g]] : kDirichlet;
    const R val = bnd ? bc_value<R>(bc, g) : R(0);
    const R area = bnd ? a.area[f] : R(0);            // used on Neumann faces only
    const int L = d.fL[f], Rc = d.fR[f];
    const R D = R(d.mesh_D[mesh_of(d, L)]);
    const R ph = a.phi[f];
    const R fxx = a.fx[f], fxy = a.fx[nf + f], fxz = a.fx[2 * nf + f];
    const R cAC = a.kAC[f], cBC = a.kBC[f], cRL = a.kRL[f];
    const int iA = d.fA[f], iB = d.fB[f], iC = d.fC[f];
    const R uL = u[L], uR = u[Rc];
    const R uA = a.unode[iA], uB = a.unode[iB], uC = a.unode[iC];
    const int up = ph >= R(0) ? L : Rc;
    const bool cellside = up < nc;          // MUSCL on a cell side; a ghost side is first order
    const int uc = cellside ? up : L;
    const R rx = fxx - a.xc[uc];
    const R ry = fxy - a.xc[NX + uc];
    const R rz = fxz - a.xc[2 * NX + uc];
    const R gr = a.grad[uc] * rx + a.grad[nc + uc] * ry + a.grad[2 * nc + uc] * rz;
    const R uupc = up == L ? uL : uR;
    const R uup = cellside ? uupc + a.psi[uc] * gr : uupc;
    const R diff = kind == kNeumann ? val * area : cAC * (uA - uC) + cBC * (uB - uC) + cRL * (uR - uL);
    a.flux[f] = kind == kZeroFlux ? R(0) : uup * ph - D * diff;
}

// ---- the step: face fluxes and update in one pass per cell ------------------
// The residual of cell i is -(1/vol_i) sum_k s_k F_k + src_i over its four
// faces, s_k = +1 where the cell is the face's L side.  On the interior
// faces the diffusive parts are regrouped per cell as in the matrix-free
// product: a face of a tetrahedron holds three of the cell's four vertices,
// so sum_k s_k (kAC (u_A - u_C) + kBC (u_B - u_C)) = sum_v w_v u_node[v], and
// s_k kRL (u_R - u_L) = kRL (u_n - u_i) with n the cell across face k.  The
// convective part is (s_k phi_f) times the upwind side's MUSCL value at the
// face centroid, which the gradient kernel stores per cell and face: uf[k][i]
// on the cell's side, uf[j][n] across (j = the face's slot among n's
// faces).  Both cells of a face take the same upwind value, so its
// convective parts cancel exactly in the sum over cells.  Boundary faces
// (the cell is always their L side) are evaluated as in k_face_flux.

// the tables: geometry only, built once per state
__global__ __launch_bounds__(kBlock) void k_fv_cell_setup(Dev d) {
    const int64_t i = gtid();
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
    uint32_t slots = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int code = d.c2f[k * nc + i];
        const int f = code >= 0 ? code : ~code;
        const double sg = code >= 0 ? 1.0 : -1.0;
        const bool in = f < d.nfi;
        // a boundary face only places its vertices (weight 0): every vertex
        // of the cell gets a slot
        const double on = in ? sg : 0.0;
        const double kac = d.kAC[f], kbc = d.kBC[f];
        add(d.fA[f], on * kac);
        add(d.fB[f], on * kbc);
        add(d.fC[f], on * (-(kac + kbc)));
        r[k] = in ? d.kRL[f] : 0.0;
        const int n = in ? d.c2n[k * nc + i] : int(i);
        uint32_t j = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cn = d.c2f[q * nc + n];
            if ((cn >= 0 ? cn : ~cn) == f) j = uint32_t(q);
        }
        slots |= (in ? j : 0u) << (2 * k);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        d.fvc_vid[q * nc + i] = vid[q] >= 0 ? vid[q] : vid[0];
        d.fvc_w[q * nc + i] = w[q];
        d.fvc_r[q * nc + i] = r[q];
        d.fvc_w32[q * nc + i] = float(w[q]);
        d.fvc_r32[q * nc + i] = float(r[q]);
    }
    d.fvc_slot[i] = uint8_t(slots);
}

// u_out[i] = u[i] + alpha dt Res(u_in)_i (u holds u^n; u_in and u_out are
// other buffers, or u_out = u on the last stage, whose cell i alone reads
// u[i]); then the ghosts behind the cell's boundary faces, from the new value
template <class R>
__global__ __launch_bounds__(kBlock) void k_cell_step(Dev d, FvArrays<R> a, BcTable bc, const R* __restrict__ uin,
                                                      R* uout, double alpha) {
    const int64_t i = gtid_m();                        // XCD-contiguous block order
    if (i >= d.nc) return;
    const int64_t nc = d.nc;
    const int m = mesh_of(d, i);
    // the cell's tables go out first (coalesced), then the gathers they
    // address; the neighbour's face value only on lanes where it is the
    // upwind side (the gathers' address work is what bounds this kernel)
    int nb[4], vid[4];
    R w[4], r[4], uo[4], po[4];
    const uint32_t sl = d.fvc_slot[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        nb[k] = d.c2n[k * nc + i];
        vid[k] = d.fvc_vid[k * nc + i];
        w[k] = a.cw[k * nc + i];
        r[k] = a.cr[k * nc + i];
        uo[k] = a.uf[k * nc + i];
        po[k] = a.cphi[k * nc + i];                    // outward
    }
    const R ui = uin[i], base = a.u[i], vol = a.vol[i], src = a.src[i];
    const R D = R(d.mesh_D[m]), a_dt = R(alpha * d.mesh_dt[m]);
    R un[4], ux[4], uv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        un[k] = uin[nb[k]];                            // a ghost's value behind a boundary face
        uv[k] = a.unode[vid[k]];
        ux[k] = R(0);
        if (nb[k] < nc && po[k] < R(0)) ux[k] = a.uf[int64_t((sl >> (2 * k)) & 3u) * nc + nb[k]];
    }
    R dif = R(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) dif += w[k] * uv[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) dif += r[k] * (un[k] - ui);
    R conv = R(0);
    bool bnd = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool in = nb[k] < nc;
        bnd = bnd || !in;
        conv += in ? po[k] * (po[k] >= R(0) ? uo[k] : ux[k]) : R(0);
    }
    R acc = conv - D * dif;
    if (bnd) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (nb[k] < nc) continue;
            const int64_t g = nb[k] - nc;              // the cell is the L side of its boundary faces
            const int64_t f = d.nfi + g;
            const int kind = bc.kind[d.gtag[g]];
            if (kind == kZeroFlux) continue;
            // upwind: the cell's MUSCL value, or the ghost's value (first order)
            const R uup = po[k] >= R(0) ? uo[k] : un[k];
            R diff;
            if (kind == kNeumann) {
                diff = bc_value<R>(bc, g) * a.area[f];
            } else {
                const R uA = a.unode[d.fA[f]], uB = a.unode[d.fB[f]], uC = a.unode[d.fC[f]];
                diff = a.kAC[f] * (uA - uC) + a.kBC[f] * (uB - uC) + a.kRL[f] * (un[k] - ui);
            }
            acc += uup * po[k] - D * diff;
        }
    }
    const R unew = base + a_dt * (-acc / vol + src);
    uout[i] = unew;
    if (bnd) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (nb[k] < nc) continue;
            const int64_t g = nb[k] - nc;
            const int kind = bc.kind[d.gtag[g]];
            const R val = bc_value<R>(bc, g);
            R ug;
            if (kind == kDirichlet) ug = R(2) * val - unew;
            else if (kind == kNeumann) ug = unew + val * a.gdist[g];
            else ug = unew;
            uout[nc + g] = ug;
        }
    }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_residual_out(Dev d, FvArrays<R> a, double* res) {
    const int64_t i = gtid();
    if (i >= d.nc) return;
    const int64_t nc = d.nc;
    R acc = R(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = d.c2f[k * nc + i];
        if (c >= 0) acc += a.flux[c];
        else acc -= a.flux[~c];
    }
    res[i] = double(-acc / a.vol[i] + a.src[i]);
}

// phi_f = 1/2 (V_L + V_R) . S_f  (V_L . S_f on the boundary), with an FP32 copy
__global__ __launch_bounds__(kBlock) void k_face_phi(Dev d) {
    const int64_t f = gtid();
    if (f >= d.nf) return;
    const int64_t nc = d.nc, nf = d.nf;
    const int L = d.fL[f];
    const int R = f < d.nfi ? d.fR[f] : L;
    const double vx = 0.5 * (d.vel[L] + d.vel[R]);
    const double vy = 0.5 * (d.vel[nc + L] + d.vel[nc + R]);
    const double vz = 0.5 * (d.vel[2 * nc + L] + d.vel[2 * nc + R]);
    const double ph = vx * d.S[f] + vy * d.S[nf + f] + vz * d.S[2 * nf + f];
    d.phi[f] = ph;
    d.phi32[f] = float(ph);
}

// the FP64 cell step's copy of phi: per cell and face, outward from the cell
__global__ __launch_bounds__(kBlock) void k_cell_phi(Dev d) {
    const int64_t i = gtid();
    if (i >= d.nc) return;
    const int64_t nc = d.nc;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int code = d.c2f[k * nc + i];
        const double po = code >= 0 ? d.phi[code] : -d.phi[~code];
        d.fvc_phi[k * nc + i] = po;
        d.fvc_phi32[k * nc + i] = float(po);
    }
}

// FP32 copies of the static geometry the FP32 kernels read
__global__ __launch_bounds__(kBlock) void k_make_fp32_geometry(Dev d, int64_t node_padded) {
    const int64_t i = gtid();
    const int64_t nc = d.nc, nf = d.nf, NX = d.nc + d.nb;
    if (i < nc) {
        d.vol32[i] = float(d.vol[i]);
        for (int k = 0; k < 6; ++k) d.minv32[k * nc + i] = float(d.minv[k * nc + i]);
    }
    if (i < NX)
        for (int k = 0; k < 3; ++k) d.xc32[k * NX + i] = float(d.xc[k * NX + i]);
    if (i < nf) {
        d.kAC32[i] = float(d.kAC[i]);
        d.kBC32[i] = float(d.kBC[i]);
        d.kRL32[i] = float(d.kRL[i]);
        d.area32[i] = float(d.area[i]);
        for (int k = 0; k < 3; ++k) d.fx32[k * nf + i] = float(d.fx[k * nf + i]);
    }
    if (i < d.nb) d.gdist32[i] = float(d.gdist[i]);
    if (i < node_padded) d.n_alpha32[i] = float(d.n_alpha[i]);
}

__global__ __launch_bounds__(kBlock) void k_cast_to_f32(int64_t n, const double* __restrict__ src, float* dst) {
    const int64_t i = gtid();
    if (i < n) dst[i] = float(src[i]);
}

__global__ __launch_bounds__(kBlock) void k_cast_to_f64(int64_t n, const float* __restrict__ src, double* dst) {
    const int64_t i = gtid();
    if (i < n) dst[i] = double(src[i]);
}

// caller order <-> internal order (perm: internal -> caller), converting
// the element type on the way (FP64 <-> FP32 rounds to nearest)
template <class Tin, class Tout>
__global__ __launch_bounds__(kBlock) void k_to_internal(const int32_t* __restrict__ perm, int64_t n,
                                                         int64_t sin, int64_t sout, int comps,
                                                         const Tin* __restrict__ src, Tout* dst) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int64_t o = perm[i];
    for (int c = 0; c < comps; ++c) dst[c * sout + i] = Tout(src[c * sin + o]);
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kBlock) void k_to_user(const int32_t* __restrict__ perm, int64_t n,
                                                     int64_t sin, int64_t sout, int comps,
                                                     const Tin* __restrict__ src, Tout* dst) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int64_t o = perm[i];
    for (int c = 0; c < comps; ++c) dst[c * sout + o] = Tout(src[c * sin + i]);
}

// boundary values of variable var at every ghost whose face carries `tag`:
// the constant `value`, or vals[the caller's boundary triangle of the ghost]
__global__ __launch_bounds__(kBlock) void k_set_bc_values(Dev d, int var, int tag, double value,
                                                           const double* __restrict__ vals) {
    const int64_t g = gtid();
    if (g >= d.nb || d.gtag[g] != tag) return;
    const double v = vals ? vals[d.gbtri[g]] : value;
    d.gval[var * d.nb + g] = v;
    if (var == 0) d.gval32[g] = float(v);
}

// dt bound of mesh m: min_i mu_i / sum_{active faces} (|phi_f| + D_m kRL_f),
// per block (FP64)
__global__ __launch_bounds__(kBlock) void k_cfl(Dev d, BcTable bc, int m) {
    __shared__ double lds[4];
    const int64_t nc = d.nc;
    const double D = d.mesh_D[m];
    double best = __builtin_huge_val();
    for (int64_t i = d.mesh_start[m] + gtid(); i < d.mesh_start[m + 1]; i += int64_t(gridDim.x) * blockDim.x) {
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

// sum_i mu_i u_i over mesh m in FP64 (FP64 volumes, the state widened to FP64)
template <class R>
__global__ __launch_bounds__(kBlock) void k_conservation(Dev d, const R* __restrict__ u, int m) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int64_t i = d.mesh_start[m] + gtid(); i < d.mesh_start[m + 1]; i += int64_t(gridDim.x) * blockDim.x)
        s += d.vol[i] * double(u[i]);
    s = block_sum256(s, lds);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = s;
}

// one block: reduce n partials into mesh m's scal[slot] (op 0 = sum, 1 = min)
__global__ __launch_bounds__(1024) void k_finalize(Dev d, int64_t n, int m, int slot, int op) {
    __shared__ double lds[16];
    const double v = op == 0 ? reduce_partials_sum(d.partial, n, lds) : reduce_partials_min(d.partial, n, lds);
    if (threadIdx.x == 0) msc(d, m)[slot] = v;
}

// the time step each mesh's update uses: dt if dt > 0, else its CFL bound
// times cfl (stored by the last CFL evaluation)
__global__ void k_set_dt(Dev d, double dt, double cfl) {
    const int m = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (m < d.nm) d.mesh_dt[m] = dt > 0.0 ? dt : cfl * msc(d, m)[SC_DT_INV];
}

// ---- launchers ---------------------------------------------------------------
FvArrays<double> fv64(const Dev& d) {
    return {d.u, d.grad, d.psi, d.unode, d.flux, d.phi, d.minv, d.kAC, d.kBC, d.kRL, d.area,
            d.vol, d.src, d.n_alpha, d.fx, d.xc, d.gdist, d.uf, d.fvc_w, d.fvc_r, d.fvc_phi};
}

FvArrays<float> fv32(const Dev& d) {
    return {d.u32, d.grad32, d.psi32, d.unode32, d.flux32, d.phi32, d.minv32, d.kAC32, d.kBC32,
            d.kRL32, d.area32, d.vol32, d.src32, d.n_alpha32, d.fx32, d.xc32, d.gdist32,
            d.uf32, d.fvc_w32, d.fvc_r32, d.fvc_phi32};
}

template <class R>
hipError_t launch_ghost_fill_t(const Dev& d, const FvArrays<R>& a, const BcTable& bc, hipStream_t s) {
    if (d.nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_fill<R>, dim3(grid_for(d.nb)), dim3(kBlock), 0, s, d.nc, d.nb, d.gowner,
                       d.gtag, a.gdist, bc, a.u);
    return hipGetLastError();
}

hipError_t launch_ghost_fill(const Dev& d, bool fp32, const BcTable& bc, hipStream_t s) {
    return fp32 ? launch_ghost_fill_t(d, fv32(d), bc, s) : launch_ghost_fill_t(d, fv64(d), bc, s);
}

// The star-moment tile kernel in either precision (it also computes the
// vertex values): LDS of the halo's two 2-vectors and the touched vertices'
// four 2-vectors
template <class R>
size_t moments_lds_bytes(const Dev& d) {
    using V2 = typename Vec2T<R>::T;
    return size_t(2 * ((d.halo_max + 1) & ~1) + 4 * d.tv_max) * sizeof(V2);
}

template <class R, bool PARTS>
hipError_t allow_lds(const Dev& d) {
    const size_t lds = moments_lds_bytes<R>(d);
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_grad_moments<R, PARTS>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
}

hipError_t setup_fv_kernels(const Dev& d) {
    hipError_t e = allow_lds<double, false>(d);
    if (e == hipSuccess) e = allow_lds<double, true>(d);
    if (e == hipSuccess) e = allow_lds<float, true>(d);
    if (e == hipSuccess) e = allow_lds<float, false>(d);
    return e;
}

template <class R>
void launch_grad_t(const Dev& d, FvArrays<R> a, bool parts, const void* u_in, hipStream_t s) {
    const dim3 b(d.tile_rows);
    // grid padded to a multiple of 8 for the XCD-contiguous tile order
    const dim3 gx(unsigned((d.ntiles + kXcds - 1) / kXcds * kXcds));
    if (u_in) a.u = const_cast<R*>(static_cast<const R*>(u_in));   // read only
    if (parts)
        hipLaunchKernelGGL((k_grad_moments<R, true>), gx, b, moments_lds_bytes<R>(d), s, d, a);
    else
        hipLaunchKernelGGL((k_grad_moments<R, false>), gx, b, moments_lds_bytes<R>(d), s, d, a);
}

hipError_t launch_grad_limiter(const Dev& d, bool fp32, hipStream_t s, bool parts, const void* u_in) {
    if (fp32) launch_grad_t(d, fv32(d), parts, u_in, s);
    else launch_grad_t(d, fv64(d), parts, u_in, s);
    return hipGetLastError();
}
hipError_t launch_face_flux(const Dev& d, bool fp32, const BcTable& bc, hipStream_t s) {
    if (fp32)
        hipLaunchKernelGGL(k_face_flux<float>, dim3(grid_for(d.nf)), dim3(kBlock), 0, s, d, fv32(d), bc);
    else
        hipLaunchKernelGGL(k_face_flux<double>, dim3(grid_for(d.nf)), dim3(kBlock), 0, s, d, fv64(d), bc);
    return hipGetLastError();
}

hipError_t launch_cell_step(const Dev& d, bool fp32, const BcTable& bc, const void* u_in, void* u_out,
                            double alpha, hipStream_t s) {
    if (fp32)
        hipLaunchKernelGGL(k_cell_step<float>, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, fv32(d), bc,
                           static_cast<const float*>(u_in), static_cast<float*>(u_out), alpha);
    else
        hipLaunchKernelGGL(k_cell_step<double>, dim3(rows_m(d.nc, kBlock)), dim3(kBlock), 0, s, d, fv64(d), bc,
                           static_cast<const double*>(u_in), static_cast<double*>(u_out), alpha);
    return hipGetLastError();
}

hipError_t launch_fv_cell_setup(const Dev& d, hipStream_t s) {
    if (d.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fv_cell_setup, dim3(grid_for(d.nc)), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_set_dt(const Dev& d, double dt, double cfl, hipStream_t s) {
    hipLaunchKernelGGL(k_set_dt, dim3((d.nm + 255) / 256), dim3(256), 0, s, d, dt, cfl);
    return hipGetLastError();
}

hipError_t launch_residual_out(const Dev& d, bool fp32, double* res, hipStream_t s) {
    if (fp32)
        hipLaunchKernelGGL(k_residual_out<float>, dim3(grid_for(d.nc)), dim3(kBlock), 0, s, d, fv32(d), res);
    else
        hipLaunchKernelGGL(k_residual_out<double>, dim3(grid_for(d.nc)), dim3(kBlock), 0, s, d, fv64(d), res);
    return hipGetLastError();
}

hipError_t launch_face_phi(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_face_phi, dim3(grid_for(d.nf)), dim3(kBlock), 0, s, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || d.nc == 0) return e;
    hipLaunchKernelGGL(k_cell_phi, dim3(grid_for(d.nc)), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_make_fp32_geometry(const Dev& d, int64_t node_padded, hipStream_t s) {
    int64_t n = d.nc + d.nb;
    if (d.nf > n) n = d.nf;
    if (node_padded > n) n = node_padded;
    hipLaunchKernelGGL(k_make_fp32_geometry, dim3(grid_for(n)), dim3(kBlock), 0, s, d, node_padded);
    return hipGetLastError();
}

hipError_t launch_cast_to_f32(int64_t n, const double* src, float* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_to_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_cast_to_f64(int64_t n, const float* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_to_f64, dim3(grid_for(n)), dim3(kBlock), 0, s, n, src, dst);
    return hipGetLastError();
}

template <class Tin, class Tout>
hipError_t to_internal_t(const int32_t* perm, int64_t n, int64_t sin, int64_t sout, int comps, const Tin* src,
                         Tout* dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_to_internal<Tin, Tout>), dim3(grid_for(n)), dim3(kBlock), 0, s, perm, n, sin, sout,
                       comps, src, dst);
    return hipGetLastError();
}

template <class Tin, class Tout>
hipError_t to_user_t(const int32_t* perm, int64_t n, int64_t sin, int64_t sout, int comps, const Tin* src,
                     Tout* dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_to_user<Tin, Tout>), dim3(grid_for(n)), dim3(kBlock), 0, s, perm, n, sin, sout, comps,
                       src, dst);
    return hipGetLastError();
}

hipError_t launch_to_internal(const int32_t* perm, int64_t n, int64_t sin, int64_t sout, int comps,
                              const double* src, double* dst, hipStream_t s) {
    return to_internal_t(perm, n, sin, sout, comps, src, dst, s);
}

hipError_t launch_to_user(const int32_t* perm, int64_t n, int64_t sin, int64_t sout, int comps,
                          const double* src, double* dst, hipStream_t s) {
    return to_user_t(perm, n, sin, sout, comps, src, dst, s);
}

hipError_t launch_to_internal_typed(const int32_t* perm, int64_t n, int comps, const void* src, bool src_f32,
                                    void* dst, bool dst_f32, hipStream_t s) {
    if (src_f32)
        return dst_f32 ? to_internal_t(perm, n, n, n, comps, (const float*)src, (float*)dst, s)
                       : to_internal_t(perm, n, n, n, comps, (const float*)src, (double*)dst, s);
    return dst_f32 ? to_internal_t(perm, n, n, n, comps, (const double*)src, (float*)dst, s)
                   : to_internal_t(perm, n, n, n, comps, (const double*)src, (double*)dst, s);
}

hipError_t launch_to_user_typed(const int32_t* perm, int64_t n, int comps, const void* src, bool src_f32,
                                void* dst, bool dst_f32, hipStream_t s) {
    if (src_f32)
        return dst_f32 ? to_user_t(perm, n, n, n, comps, (const float*)src, (float*)dst, s)
                       : to_user_t(perm, n, n, n, comps, (const float*)src, (double*)dst, s);
    return dst_f32 ? to_user_t(perm, n, n, n, comps, (const double*)src, (float*)dst, s)
                   : to_user_t(perm, n, n, n, comps, (const double*)src, (double*)dst, s);
}

hipError_t launch_set_bc_values(const Dev& d, int var, int tag, double value, const double* vals, hipStream_t s) {
    if (d.nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_bc_values, dim3(grid_for(d.nb)), dim3(kBlock), 0, s, d, var, tag, value, vals);
    return hipGetLastError();
}

// per mesh: one grid-stride reduction over the mesh's cells, then a finalize
static int blocks_for_range(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return int(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_cfl(const Dev& d, const Mesh& mh, const BcTable& bc, hipStream_t s) {
    for (int m = 0; m < d.nm; ++m) {
        const int nblk = blocks_for_range(mh.mesh_start[m + 1] - mh.mesh_start[m]);
        hipLaunchKernelGGL(k_cfl, dim3(nblk), dim3(kBlock), 0, s, d, bc, m);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, d, int64_t(nblk), m, int(SC_DT_INV), 1);
    }
    return hipGetLastError();
}

hipError_t launch_conservation(const Dev& d, const Mesh& mh, bool fp32, hipStream_t s) {
    for (int m = 0; m < d.nm; ++m) {
        const int nblk = blocks_for_range(mh.mesh_start[m + 1] - mh.mesh_start[m]);
        if (fp32)
            hipLaunchKernelGGL(k_conservation<float>, dim3(nblk), dim3(kBlock), 0, s, d, (const float*)d.u32, m);
        else
            hipLaunchKernelGGL(k_conservation<double>, dim3(nblk), dim3(kBlock), 0, s, d, (const double*)d.u, m);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, d, int64_t(nblk), m, int(SC_CONS), 0);
    }
    return hipGetLastError();
}

}  // namespace mifvm
