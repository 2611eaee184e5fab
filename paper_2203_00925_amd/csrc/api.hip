// C ABI of the library (declared in include/mifvm.h): argument checking,
// workspace layout, and the host-side sequencing of the kernels (stages of
// eq. (6), chunks of CG iterations).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <array>
#include <string>

#include "../../include/mifvm.h"
#include "api_util.h"
#include "gmres.h"
#include "mesh.h"
#include "nn.h"
#include "state.h"

using namespace mifvm_api;

static_assert(mifvm::kNumKernels == MIFVM_K_COUNT, "kernel timing slots and the ABI's kernel ids disagree");


namespace mifvm {

size_t layout(const Mesh& m, char* base, Dev& d) {
    size_t off = 0;
    const int64_t nc = m.nc, nv = m.nv, nf = m.nf, nb = m.nb, NX = nc + nb;
    d.nc = nc; d.nv = nv; d.nf = nf; d.nfi = m.nfi; d.nb = nb;
    d.ns = m.stencil.nslices; d.nvs = m.node.nslices;
    d.vol = carve<double>(base, off, nc);
    d.xc = carve<double>(base, off, 3 * NX);
    d.minv = carve<double>(base, off, 6 * nc);
    d.xyz4 = carve<double4>(base, off, NX);
    d.fx4 = carve<double4>(base, off, nf);
    d.c2f = carve<int32_t>(base, off, 4 * nc);
    d.c2n = carve<int32_t>(base, off, 4 * nc);
    d.s_off = carve<int64_t>(base, off, m.stencil.off.size());
    d.s_w = carve<int32_t>(base, off, m.stencil.width.size());
    d.s_idx = carve<int32_t>(base, off, m.stencil.idx.size());
    d.fL = carve<int32_t>(base, off, nf);
    d.fR = carve<int32_t>(base, off, nf);
    d.fA = carve<int32_t>(base, off, nf);
    d.fB = carve<int32_t>(base, off, nf);
    d.fC = carve<int32_t>(base, off, nf);
    d.kAC = carve<double>(base, off, nf);
    d.kBC = carve<double>(base, off, nf);
    d.kRL = carve<double>(base, off, nf);
    d.fx = carve<double>(base, off, 3 * nf);
    d.S = carve<double>(base, off, 3 * nf);
    d.area = carve<double>(base, off, nf);
    d.gowner = carve<int32_t>(base, off, nb);
    d.gtag = carve<int32_t>(base, off, nb);
    d.gdist = carve<double>(base, off, nb);
    d.gbtri = carve<int32_t>(base, off, nb);
    d.gval = carve<double>(base, off, 2 * nb);
    d.gval32 = carve<float>(base, off, nb);
    d.n_off = carve<int64_t>(base, off, m.node.off.size());
    d.n_w = carve<int32_t>(base, off, m.node.width.size());
    d.n_idx = carve<int32_t>(base, off, m.node.idx.size());
    d.n_alpha = carve<double>(base, off, m.node.val.size());
    d.n_len = carve<int32_t>(base, off, nv);
    d.tv_max = m.tv_max;
    d.e_off = carve<int64_t>(base, off, m.enbr.off.size());
    d.e_w = carve<int32_t>(base, off, m.enbr.width.size());
    d.e_lidx = carve<uint16_t>(base, off, m.e_lidx.size() > 0 ? m.e_lidx.size() : 1);
    d.c2v_l = carve<uint16_t>(base, off, 4 * nc);
    d.fv_off = carve<int64_t>(base, off, m.fv_off.size());
    d.fv_len = carve<int32_t>(base, off, m.fv_len.size() > 0 ? m.fv_len.size() : 1);
    d.f_off = carve<int64_t>(base, off, m.fnode.off.size());
    d.f_w = carve<int32_t>(base, off, m.fnode.width.size() > 0 ? m.fnode.width.size() : 1);
    d.f_lidx = carve<uint16_t>(base, off, m.f_lidx.size() > 0 ? m.f_lidx.size() : 1);
    d.k_off = carve<int64_t>(base, off, m.kmat.off.size());
    d.k_w = carve<int32_t>(base, off, m.kmat.width.size());
    d.k_col = carve<int32_t>(base, off, m.kmat.idx.size());
    d.k_len = carve<int32_t>(base, off, nc);
    d.k_val = carve<double>(base, off, m.kmat.idx.size());
    d.k_diag = carve<double>(base, off, nc);
    d.k_dinv = carve<double>(base, off, nc);
    d.k_c = carve<double>(base, off, nc);
    d.k_val32 = carve<float>(base, off, m.kmat.idx.size());
    d.k_diag32 = carve<float>(base, off, nc);
    d.k_dinv32 = carve<float>(base, off, nc);
    d.d32 = carve<float>(base, off, nc);
    d.r32 = carve<float>(base, off, nc);
    d.z32 = carve<float>(base, off, nc);
    d.p32 = carve<float>(base, off, nc);
    d.q32 = carve<float>(base, off, nc);
    d.tile_rows = m.tile_rows;
    d.halo_max = m.halo_max;
    d.ntiles = (int64_t)m.h_self.size();
    d.h_off = carve<int64_t>(base, off, m.h_off.size());
    d.h_idx = carve<int32_t>(base, off, m.h_idx.size());
    d.h_self = carve<int32_t>(base, off, m.h_self.size());
    d.k_lidx = carve<uint16_t>(base, off, m.k_lidx.size());
    d.c2n_l = carve<uint16_t>(base, off, m.c2n_l.size());
    d.n_lidx = carve<uint16_t>(base, off, m.n_lidx.size());
    d.v_off = carve<int64_t>(base, off, m.v_off.size());
    d.cell_perm = carve<int32_t>(base, off, nc);
    d.vert_perm = carve<int32_t>(base, off, nv);
    d.u = carve<double>(base, off, NX);
    d.src = carve<double>(base, off, nc);
    d.vel = carve<double>(base, off, 3 * nc);
    d.phi = carve<double>(base, off, nf);
    d.grad = carve<double>(base, off, 3 * nc);
    d.psi = carve<double>(base, off, nc);
    d.uf = carve<double>(base, off, 4 * nc);
    d.u_b = carve<double>(base, off, NX);
    d.u_c = carve<double>(base, off, NX);
    d.fvc_vid = carve<int32_t>(base, off, 4 * nc);
    d.fvc_w = carve<double>(base, off, 4 * nc);
    d.fvc_r = carve<double>(base, off, 4 * nc);
    d.fvc_slot = carve<uint8_t>(base, off, nc);
    d.fvc_phi = carve<double>(base, off, 4 * nc);
    d.uf32 = carve<float>(base, off, 4 * nc);
    d.u_b32 = carve<float>(base, off, NX);
    d.u_c32 = carve<float>(base, off, NX);
    d.fvc_w32 = carve<float>(base, off, 4 * nc);
    d.fvc_r32 = carve<float>(base, off, 4 * nc);
    d.fvc_phi32 = carve<float>(base, off, 4 * nc);
    d.unode = carve<double>(base, off, nv);
    d.flux = carve<double>(base, off, nf);
    d.x = carve<double>(base, off, nc);
    d.r = carve<double>(base, off, nc);
    d.z = carve<double>(base, off, nc);
    d.p = carve<double>(base, off, nc);
    d.q = carve<double>(base, off, nc);
    d.b = carve<double>(base, off, nc);
    d.u32 = carve<float>(base, off, NX);
    d.src32 = carve<float>(base, off, nc);
    d.phi32 = carve<float>(base, off, nf);
    d.grad32 = carve<float>(base, off, 3 * nc);
    d.psi32 = carve<float>(base, off, nc);
    d.unode32 = carve<float>(base, off, nv);
    d.flux32 = carve<float>(base, off, nf);
    d.minv32 = carve<float>(base, off, 6 * nc);
    d.kAC32 = carve<float>(base, off, nf);
    d.kBC32 = carve<float>(base, off, nf);
    d.kRL32 = carve<float>(base, off, nf);
    d.area32 = carve<float>(base, off, nf);
    d.vol32 = carve<float>(base, off, nc);
    d.n_alpha32 = carve<float>(base, off, m.node.val.size());
    d.fx32 = carve<float>(base, off, 3 * nf);
    d.xc32 = carve<float>(base, off, 3 * NX);
    d.gdist32 = carve<float>(base, off, nb);
    d.tmp = carve<double>(base, off, 3 * NX);
    d.np_ion = carve<double>(base, off, nc);
    d.efield = carve<double>(base, off, 3 * nc);
    d.mf_xv = carve<double>(base, off, nv);
    d.mf_nidx = carve<int32_t>(base, off, m.node.idx.size() > 0 ? m.node.idx.size() : 1);
    d.n_entries = int64_t(m.node.idx.size());
    d.mfc_vid = carve<int32_t>(base, off, 4 * nc);
    d.mfc_w = carve<double>(base, off, 4 * nc);
    d.mfc_r = carve<double>(base, off, 4 * nc);
    d.mfc_w32 = carve<float>(base, off, 4 * nc);
    d.mfc_r32 = carve<float>(base, off, 4 * nc);
    // per-block partials of up to 4 sums x 2 mesh slots, for blocks of >= 64 rows
    const int64_t nblk = (nc + 63) / 64;
    d.partial = carve<double>(base, off, 8 * (nblk + 1024));
    d.nm = int32_t(m.mesh_start.size() - 1);
    d.mesh_start = carve<int64_t>(base, off, m.mesh_start.size());
    d.mesh_D = carve<double>(base, off, d.nm);
    d.mesh_dt = carve<double>(base, off, d.nm);
    d.scal = carve<double>(base, off, size_t(d.nm) * SC_COUNT_);
    return (off + 255) & ~size_t(255);
}

void drop_graphs(State& s) {
    hipGraphExec_t* execs[] = {&s.cg_exec, &s.step_exec, &s.fcg_exec, &s.gm_exec, &s.amg_exec};
    for (hipGraphExec_t* e : execs) {
        if (*e) (void)hipGraphExecDestroy(*e);
        *e = nullptr;
    }
    s.cg_exec_chunk = 0;
    s.cg_exec_method = -1;
    s.step_exec_n = 0;
    s.step_exec_dt = -1.0;
    s.step_exec_cfl = -1.0;
    s.fcg_exec_chunk = 0;
    s.gm_exec_key = 0;
    s.amg_exec_key = 0;
    ++s.graph_gen;                            // graphs held elsewhere (a batch's) follow
}

}  // namespace mifvm

using namespace mifvm;

namespace {
// one chunk of n CG iterations (plain FP64, matrix-free or stored K, or FP32
// inner), no timing events
hipError_t enqueue_cg_chunk(const State& s, int method, int n, hipStream_t q) {
    const Dev& d = s.d;
    for (int c = 0; c < n; ++c) {
        hipError_t e = method == MIFVM_SOLVE_PLAIN
                           ? (s.mf ? launch_mf_cg_spmv(d, s.bc[1], q) : launch_cg_spmv(d, q))
                           : (s.mf ? launch_mf_cg32_spmv(d, s.bc[1], q) : launch_cg32_spmv(d, q));
        if (e == hipSuccess) e = method == MIFVM_SOLVE_PLAIN ? launch_cg_axpy(d, q) : launch_cg32_axpy(d, q);
        if (e == hipSuccess) e = method == MIFVM_SOLVE_PLAIN ? launch_cg_dir(d, q) : launch_cg32_dir(d, q);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

extern "C" {

const char* mifvm_last_error(void) { return g_err.c_str(); }
const char* mifvm_version(void) { return "mifvm 0.1 (gfx950, fp64)"; }

int mifvm_mesh_preprocess(const double* xyz, int64_t nv, const int32_t* tets, int64_t nc,
                          const int32_t* btris, const int32_t* btags, int64_t nb,
                          const mifvm_mesh_opts* opts, mifvm_mesh** out) {
    if (!out) return fail(MIFVM_E_ARG, "out is null");
    *out = nullptr;
    auto* h = new (std::nothrow) mifvm_mesh();
    if (!h) return fail(MIFVM_E_ARG, "out of host memory");
    std::string err;
    int rc;
    try {
        rc = preprocess(xyz, nv, tets, nc, btris, btags, nb, opts ? opts->renumber : 1,
                        opts ? opts->mesh_cell_start : nullptr, opts ? opts->nmeshes : 1,
                        opts && opts->no_matrix != 0, h->m, err);
    } catch (const std::bad_alloc&) {
        rc = MIFVM_E_ARG;
        err = "out of host memory";
    }
    if (rc != 0) {
        delete h;
        return fail(rc, err);
    }
    *out = h;
    return MIFVM_OK;
}

int mifvm_mesh_get_info(const mifvm_mesh* mesh, mifvm_mesh_info* out) {
    if (!mesh || !out) return fail(MIFVM_E_ARG, "null argument");
    const Mesh& m = mesh->m;
    std::memset(out, 0, sizeof(*out));
    out->nc = m.nc; out->nv = m.nv; out->nf = m.nf; out->nf_interior = m.nfi; out->nb = m.nb;
    out->nmeshes = int32_t(m.mesh_start.size() - 1);
    out->stencil_entries = (int64_t)m.sidx.size();
    out->stencil_padded = (int64_t)m.stencil.idx.size();
    out->node_entries = (int64_t)m.nidx.size();
    out->matrix_nnz = m.matrix_nnz;
    out->matrix_padded = (int64_t)m.kmat.idx.size();
    out->stencil_max = m.stencil_max;
    out->node_max = m.node_max;
    out->row_max = m.row_max;
    out->tile_rows = m.tile_rows;
    out->halo_max = m.halo_max;
    out->tile_vertices_max = m.tv_max;
    out->halo_entries = (int64_t)m.h_idx.size();
    Dev d{};
    out->ws_bytes = layout(m, nullptr, d);
    out->edge_nbr_entries = (int64_t)m.eidx.size();
    out->foreign_rows = (int64_t)m.fv_idx.size();
    int64_t fe = 0;
    for (int32_t n : m.fv_len) fe += n;
    out->foreign_entries = fe;
    return MIFVM_OK;
}

void mifvm_mesh_destroy(mifvm_mesh* mesh) { delete mesh; }

int mifvm_mesh_export(const mifvm_mesh* mesh, int32_t what, void* dst, size_t bytes) {
    if (!mesh || !dst) return fail(MIFVM_E_ARG, "null argument");
    const Mesh& m = mesh->m;
    const void* src = nullptr;
    size_t n = 0;
    std::vector<int32_t> tmp32;
    std::vector<double> tmp64;
    switch (what) {
        case 0: src = m.cell_perm.data(); n = m.cell_perm.size() * 4; break;
        case 1: src = m.vert_perm.data(); n = m.vert_perm.size() * 4; break;
        case 2: src = m.vol.data(); n = m.vol.size() * 8; break;
        case 3: src = m.xc.data(); n = m.xc.size() * 8; break;
        case 4:
            tmp32 = m.fL; tmp32.insert(tmp32.end(), m.fR.begin(), m.fR.end());
            src = tmp32.data(); n = tmp32.size() * 4; break;
        case 5:
            tmp32 = m.fA; tmp32.insert(tmp32.end(), m.fB.begin(), m.fB.end());
            tmp32.insert(tmp32.end(), m.fC.begin(), m.fC.end());
            src = tmp32.data(); n = tmp32.size() * 4; break;
        case 6:
            tmp64 = m.kAC; tmp64.insert(tmp64.end(), m.kBC.begin(), m.kBC.end());
            tmp64.insert(tmp64.end(), m.kRL.begin(), m.kRL.end());
            src = tmp64.data(); n = tmp64.size() * 8; break;
        case 7: src = m.S.data(); n = m.S.size() * 8; break;
        case 8: src = m.sptr.data(); n = m.sptr.size() * 8; break;
        case 9: src = m.sidx.data(); n = m.sidx.size() * 4; break;
        case 10: src = m.nptr.data(); n = m.nptr.size() * 8; break;
        case 11: src = m.nidx.data(); n = m.nidx.size() * 4; break;
        case 12: src = m.nalpha.data(); n = m.nalpha.size() * 8; break;
        case 13: src = m.gowner.data(); n = m.gowner.size() * 4; break;
        case 14: src = m.gtag.data(); n = m.gtag.size() * 4; break;
        case 15: src = m.minv.data(); n = m.minv.size() * 8; break;
        case 16: src = m.eptr.data(); n = m.eptr.size() * 8; break;
        case 17: src = m.eidx.data(); n = m.eidx.size() * 4; break;
        default: return fail(MIFVM_E_ARG, "unknown export id");
    }
    if (bytes != n) return fail(MIFVM_E_ARG, "size mismatch: expected " + std::to_string(n) + " bytes");
    if (n) std::memcpy(dst, src, n);
    return MIFVM_OK;
}

int mifvm_state_create(const mifvm_mesh* mesh, const mifvm_params* params, void* d_ws, size_t ws_bytes,
                       void* stream, mifvm_state** out) {
    if (!mesh || !out || !d_ws) return fail(MIFVM_E_ARG, "null argument");
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(MIFVM_E_WORKSPACE, "workspace not 256-byte aligned");
    const Mesh& m = mesh->m;
    Dev probe{};
    const size_t need = layout(m, nullptr, probe);
    if (ws_bytes < need) return fail(MIFVM_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
    auto* h = new (std::nothrow) mifvm_state();
    if (!h) return fail(MIFVM_E_ARG, "out of host memory");
    State& st = h->s;
    st.mesh = &m;
    layout(m, static_cast<char*>(d_ws), st.d);
    st.diffusivity = params ? params->diffusivity : 0.0;
    st.fp32 = params && params->precision == MIFVM_FP32;
    if (params && params->precision != MIFVM_FP64 && params->precision != MIFVM_FP32) {
        delete h;
        return fail(MIFVM_E_ARG, "unknown precision");
    }
    for (int v = 0; v < 2; ++v) {
        for (int t = 0; t < kMaxTags; ++t) {
            st.bc[v].kind[t] = kZeroFlux;
            st.bc_tag_value[v][t] = 0.0;
        }
        st.bc[v].val = st.d.gval + v * m.nb;
        st.bc[v].val32 = v == 0 ? st.d.gval32 : nullptr;
    }
    st.nblk_cells = reduce_blocks(m.nc);
    hipStream_t s = S(stream);
    const Dev& d = st.d;
    auto cleanup = [&](int rc) {
        delete h;
        return rc;
    };
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&st.h_scal),
                                 size_t(st.d.nm) * SC_COUNT_ * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipHostMalloc"));
#define UP(dst, vec)                                            \
    do {                                                        \
        hipError_t e2 = up(dst, vec, s);                        \
        if (e2 != hipSuccess) return cleanup(hip_fail(e2, "upload " #vec)); \
    } while (0)
    UP(d.vol, m.vol); UP(d.xc, m.xc); UP(d.minv, m.minv); UP(d.c2f, m.c2f); UP(d.c2n, m.c2n);
    UP(d.s_off, m.stencil.off); UP(d.s_w, m.stencil.width); UP(d.s_idx, m.stencil.idx);
    UP(d.fL, m.fL); UP(d.fR, m.fR); UP(d.fA, m.fA); UP(d.fB, m.fB); UP(d.fC, m.fC);
    UP(d.kAC, m.kAC); UP(d.kBC, m.kBC); UP(d.kRL, m.kRL); UP(d.fx, m.fx); UP(d.S, m.S); UP(d.area, m.area);
    UP(d.gowner, m.gowner); UP(d.gtag, m.gtag); UP(d.gdist, m.gdist); UP(d.gbtri, m.gbtri);
    UP(d.n_off, m.node.off); UP(d.n_w, m.node.width); UP(d.n_idx, m.node.idx); UP(d.n_alpha, m.node.val);
    UP(d.n_len, m.n_len); UP(d.e_off, m.enbr.off); UP(d.e_w, m.enbr.width); UP(d.e_lidx, m.e_lidx);
    UP(d.c2v_l, m.c2v_l); UP(d.fv_off, m.fv_off); UP(d.fv_len, m.fv_len);
    UP(d.f_off, m.fnode.off); UP(d.f_w, m.fnode.width); UP(d.f_lidx, m.f_lidx);
    UP(d.k_off, m.kmat.off); UP(d.k_w, m.kmat.width); UP(d.k_col, m.kmat.idx); UP(d.k_len, m.klen);
    UP(d.cell_perm, m.cell_perm); UP(d.vert_perm, m.vert_perm);
    UP(d.h_off, m.h_off); UP(d.h_idx, m.h_idx); UP(d.h_self, m.h_self);
    UP(d.mesh_start, m.mesh_start);
    {
        const std::vector<double> Dm(d.nm, st.diffusivity), zero(d.nm, 0.0);
        UP(d.mesh_D, Dm);
        UP(d.mesh_dt, zero);
        e = hipStreamSynchronize(s);                       // Dm/zero are freed at scope exit
        if (e != hipSuccess) return cleanup(hip_fail(e, "upload mesh parameters"));
    }
    UP(d.k_lidx, m.k_lidx); UP(d.c2n_l, m.c2n_l);
    UP(d.n_lidx, m.n_lidx); UP(d.v_off, m.v_off);
    {   // packed records of the centres and face centroids (gathered by tiles)
        std::vector<double> rec(4 * (m.nc + m.nb)), frec(4 * m.nf);
        const int64_t NXh = m.nc + m.nb;
        for (int64_t e = 0; e < NXh; ++e) {
            rec[4 * e] = m.xc[e]; rec[4 * e + 1] = m.xc[NXh + e]; rec[4 * e + 2] = m.xc[2 * NXh + e]; rec[4 * e + 3] = 0.0;
        }
        for (int64_t f = 0; f < m.nf; ++f) {
            frec[4 * f] = m.fx[f]; frec[4 * f + 1] = m.fx[m.nf + f]; frec[4 * f + 2] = m.fx[2 * m.nf + f]; frec[4 * f + 3] = 0.0;
        }
        hipError_t e1 = hipMemcpyAsync(d.xyz4, rec.data(), rec.size() * 8, hipMemcpyHostToDevice, s);
        if (e1 == hipSuccess) e1 = hipMemcpyAsync(d.fx4, frec.data(), frec.size() * 8, hipMemcpyHostToDevice, s);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);      // rec/frec are freed at scope exit
        if (e1 != hipSuccess) return cleanup(hip_fail(e1, "upload packed records"));
    }
#undef UP
    const int64_t NX = m.nc + m.nb;
    e = hipMemsetAsync(d.u, 0, NX * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.src, 0, m.nc * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.vel, 0, 3 * m.nc * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.phi, 0, m.nf * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.fvc_phi, 0, 4 * m.nc * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.fvc_phi32, 0, 4 * m.nc * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.x, 0, m.nc * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.np_ion, 0, m.nc * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.efield, 0, 3 * m.nc * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.scal, 0, size_t(d.nm) * SC_COUNT_ * sizeof(double), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.u32, 0, NX * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.src32, 0, m.nc * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.phi32, 0, m.nf * sizeof(float), s);
    if (e == hipSuccess && m.nb > 0) e = hipMemsetAsync(d.gval, 0, 2 * m.nb * sizeof(double), s);
    if (e == hipSuccess && m.nb > 0) e = hipMemsetAsync(d.gval32, 0, m.nb * sizeof(float), s);
    if (e == hipSuccess) e = setup_fv_kernels(d);
    if (e == hipSuccess) e = launch_make_fp32_geometry(d, (int64_t)m.node.val.size(), s);
    if (e == hipSuccess) e = launch_fv_cell_setup(d, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // host vectors are not pinned
    if (e != hipSuccess) return cleanup(hip_fail(e, "state init"));
    *out = h;
    return MIFVM_OK;
}

void mifvm_state_destroy(mifvm_state* st) {
    if (!st) return;
    drop_graphs(st->s);
    amg_release(st->s);
    delete st->s.gm;
    delete st->s.nn_state;
    if (st->s.cap_stream) (void)hipStreamDestroy(st->s.cap_stream);
    if (st->s.h_scal) (void)hipHostFree(st->s.h_scal);
    for (hipEvent_t e : st->s.timer.pool) (void)hipEventDestroy(e);
    delete st;
}

int mifvm_kernel_timing_select(mifvm_state* st, uint64_t kernels) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    if (kernels >> kNumKernels) return fail(MIFVM_E_ARG, "kernel bit at or above MIFVM_K_COUNT");
    KernelTimer& t = st->s.timer;
    if (!t.pending.empty()) return fail(MIFVM_E_STATE, "timed launches not yet collected (call mifvm_kernel_stats)");
    t.on = kernels != 0;
    t.mask = kernels;
    if (t.on)
        for (int k = 0; k < kNumKernels; ++k) {
            t.total_ms[k] = 0.0;
            t.count[k] = 0;
        }
    return MIFVM_OK;
}

int mifvm_kernel_timing(mifvm_state* st, int32_t enable) {
    return mifvm_kernel_timing_select(st, enable != 0 ? (uint64_t(1) << kNumKernels) - 1 : 0);
}

int mifvm_kernel_stats(mifvm_state* st, int32_t kernel, double* total_ms, int64_t* launches, void* stream) {
    if (!st || !total_ms || !launches) return fail(MIFVM_E_ARG, "null argument");
    if (kernel < 0 || kernel >= kNumKernels) return fail(MIFVM_E_ARG, "unknown kernel id");
    KernelTimer& t = st->s.timer;
    HIPCHK(hipStreamSynchronize(S(stream)));
    HIPCHK(timer_flush(t));
    *total_ms = t.total_ms[kernel];
    *launches = t.count[kernel];
    return MIFVM_OK;
}

int mifvm_set_bc(mifvm_state* st, int32_t var, int32_t tag, int32_t kind, double value) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    if (var < 0 || var > 1) return fail(MIFVM_E_ARG, "unknown variable");
    if (tag < 0 || tag >= kMaxTags) return fail(MIFVM_E_ARG, "tag out of range");
    if (kind < 0 || kind > 2) return fail(MIFVM_E_ARG, "unknown boundary-condition kind");
    if (!std::isfinite(value)) return fail(MIFVM_E_ARG, "non-finite boundary value");
    State& s = st->s;
    // the value goes to every ghost of the tag in device memory, ordered
    // against work on any stream (this call has no stream argument)
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(launch_set_bc_values(s.d, var, tag, value, nullptr, nullptr));
    HIPCHK(hipDeviceSynchronize());
    s.bc[var].kind[tag] = kind;
    s.bc_tag_value[var][tag] = value;
    drop_graphs(s);                           // captured launches hold the kinds by value
    if (var == MIFVM_VAR_POTENTIAL) {
        s.assembled = false;
        s.consts_ready = false;
        s.mfc_ready = false;
    }
    return MIFVM_OK;
}

int mifvm_set_bc_values(mifvm_state* st, int32_t var, int32_t tag, const double* d_vals, void* stream) {
    if (!st || !d_vals) return fail(MIFVM_E_ARG, "null argument");
    if (var < 0 || var > 1) return fail(MIFVM_E_ARG, "unknown variable");
    if (tag < 0 || tag >= kMaxTags) return fail(MIFVM_E_ARG, "tag out of range");
    State& s = st->s;
    HIPCHK(launch_set_bc_values(s.d, var, tag, 0.0, d_vals, S(stream)));
    if (var == MIFVM_VAR_POTENTIAL) {         // the ghost constants c of the system change
        s.assembled = false;
        s.consts_ready = false;
    }
    return MIFVM_OK;
}

namespace {
int upload_mesh_D(State& s, const std::vector<double>& Dm) {
    HIPCHK(hipDeviceSynchronize());           // order against work on any stream
    HIPCHK(hipMemcpy(s.d.mesh_D, Dm.data(), Dm.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipDeviceSynchronize());
    return MIFVM_OK;
}
}  // namespace

int mifvm_set_diffusivity(mifvm_state* st, double D) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    if (!(D >= 0) || !std::isfinite(D)) return fail(MIFVM_E_ARG, "diffusivity must be finite and >= 0");
    st->s.diffusivity = D;
    return upload_mesh_D(st->s, std::vector<double>(st->s.d.nm, D));
}

int mifvm_set_mesh_diffusivity(mifvm_state* st, const double* D, int32_t n) {
    if (!st || !D) return fail(MIFVM_E_ARG, "null argument");
    if (n != st->s.d.nm) return fail(MIFVM_E_ARG, "need one diffusivity per mesh");
    for (int32_t m = 0; m < n; ++m)
        if (!(D[m] >= 0) || !std::isfinite(D[m])) return fail(MIFVM_E_ARG, "diffusivity must be finite and >= 0");
    return upload_mesh_D(st->s, std::vector<double>(D, D + n));
}

int mifvm_set_field(mifvm_state* st, int32_t field, const void* d_src, int32_t dtype, void* stream) {
    if (!st || !d_src) return fail(MIFVM_E_ARG, "null argument");
    if (dtype != MIFVM_F64 && dtype != MIFVM_F32) return fail(MIFVM_E_ARG, "unknown dtype");
    State& s = st->s;
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    const bool f32 = dtype == MIFVM_F32;
    auto in64 = [&](int comps, double* dst) { return launch_to_internal_typed(d.cell_perm, d.nc, comps, d_src, f32, dst, false, hs); };
    switch (field) {
        case MIFVM_FIELD_U:
            if (s.fp32 && f32) {                  // FP32 state from FP32 data: no rounding on the way
                HIPCHK(launch_to_internal_typed(d.cell_perm, d.nc, 1, d_src, true, d.u32, true, hs));
                HIPCHK(launch_cast_to_f64(d.nc, d.u32, d.u, hs));
            } else {
                HIPCHK(in64(1, d.u));
                if (s.fp32) HIPCHK(launch_cast_to_f32(d.nc, d.u, d.u32, hs));
            }
            HIPCHK(launch_ghost_fill(d, s.fp32, s.bc[0], hs));
            break;
        case MIFVM_FIELD_VEL:
            HIPCHK(in64(3, d.vel));
            HIPCHK(launch_face_phi(d, hs));
            s.vel_set = true;
            break;
        case MIFVM_FIELD_SOURCE:
            HIPCHK(in64(1, d.src));
            HIPCHK(launch_cast_to_f32(d.nc, d.src, d.src32, hs));
            break;
        case MIFVM_FIELD_P:
            HIPCHK(in64(1, d.x));
            break;
        case MIFVM_FIELD_ION:
            HIPCHK(in64(1, d.np_ion));
            break;
        case MIFVM_FIELD_EFIELD:
            return fail(MIFVM_E_ARG, "FIELD_EFIELD is computed by mifvm_streamer_step (get only)");
        default:
            return fail(MIFVM_E_ARG, "unknown field");
    }
    return MIFVM_OK;
}

int mifvm_get_field(const mifvm_state* st, int32_t field, void* d_dst, int32_t dtype, void* stream) {
    if (!st || !d_dst) return fail(MIFVM_E_ARG, "null argument");
    if (dtype != MIFVM_F64 && dtype != MIFVM_F32) return fail(MIFVM_E_ARG, "unknown dtype");
    const Dev& d = st->s.d;
    hipStream_t hs = S(stream);
    const bool f32 = dtype == MIFVM_F32;
    auto out64 = [&](int comps, const double* src) { return launch_to_user_typed(d.cell_perm, d.nc, comps, src, false, d_dst, f32, hs); };
    switch (field) {
        case MIFVM_FIELD_U:
            if (st->s.fp32) HIPCHK(launch_to_user_typed(d.cell_perm, d.nc, 1, d.u32, true, d_dst, f32, hs));
            else HIPCHK(out64(1, d.u));
            break;
        case MIFVM_FIELD_VEL: HIPCHK(out64(3, d.vel)); break;
        case MIFVM_FIELD_SOURCE: HIPCHK(out64(1, d.src)); break;
        case MIFVM_FIELD_P: HIPCHK(out64(1, d.x)); break;
        case MIFVM_FIELD_ION: HIPCHK(out64(1, d.np_ion)); break;
        case MIFVM_FIELD_EFIELD: HIPCHK(out64(3, d.efield)); break;
        default: return fail(MIFVM_E_ARG, "unknown field");
    }
    return MIFVM_OK;
}


int mifvm_cfl_dt(mifvm_state* st, double cfl, double* dt_out, void* stream) {
    if (!st || !dt_out) return fail(MIFVM_E_ARG, "null argument");
    if (!(cfl > 0)) return fail(MIFVM_E_ARG, "cfl must be > 0");
    State& s = st->s;
    hipStream_t hs = S(stream);
    HIPCHK(launch_cfl(s.d, *s.mesh, s.bc[0], hs));
    int rc = pull_scalars(s, hs);
    if (rc) return rc;
    double dmin = __builtin_huge_val();
    for (int m = 0; m < s.d.nm; ++m) {
        const double v = hsc(s, m, SC_DT_INV);
        if (!std::isfinite(v)) return fail(MIFVM_E_STATE, "no active face: time step unbounded");
        dmin = std::fmin(dmin, cfl * v);
    }
    s.cfl = cfl;
    *dt_out = dmin;
    return MIFVM_OK;
}

namespace {
// ghost fill (unless the ghosts are known current), gradient + limiter +
// vertex values, face fluxes: the residual evaluation and the FP32 step
int residual_parts(State& s, hipStream_t hs, bool ghosts = true) {
    const Dev& d = s.d;
    KernelTimer& t = s.timer;
    if (ghosts)
        HIPCHK(timed(t, MIFVM_K_GHOST_FILL, hs, [&] { return launch_ghost_fill(d, s.fp32, s.bc[0], hs); }));
    HIPCHK(timed(t, MIFVM_K_GRAD_LIMITER, hs, [&] { return launch_grad_limiter(d, s.fp32, hs, true); }));
    HIPCHK(timed(t, MIFVM_K_FACE_FLUX, hs, [&] { return launch_face_flux(d, s.fp32, s.bc[0], hs); }));
    return MIFVM_OK;
}

// the step's buffers of RK stage k: every stage adds to u^n (kept in u), so
// stage 0 reads u and writes u_b, stage 1 reads u_b and writes u_c, stage 2
// reads u_c and writes u (cell i alone reads u[i] there)
void stage_buffers(const Dev& d, bool fp32, int k, const void** uin, void** uout) {
    if (fp32) {
        *uin = k == 0 ? d.u32 : (k == 1 ? d.u_b32 : d.u_c32);
        *uout = k == 0 ? d.u_b32 : (k == 1 ? d.u_c32 : d.u32);
    } else {
        *uin = k == 0 ? d.u : (k == 1 ? d.u_b : d.u_c);
        *uout = k == 0 ? d.u_b : (k == 1 ? d.u_c : d.u);
    }
}
}  // namespace

int mifvm_step(mifvm_state* st, int32_t n_steps, double dt, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    if (n_steps < 0 || !(dt >= 0) || !std::isfinite(dt)) return fail(MIFVM_E_ARG, "bad n_steps or dt");
    State& s = st->s;
    hipStream_t hs = S(stream);
    if (dt == 0.0 && !(s.cfl > 0)) return fail(MIFVM_E_STATE, "dt = 0 asks for the CFL steps: call mifvm_cfl_dt first");
    if (n_steps > 0) HIPCHK(launch_set_dt(s.d, dt, s.cfl, hs));
    static const double alpha[3] = {0.5, 0.5, 1.0};
    const Dev& d = s.d;
    KernelTimer& t = s.timer;
    // the ghosts are filled once; every update then sets those of its cells
    for (int n = 0; n < n_steps; ++n)
        for (int k = 0; k < 3; ++k) {
            const bool fill = n == 0 && k == 0;
            const void* uin;
            void* uout;
            stage_buffers(d, s.fp32, k, &uin, &uout);
            if (fill)
                HIPCHK(timed(t, MIFVM_K_GHOST_FILL, hs, [&] { return launch_ghost_fill(d, s.fp32, s.bc[0], hs); }));
            HIPCHK(timed(t, MIFVM_K_GRAD_LIMITER, hs,
                         [&] { return launch_grad_limiter(d, s.fp32, hs, false, uin); }));
            HIPCHK(timed(t, MIFVM_K_FV_CELL, hs,
                         [&] { return launch_cell_step(d, s.fp32, s.bc[0], uin, uout, alpha[k], hs); }));
        }
    return MIFVM_OK;
}

}  // extern "C"

namespace mifvm_api {
// n RK3 steps without timing events (the body of a captured step graph)
hipError_t enqueue_steps(const State& s, int n, double dt, hipStream_t q) {
    static const double alpha[3] = {0.5, 0.5, 1.0};
    const Dev& d = s.d;
    hipError_t e = launch_set_dt(d, dt, s.cfl, q);
    // the ghosts are filled once; every update then sets those of its cells
    if (e == hipSuccess && n > 0) e = launch_ghost_fill(d, s.fp32, s.bc[0], q);
    for (int k = 0; e == hipSuccess && k < 3 * n; ++k) {
        const void* uin;
        void* uout;
        stage_buffers(d, s.fp32, k % 3, &uin, &uout);
        e = launch_grad_limiter(d, s.fp32, q, false, uin);
        if (e == hipSuccess) e = launch_cell_step(d, s.fp32, s.bc[0], uin, uout, alpha[k % 3], q);
    }
    return e;
}
}  // namespace mifvm_api

extern "C" {

int mifvm_step_graph(mifvm_state* st, int32_t n_steps, double dt, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    if (n_steps < 0 || !(dt >= 0) || !std::isfinite(dt)) return fail(MIFVM_E_ARG, "bad n_steps or dt");
    State& s = st->s;
    if (dt == 0.0 && !(s.cfl > 0)) return fail(MIFVM_E_STATE, "dt = 0 asks for the CFL steps: call mifvm_cfl_dt first");
    if (n_steps == 0) return MIFVM_OK;
    if (s.step_exec == nullptr || s.step_exec_n != n_steps || s.step_exec_dt != dt || s.step_exec_cfl != s.cfl) {
        HIPCHK(capture_graph(s, &s.step_exec, [&](hipStream_t q) { return enqueue_steps(s, n_steps, dt, q); }));
        s.step_exec_n = n_steps;
        s.step_exec_dt = dt;
        s.step_exec_cfl = s.cfl;
    }
    HIPCHK(hipGraphLaunch(s.step_exec, S(stream)));
    return MIFVM_OK;
}

int mifvm_residual(mifvm_state* st, double* d_res, double* d_grad, double* d_psi, double* d_unode,
                   double* d_flux, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    int rc = residual_parts(s, hs);
    if (rc) return rc;
    if (d_res) {
        HIPCHK(launch_residual_out(d, s.fp32, d.tmp, hs));
        HIPCHK(launch_to_user(d.cell_perm, d.nc, d.nc, d.nc, 1, d.tmp, d_res, hs));
    }
    // FP32 parts are widened into the scratch buffer before being reordered
    auto out = [&](const double* a64, const float* a32, int64_t n, int comps, const int32_t* perm,
                   double* dst) -> int {
        const double* src = a64;
        if (s.fp32) {
            HIPCHK(launch_cast_to_f64(n * comps, a32, d.tmp, hs));
            src = d.tmp;
        }
        if (perm) HIPCHK(launch_to_user(perm, n, n, n, comps, src, dst, hs));
        else HIPCHK(hipMemcpyAsync(dst, src, n * comps * sizeof(double), hipMemcpyDeviceToDevice, hs));
        return MIFVM_OK;
    };
    if (d_grad && (rc = out(d.grad, d.grad32, d.nc, 3, d.cell_perm, d_grad))) return rc;
    if (d_psi && (rc = out(d.psi, d.psi32, d.nc, 1, d.cell_perm, d_psi))) return rc;
    if (d_unode && (rc = out(d.unode, d.unode32, d.nv, 1, d.vert_perm, d_unode))) return rc;
    if (d_flux && (rc = out(d.flux, d.flux32, d.nf, 1, nullptr, d_flux))) return rc;
    return MIFVM_OK;
}

int mifvm_norm_l2(mifvm_state* st, int32_t field, const double* d_exact, double* out, void* stream) {
    if (!st || !out) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    const double* a = nullptr;
    if (field == MIFVM_FIELD_U) {
        if (s.fp32) {
            HIPCHK(launch_cast_to_f64(d.nc, d.u32, d.efield, hs));     // widened into scratch
            a = d.efield;
        } else {
            a = d.u;
        }
    } else if (field == MIFVM_FIELD_P) {
        a = d.x;
    } else if (field == MIFVM_FIELD_ION) {
        a = d.np_ion;
    } else {
        return fail(MIFVM_E_ARG, "norm of FIELD_U, FIELD_P or FIELD_ION");
    }
    const double* e = nullptr;
    if (d_exact) {
        HIPCHK(launch_to_internal(d.cell_perm, d.nc, d.nc, d.nc, 1, d_exact, d.tmp, hs));
        e = d.tmp;
    }
    HIPCHK(launch_norm_l2(d, a, e, hs));
    int rc = pull_scalars(s, hs);
    if (rc) return rc;
    *out = std::sqrt(hsc(s, 0, SC_NORM));
    return MIFVM_OK;
}

int mifvm_conservation(mifvm_state* st, double* total_out, void* stream) {
    if (!st || !total_out) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    hipStream_t hs = S(stream);
    HIPCHK(launch_conservation(s.d, *s.mesh, s.fp32, hs));
    int rc = pull_scalars(s, hs);
    if (rc) return rc;
    double total = 0.0;
    for (int m = 0; m < s.d.nm; ++m) total += hsc(s, m, SC_CONS);
    *total_out = total;
    return MIFVM_OK;
}

}  // extern "C"

namespace {
bool has_matrix(const State& s) { return !s.mesh->kmat.off.empty(); }
}  // namespace

namespace mifvm_api {
// the diagonal, D^-1 and the ghost constants c of the current potential
// BCs, which every solve needs; the matrix-free solves need nothing else
int ensure_mf_tables(State& s, hipStream_t hs) {
    if (!s.mfc_ready) {                       // the matrix-free product's per-cell tables
        HIPCHK(launch_mf_cell_setup(s.d, s.bc[1], hs));
        s.mfc_ready = true;
    }
    return MIFVM_OK;
}

int ensure_consts(State& s, hipStream_t hs) {
    if (int rc = ensure_mf_tables(s, hs)) return rc;
    if (s.assembled || s.consts_ready) return MIFVM_OK;
    HIPCHK(timed(s.timer, MIFVM_K_ASSEMBLE, hs, [&] { return launch_assemble_consts(s.d, s.bc[1], hs); }));
    s.consts_ready = true;
    s.k32_ready = false;                      // the FP32 copies of the diagonal follow it
    return MIFVM_OK;
}
}  // namespace mifvm_api

extern "C" {

int mifvm_poisson_assemble(mifvm_state* st, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    if (!has_matrix(s))
        return fail(MIFVM_E_STATE, "mesh preprocessed without the Poisson matrix (no_matrix): matrix-free solves only");
    hipStream_t hs = S(stream);
    HIPCHK(timed(s.timer, MIFVM_K_ASSEMBLE, hs, [&] { return launch_assemble(s.d, s.bc[1], s.mesh->row_max, hs); }));
    s.assembled = true;
    s.consts_ready = true;
    s.k32_ready = false;
    s.kt_ready = false;
    drop_graphs(s);
    return MIFVM_OK;
}

int mifvm_poisson_apply_free(mifvm_state* st, const double* d_x, double* d_y, void* stream) {
    if (!st || !d_x || !d_y) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    if (int rc = ensure_mf_tables(s, hs)) return rc;
    HIPCHK(launch_to_internal(d.cell_perm, d.nc, d.nc, d.nc, 1, d_x, d.tmp, hs));
    HIPCHK(launch_mf_apply(d, s.bc[1], d.tmp, d.tmp + d.nc, hs));
    HIPCHK(launch_to_user(d.cell_perm, d.nc, d.nc, d.nc, 1, d.tmp + d.nc, d_y, hs));
    return MIFVM_OK;
}

int mifvm_poisson_apply(mifvm_state* st, const double* d_x, double* d_y, void* stream) {
    if (!st || !d_x || !d_y) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    if (!s.assembled) return fail(MIFVM_E_STATE, "poisson system not assembled");
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    HIPCHK(launch_to_internal(d.cell_perm, d.nc, d.nc, d.nc, 1, d_x, d.tmp, hs));
    HIPCHK(launch_spmv_plain(d, d.tmp, d.tmp + d.nc, hs));
    HIPCHK(launch_to_user(d.cell_perm, d.nc, d.nc, d.nc, 1, d.tmp + d.nc, d_y, hs));
    return MIFVM_OK;
}

namespace {
// f_internal: a right-hand side already in internal order (the coupled loop)
int rhs_internal(State& s, const double* d_f, hipStream_t hs, const double* f_internal = nullptr) {
    const Dev& d = s.d;
    if (f_internal) {
        HIPCHK(timed(s.timer, MIFVM_K_RHS, hs, [&] { return launch_rhs(d, f_internal, hs); }));
        s.b_ready = true;
        return MIFVM_OK;
    }
    if (d_f) HIPCHK(launch_to_internal(d.cell_perm, d.nc, d.nc, d.nc, 1, d_f, d.tmp, hs));
    else if (s.fp32) HIPCHK(launch_cast_to_f64(d.nc, d.u32, d.tmp, hs));   // f = the FP32 state, widened
    const double* f = (d_f || s.fp32) ? d.tmp : d.u;
    HIPCHK(timed(s.timer, MIFVM_K_RHS, hs, [&] { return launch_rhs(d, f, hs); }));
    s.b_ready = true;
    return MIFVM_OK;
}
}  // namespace

int mifvm_poisson_rhs(mifvm_state* st, const double* d_f, double* d_b, void* stream) {
    if (!st || !d_b) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    hipStream_t hs = S(stream);
    int rc = ensure_consts(s, hs);
    if (rc) return rc;
    rc = rhs_internal(s, d_f, hs);
    if (rc) return rc;
    HIPCHK(launch_to_user(s.d.cell_perm, s.d.nc, s.d.nc, s.d.nc, 1, s.d.b, d_b, hs));
    return MIFVM_OK;
}

namespace {
int solve_impl(mifvm_state* st, const double* d_f, const double* f_internal, const mifvm_solve_opts* opts,
               mifvm_solve_info* info, void* stream);
}

int mifvm_poisson_solve(mifvm_state* st, const double* d_f, const mifvm_solve_opts* opts,
                        mifvm_solve_info* info, void* stream) {
    return solve_impl(st, d_f, nullptr, opts, info, stream);
}

namespace {
int solve_impl(mifvm_state* st, const double* d_f, const double* f_internal, const mifvm_solve_opts* opts,
               mifvm_solve_info* info, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    const double tol = opts ? opts->tol : 1e-10;
    const int maxit = opts ? opts->maxit : 20000;
    const int chunk = opts && opts->chunk > 0 ? opts->chunk : (s.tuned_chunk > 0 ? s.tuned_chunk : 32);
    const int restart = opts ? opts->restart : 500;
    const int method = opts ? opts->method : MIFVM_SOLVE_PLAIN;
    const int graph_opt = opts ? opts->graph : -1;
    const bool use_graph = !s.timer.on && (graph_opt == 1 || (graph_opt < 0 && s.tuned_graph == 1));
    const double tol_in = opts && opts->inner_tol > 0 ? opts->inner_tol : 1e-4;
    double* hist = opts ? opts->history : nullptr;
    const int hist_cap = opts && opts->history ? opts->history_cap : 0;
    if (!(tol > 0) || maxit < 0 || restart < 0 || hist_cap < 0 || !(tol_in < 1))
        return fail(MIFVM_E_ARG, "bad tol, maxit, restart, inner_tol or history");
    if (method != MIFVM_SOLVE_PLAIN && method != MIFVM_SOLVE_IR_FP32 && method != MIFVM_SOLVE_LEARNED &&
        method != MIFVM_SOLVE_FGMRES && method != MIFVM_SOLVE_AMG)
        return fail(MIFVM_E_ARG, "unknown method");
    const bool learned_smoother = opts && opts->learned_smoother != 0;
    if (method == MIFVM_SOLVE_AMG) {
        if (!s.amg) return fail(MIFVM_E_STATE, "method AMG needs an attached hierarchy (mifvm_amg_build/attach)");
        if (s.d.nm != 1) return fail(MIFVM_E_ARG, "method AMG needs a single-mesh state");
        if (learned_smoother && (!s.nn || !s.nn_state))
            return fail(MIFVM_E_STATE, "learned_smoother needs an attached network");
    }
    if (method == MIFVM_SOLVE_FGMRES) {
        if (!s.gm) return fail(MIFVM_E_STATE, "method FGMRES needs a workspace (mifvm_fgmres_attach)");
        if (s.d.nm != 1) return fail(MIFVM_E_ARG, "method FGMRES needs a single-mesh state");
    }
    const bool matrix_free = opts && opts->matrix_free != 0;
    // the stored K is read by every solve that does not apply K matrix-free,
    // and by the multigrid hierarchy (built from it)
    if (!matrix_free && !s.assembled) return fail(MIFVM_E_STATE, "poisson system not assembled");
    const int stall_window = opts ? opts->stall_window : 0;
    const int learned_maxit = opts ? opts->learned_maxit : 0;
    if (stall_window < 0 || learned_maxit < 0) return fail(MIFVM_E_ARG, "bad stall_window or learned_maxit");
    if (method == MIFVM_SOLVE_LEARNED) {
        if (!s.nn || !s.nn_state) return fail(MIFVM_E_STATE, "method LEARNED needs an attached network");
        if (s.d.nm != 1) return fail(MIFVM_E_ARG, "method LEARNED needs a single-mesh state");
    }
    const Dev& d = s.d;
    const int nm = d.nm;
    hipStream_t hs = S(stream);
    s.mf = matrix_free;
    auto t0 = std::chrono::steady_clock::now();
    int rc = ensure_consts(s, hs);
    if (rc) return rc;
    rc = rhs_internal(s, d_f, hs, f_internal);
    if (rc) return rc;
    KernelTimer& tm = s.timer;
    int nhist = 0;
    // every mesh's scalars to the host; the history records the largest
    // recurrence residual over the meshes
    auto pull = [&]() -> int {
        int r = pull_scalars(s, hs);
        if (r) return r;
        HIPCHK(timer_flush(tm));
        if (nhist < hist_cap) {
            double worst = 0.0;
            for (int m = 0; m < nm; ++m) {
                const double bb = hsc(s, m, SC_BB);
                if (bb > 0) worst = std::fmax(worst, std::sqrt(hsc(s, m, SC_RR) / bb));
            }
            hist[nhist++] = worst;
        }
        return MIFVM_OK;
    };
    auto any_running = [&]() {
        for (int m = 0; m < nm; ++m)
            if (hsc(s, m, SC_DONE) == 0.0) return true;
        return false;
    };
    // learned: flexible CG first; the plain solver finishes after a fallback
    LearnedRun learned;
    int budget = maxit;
    if (method == MIFVM_SOLVE_LEARNED) {
        rc = learned_phase(s, tol, maxit, chunk, restart, stall_window, learned_maxit, use_graph, hs, pull, learned);
        if (rc) return rc;
        budget = maxit - learned.iterations;
    }
    const int run_method = method == MIFVM_SOLVE_LEARNED ? MIFVM_SOLVE_PLAIN : method;
    const int graph_key = run_method + (matrix_free ? 16 : 0);
    if (use_graph && (method != MIFVM_SOLVE_LEARNED || learned.fell_back) && method != MIFVM_SOLVE_AMG &&
        method != MIFVM_SOLVE_FGMRES && (s.cg_exec == nullptr || s.cg_exec_chunk != chunk || s.cg_exec_method != graph_key)) {
        HIPCHK(capture_graph(s, &s.cg_exec, [&](hipStream_t q) { return enqueue_cg_chunk(s, run_method, chunk, q); }));
        s.cg_exec_chunk = chunk;
        s.cg_exec_method = graph_key;
    }
    // one chunk of iterations: a graph replay, or timed direct launches
    auto run_chunk = [&]() -> int {
        if (use_graph) {
            HIPCHK(hipGraphLaunch(s.cg_exec, hs));
            return MIFVM_OK;
        }
        for (int c = 0; c < chunk; ++c) {
            if (run_method == MIFVM_SOLVE_PLAIN) {
                if (matrix_free) {
                    for (int part = 0; part < kMfParts; ++part)
                        HIPCHK(timed(tm, (part == 0 ? MIFVM_K_MF_VERTEX : part == 1 ? MIFVM_K_MF_GATHER : MIFVM_K_CG_ALPHA), hs,
                                     [&] { return launch_mf_cg_part(d, s.bc[1], part, hs); }));
                } else {
                    HIPCHK(timed(tm, MIFVM_K_CG_SPMV, hs, [&] { return launch_cg_spmv(d, hs); }));
                }
                HIPCHK(timed(tm, MIFVM_K_CG_AXPY, hs, [&] { return launch_cg_axpy(d, hs); }));
                HIPCHK(timed(tm, MIFVM_K_CG_DIR, hs, [&] { return launch_cg_dir(d, hs); }));
            } else if (matrix_free) {
                for (int part = 0; part < kMfParts; ++part)
                    HIPCHK(timed(tm, (part == 0 ? MIFVM_K_MF_VERTEX : part == 1 ? MIFVM_K_MF_GATHER : MIFVM_K_CG_ALPHA), hs,
                                 [&] { return launch_mf_cg32_part(d, s.bc[1], part, hs); }));
                HIPCHK(timed(tm, MIFVM_K_CG_AXPY, hs, [&] { return launch_cg32_axpy(d, hs); }));
                HIPCHK(timed(tm, MIFVM_K_CG_DIR, hs, [&] { return launch_cg32_dir(d, hs); }));
            } else {
                HIPCHK(timed(tm, MIFVM_K_CG_SPMV, hs, [&] { return launch_cg32_spmv(d, hs); }));
                HIPCHK(timed(tm, MIFVM_K_CG_AXPY, hs, [&] { return launch_cg32_axpy(d, hs); }));
                HIPCHK(timed(tm, MIFVM_K_CG_DIR, hs, [&] { return launch_cg32_dir(d, hs); }));
            }
        }
        return MIFVM_OK;
    };
    int restarts = learned.restarts, outer = 0;
    if (method == MIFVM_SOLVE_FGMRES) {
        const GmDev& g = *s.gm;
        const BcTable& bcp = s.bc[1];
        auto open = [&](bool fresh) -> int {
            HIPCHK(timed(tm, MIFVM_K_CG_SETUP, hs, [&]() -> hipError_t {
                if (matrix_free) {
                    hipError_t e = launch_mf_apply(d, bcp, d.x, d.tmp, hs);
                    if (e != hipSuccess) return e;
                }
                return launch_gm_open(d, g, matrix_free ? d.tmp : nullptr, tol, maxit, fresh, hs);
            }));
            return pull();
        };
        auto step_spmv = [&](int j, hipStream_t q) {
            return matrix_free ? launch_mf_apply(d, bcp, g.Z + int64_t(j) * d.nc, g.V + int64_t(j + 1) * d.nc, q,
                                                 d.scal + SC_DONE)
                               : launch_gm_spmv(d, g, j, q);
        };
        auto enqueue_cycle = [&](hipStream_t q) -> hipError_t {
            for (int j = 0; j < g.m; ++j) {
                hipError_t e = step_spmv(j, q);
                if (e == hipSuccess) e = launch_gm_orth(d, g, j, q);
                if (e != hipSuccess) return e;
            }
            return launch_gm_close(d, g, q);
        };
        const int key = g.m + (matrix_free ? 1 << 20 : 0);
        if (use_graph && (s.gm_exec == nullptr || s.gm_exec_key != key)) {
            HIPCHK(capture_graph(s, &s.gm_exec, enqueue_cycle));
            s.gm_exec_key = key;
        }
        if ((rc = open(true))) return rc;
        while (hsc(s, 0, SC_DONE) == 0.0) {
            if (use_graph) {
                HIPCHK(hipGraphLaunch(s.gm_exec, hs));
            } else {
                for (int j = 0; j < g.m; ++j) {
                    HIPCHK(timed(tm, MIFVM_K_CG_SPMV, hs, [&] { return step_spmv(j, hs); }));
                    HIPCHK(timed(tm, MIFVM_K_CG_AXPY, hs, [&] { return launch_gm_orth(d, g, j, hs); }));
                }
                HIPCHK(timed(tm, MIFVM_K_CG_DIR, hs, [&] { return launch_gm_close(d, g, hs); }));
            }
            ++outer;
            if ((rc = open(false))) return rc;       // the true residual decides
            if (hsc(s, 0, SC_DONE) == 0.0) ++restarts;
        }
    } else if (method == MIFVM_SOLVE_AMG) {
        if ((rc = amg_phase(s, tol, maxit, chunk, restart, use_graph, matrix_free, learned_smoother, hs, pull,
                            restarts)))
            return rc;
    } else if (method == MIFVM_SOLVE_LEARNED && !learned.fell_back) {
        // the flexible CG ended: converged, or at maxit
    } else if (run_method == MIFVM_SOLVE_PLAIN) {
        // r = b - K x with K x from the matrix-free product or the stored K
        auto setup = [&](int limit, bool fresh) -> hipError_t {
            if (matrix_free) {
                hipError_t e = launch_mf_apply(d, s.bc[1], d.x, d.tmp, hs);
                if (e != hipSuccess) return e;
            }
            return launch_cg_setup(d, tol, limit, restart, fresh, hs, matrix_free ? d.tmp : nullptr);
        };
        HIPCHK(timed(tm, MIFVM_K_CG_SETUP, hs, [&] { return setup(budget, true); }));
        if ((rc = pull())) return rc;
        while (any_running()) {
            while (any_running()) {
                if ((rc = run_chunk())) return rc;
                if ((rc = pull())) return rc;
            }
            // every mesh's recurrence converged, reached its limit or is due a
            // restart: recompute the true residual r = b - K x (FP64) and reopen
            HIPCHK(timed(tm, MIFVM_K_CG_SETUP, hs, [&] { return setup(maxit, false); }));
            if ((rc = pull())) return rc;
            if (any_running()) ++restarts;
        }
    } else {
        if (!s.k32_ready) {
            HIPCHK(launch_cast_matrix(d, (int64_t)s.mesh->kmat.idx.size(), hs));
            s.k32_ready = true;
        }
        bool fresh = true;
        for (;;) {
            HIPCHK(timed(tm, MIFVM_K_CG_SETUP, hs, [&]() -> hipError_t {
                if (matrix_free) {      // K x by the FP64 matrix-free product
                    hipError_t e = launch_mf_apply(d, s.bc[1], d.x, d.tmp, hs);
                    if (e != hipSuccess) return e;
                }
                return launch_ir_residual(d, tol, tol_in, maxit, restart, fresh, matrix_free ? d.tmp : nullptr, hs);
            }));
            fresh = false;
            if ((rc = pull())) return rc;
            if (!any_running()) break;                   // every mesh converged, or at its limit
            while (any_running()) {
                if ((rc = run_chunk())) return rc;
                if ((rc = pull())) return rc;
            }
            HIPCHK(launch_ir_update(d, hs));
            ++outer;
        }
    }
    // per-mesh outcome; b = 0 on a mesh: its solution is 0
    s.last_iters.assign(nm, 0);
    s.last_rel.assign(nm, 0.0);
    int iters = 0;
    double rel = 0.0;
    for (int m = 0; m < nm; ++m) {
        const double bb = hsc(s, m, SC_BB);
        if (bb == 0.0) {
            const int64_t lo = s.mesh->mesh_start[m], hi = s.mesh->mesh_start[m + 1];
            HIPCHK(hipMemsetAsync(d.x + lo, 0, (hi - lo) * sizeof(double), hs));
        }
        s.last_rel[m] = bb > 0 ? std::sqrt(hsc(s, m, SC_TRUE_RR) / bb) : 0.0;
        s.last_iters[m] = int(hsc(s, m, SC_IT)) + (learned.fell_back ? learned.iterations : 0);
        iters = std::max(iters, s.last_iters[m]);
        rel = std::fmax(rel, s.last_rel[m]);
    }
    HIPCHK(hipStreamSynchronize(hs));
    if (info) {
        info->iterations = iters;
        info->restarts = restarts;
        info->history_len = nhist;
        info->outer = outer;
        info->rel_residual = rel;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        info->fell_back = learned.fell_back ? 1 : 0;
        info->learned_iterations = learned.iterations;
    }
    if (!(rel <= tol)) return MIFVM_NOT_CONVERGED;
    return learned.fell_back ? MIFVM_FELL_BACK : MIFVM_OK;
}
}  // namespace

int mifvm_streamer_step(mifvm_state* st, int32_t n_steps, const mifvm_streamer_opts* opts,
                        mifvm_streamer_info* info, void* stream) {
    if (!st || !opts) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    if (n_steps < 0) return fail(MIFVM_E_ARG, "n_steps must be >= 0");
    if (!(opts->mobility >= 0) || !std::isfinite(opts->mobility) || !std::isfinite(opts->charge_scale) ||
        !(opts->alpha_a >= 0) || !std::isfinite(opts->alpha_a) || !(opts->alpha_b >= 0) ||
        !std::isfinite(opts->alpha_b) || !(opts->cfl > 0) || !std::isfinite(opts->cfl) || opts->tol < 0 ||
        opts->maxit < 0 || opts->restart < 0)
        return fail(MIFVM_E_ARG, "bad streamer options");
    if (s.fp32) return fail(MIFVM_E_STATE, "the coupled loop runs on FP64 states");
    if (!opts->matrix_free && !s.assembled) return fail(MIFVM_E_STATE, "poisson system not assembled");
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    mifvm_solve_opts so{};
    so.tol = opts->tol > 0 ? opts->tol : 1e-10;
    so.maxit = opts->maxit > 0 ? opts->maxit : 20000;
    so.restart = opts->restart > 0 ? opts->restart : 500;
    so.method = MIFVM_SOLVE_PLAIN;
    so.graph = -1;
    so.matrix_free = opts->matrix_free ? 1 : 0;
    mifvm_streamer_info out{};
    for (int n = 0; n < n_steps; ++n) {
        // Delta P = kappa (n_e - n_p), warm-started from the last P
        HIPCHK(launch_streamer_rhs(d, opts->charge_scale, d.tmp, hs));
        mifvm_solve_info si{};
        int rc = solve_impl(st, nullptr, d.tmp, &so, &si, stream);
        out.iterations_max = std::max(out.iterations_max, si.iterations);
        out.iterations_sum += si.iterations;
        if (rc) {
            if (info) *info = out;
            return rc;
        }
        // E, v_e and S_e per cell; face velocities; the CFL step; n_p
        HIPCHK(launch_streamer_fields(d, s.bc[1], opts->mobility, opts->alpha_a, opts->alpha_b, hs));
        HIPCHK(launch_face_phi(d, hs));
        s.vel_set = true;
        double dt = 0.0;
        if ((rc = mifvm_cfl_dt(st, opts->cfl, &dt, stream))) return rc;
        if ((rc = mifvm_step(st, 1, 0.0, stream))) return rc;
        HIPCHK(launch_ion_update(d, hs));
        out.steps += 1;
        out.time += dt;
        out.last_dt = dt;
    }
    HIPCHK(hipStreamSynchronize(hs));
    if (info) *info = out;
    return MIFVM_OK;
}

int mifvm_fgmres_bytes(const mifvm_state* st, int32_t m, size_t* out) {
    if (!st || !out) return fail(MIFVM_E_ARG, "null argument");
    if (m < 1 || m > kGmMaxM) return fail(MIFVM_E_ARG, "m must be in [1, 64]");
    GmDev probe{};
    *out = gm_layout(st->s.d.nc, m, nullptr, probe);
    return MIFVM_OK;
}

int mifvm_fgmres_attach(mifvm_state* st, int32_t m, void* d_ws, size_t ws_bytes) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    if (s.gm_exec) (void)hipGraphExecDestroy(s.gm_exec);
    s.gm_exec = nullptr;
    if (!d_ws) {
        delete s.gm;
        s.gm = nullptr;
        return MIFVM_OK;
    }
    if (s.d.nm != 1) return fail(MIFVM_E_ARG, "FGMRES needs a single-mesh state");
    if (m < 1 || m > kGmMaxM) return fail(MIFVM_E_ARG, "m must be in [1, 64]");
    if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(MIFVM_E_WORKSPACE, "workspace not 256-byte aligned");
    GmDev probe{};
    const size_t need = gm_layout(s.d.nc, m, nullptr, probe);
    if (ws_bytes < need) return fail(MIFVM_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
    auto* g = new (std::nothrow) GmDev();
    if (!g) return fail(MIFVM_E_ARG, "out of host memory");
    gm_layout(s.d.nc, m, static_cast<char*>(d_ws), *g);
    delete s.gm;
    s.gm = g;
    return MIFVM_OK;
}

int mifvm_mesh_values(const mifvm_state* st, int32_t what, double* out, int32_t n) {
    if (!st || !out) return fail(MIFVM_E_ARG, "null argument");
    const State& s = st->s;
    if (n != s.d.nm) return fail(MIFVM_E_ARG, "need one value per mesh");
    for (int m = 0; m < n; ++m) {
        switch (what) {
            case 0: out[m] = s.cfl * hsc(s, m, SC_DT_INV); break;
            case 1: out[m] = hsc(s, m, SC_CONS); break;
            case 2: out[m] = m < int(s.last_iters.size()) ? double(s.last_iters[m]) : 0.0; break;
            case 3: out[m] = m < int(s.last_rel.size()) ? s.last_rel[m] : 0.0; break;
            default: return fail(MIFVM_E_ARG, "unknown value id");
        }
    }
    return MIFVM_OK;
}

}  // extern "C"

namespace {
std::map<std::string, std::array<int, 3>> read_tune_cache(const char* path) {
    std::map<std::string, std::array<int, 3>> out;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        char key[256];
        int c = 0, g = 0, sg = 0;
        if (std::sscanf(line.c_str(), " \"%255[^\"]\": {\"chunk\": %d, \"graph\": %d, \"step_graph\": %d}", key, &c,
                        &g, &sg) == 4)
            out[key] = {c, g, sg};
    }
    return out;
}

void write_tune_cache(const char* path, const std::map<std::string, std::array<int, 3>>& m) {
    std::ofstream o(path);
    o << "{\n";
    size_t k = 0;
    for (auto& kv : m) {
        o << "  \"" << kv.first << "\": {\"chunk\": " << kv.second[0] << ", \"graph\": " << kv.second[1]
          << ", \"step_graph\": " << kv.second[2] << "}" << (++k < m.size() ? "," : "") << "\n";
    }
    o << "}\n";
}
}  // namespace

extern "C" {

int mifvm_autotune(mifvm_state* st, const char* cache_path, mifvm_tune_info* out, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    if (!s.assembled) return fail(MIFVM_E_STATE, "autotune times the solve: assemble first");
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= d.nc) ++lg;
    const std::string key = "gfx950/" + std::to_string(d.nm) + "/" + std::to_string(lg);
    mifvm_tune_info info{};
    std::map<std::string, std::array<int, 3>> cache;
    if (cache_path) {
        cache = read_tune_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            s.tuned_chunk = it->second[0];
            s.tuned_graph = it->second[1];
            s.tuned_step_graph = it->second[2];
            info.chunk = s.tuned_chunk;
            info.graph = s.tuned_graph;
            info.step_graph = s.tuned_step_graph;
            info.from_cache = 1;
            if (out) *out = info;
            return MIFVM_OK;
        }
    }
    const bool timing_was_on = s.timer.on;
    if (!s.timer.pending.empty()) return fail(MIFVM_E_STATE, "collect kernel timing first");
    s.timer.on = false;
    const int64_t NX = d.nc + d.nb;
    double* saved_x = d.tmp + NX;                    // P is restored after the trials
    HIPCHK(hipMemcpyAsync(saved_x, d.x, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
    auto clock_ms = [&](auto fn) -> double {
        HIPCHK(hipStreamSynchronize(hs));
        auto t0 = std::chrono::steady_clock::now();
        int r = fn();
        HIPCHK(hipStreamSynchronize(hs));
        if (r) return -1.0;
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    double best = 1e300;
    int best_chunk = 32, best_graph = 0;
    for (int chunk : {8, 16, 32, 64}) {
        for (int graph : {0, 1}) {
            HIPCHK(hipMemcpyAsync(d.x, saved_x, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
            mifvm_solve_opts o{};
            o.tol = 1e-300;                           // never met: exactly maxit iterations
            o.maxit = 4 * chunk < 128 ? 128 : 4 * chunk;
            o.chunk = chunk;
            o.restart = 0;
            o.graph = graph;
            o.method = MIFVM_SOLVE_PLAIN;
            mifvm_solve_info si{};
            const double ms = clock_ms([&]() {
                const int r = mifvm_poisson_solve(st, nullptr, &o, &si, stream);
                return r == MIFVM_NOT_CONVERGED ? 0 : r;
            });
            if (ms < 0) return MIFVM_E_HIP;
            const double per = ms / std::max(si.iterations, 1);
            if (per < best) {
                best = per;
                best_chunk = chunk;
                best_graph = graph;
            }
        }
    }
    HIPCHK(hipMemcpyAsync(d.x, saved_x, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
    // one step, direct launches against a graph replay; the state is restored
    double* saved_u = d.tmp + 2 * NX;
    float* saved_u32 = d.d32;                         // inner-CG scratch, free here
    HIPCHK(hipMemcpyAsync(saved_u, d.u, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
    HIPCHK(hipMemcpyAsync(saved_u32, d.u32, d.nc * sizeof(float), hipMemcpyDeviceToDevice, hs));
    const double dt = 1e-12;
    auto restore_u = [&]() -> int {
        HIPCHK(hipMemcpyAsync(d.u, saved_u, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
        HIPCHK(hipMemcpyAsync(d.u32, saved_u32, d.nc * sizeof(float), hipMemcpyDeviceToDevice, hs));
        HIPCHK(launch_ghost_fill(d, s.fp32, s.bc[0], hs));
        return MIFVM_OK;
    };
    const double t_direct = clock_ms([&]() { return mifvm_step(st, 2, dt, stream); });
    int rc = restore_u();
    if (rc) return rc;
    rc = mifvm_step_graph(st, 2, dt, stream);         // capture outside the timed call
    if (rc) return rc;
    rc = restore_u();
    if (rc) return rc;
    const double t_graph = clock_ms([&]() { return mifvm_step_graph(st, 2, dt, stream); });
    rc = restore_u();
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(hs));
    s.timer.on = timing_was_on;
    s.tuned_chunk = best_chunk;
    s.tuned_graph = best_graph;
    s.tuned_step_graph = t_graph < t_direct ? 1 : 0;
    info.chunk = best_chunk;
    info.graph = best_graph;
    info.step_graph = s.tuned_step_graph;
    info.ms_per_iteration = best;
    info.ms_per_step_direct = t_direct / 2;
    info.ms_per_step_graph = t_graph / 2;
    if (cache_path) {
        cache[key] = {best_chunk, best_graph, s.tuned_step_graph};
        write_tune_cache(cache_path, cache);
    }
    if (out) *out = info;
    return MIFVM_OK;
}

}  // extern "C"
