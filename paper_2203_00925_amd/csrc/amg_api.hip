// C ABI of the aggregation multigrid preconditioner (include/mifvm.h):
// hierarchy setup on the host from the state's assembled K, upload into a
// caller workspace, the V-cycle as an operator, the multigrid-preconditioned
// flexible CG, and a host-only build for inspection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>

#include "amg_dev.h"
#include "api_util.h"
#include "mifvm.h"

using namespace mifvm;
using namespace mifvm_api;

struct mifvm_amg_host {
    AmgHierarchy h;
};

namespace {

int read_opts(const mifvm_amg_opts* o, double& theta, int& levels, int64_t& cmax, double& omega) {
    theta = o && o->theta > 0 ? o->theta : 0.25;
    levels = o && o->max_levels > 0 ? o->max_levels : 10;
    cmax = o && o->coarse_max > 0 ? o->coarse_max : 1024;
    omega = o && o->omega > 0 ? o->omega : 2.0 / 3.0;
    return MIFVM_OK;
}

void fill_info(const AmgHierarchy& h, mifvm_amg_info* info) {
    std::memset(info, 0, sizeof(*info));
    info->levels = int32_t(h.lv.size());
    for (size_t l = 0; l < h.lv.size() && l < 16; ++l) {
        info->rows[l] = h.lv[l].A.n;
        info->nnz[l] = (int64_t)h.lv[l].A.col.size();
    }
}

// device bytes of a hierarchy (level 0 lives in the state)
size_t amg_layout(const AmgHierarchy& h, int64_t nc, char* base, AmgDev* a) {
    size_t off = 0;
    AmgDev tmp;
    AmgDev& A = a ? *a : tmp;
    A.nl = int(h.lv.size());
    A.omega = h.omega;
    A.gamma = h.gamma;
    for (int l = 0; l < A.nl; ++l) {
        const AmgLevel& L = h.lv[l];
        AmgLevelDev& D = A.lv[l];
        D.n = L.A.n;
        if (l >= 1) {
            Sell64 s;
            std::vector<double> diag;
            amg_pack(L.A, s, diag);
            D.off = carve<int64_t>(base, off, s.off.size());
            D.w = carve<int32_t>(base, off, std::max<size_t>(s.width.size(), 1));
            D.idx = carve<int32_t>(base, off, std::max<size_t>(s.idx.size(), 1));
            D.val = carve<double>(base, off, std::max<size_t>(s.val.size(), 1));
            D.diag = carve<double>(base, off, D.n);
            D.dinv = carve<double>(base, off, D.n);
            D.b = carve<double>(base, off, D.n);
            D.x = carve<double>(base, off, D.n);
            D.t = carve<double>(base, off, D.n);
            D.r = carve<double>(base, off, D.n);
            D.e = carve<double>(base, off, D.n);
        }
        if (l + 1 < A.nl) {
            D.agg = carve<int32_t>(base, off, D.n);
            D.mptr = carve<int64_t>(base, off, L.ncoarse + 1);
            D.midx = carve<int32_t>(base, off, D.n);
        }
    }
    A.cinv = carve<double>(base, off, h.cinv.size());
    A.r_old = carve<double>(base, off, nc);
    A.s0 = carve<double>(base, off, nc);
    A.s1 = carve<double>(base, off, nc);
    return (off + 255) & ~size_t(255);
}

// K of the state (64-row slices + diagonal on the device) as host CSR
int state_matrix(State& s, hipStream_t hs, AmgCsr& A) {
    const Mesh& m = *s.mesh;
    const Dev& d = s.d;
    std::vector<double> val(m.kmat.idx.size()), diag(m.nc);
    HIPCHK(hipMemcpyAsync(val.data(), d.k_val, val.size() * sizeof(double), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipMemcpyAsync(diag.data(), d.k_diag, diag.size() * sizeof(double), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    A.n = m.nc;
    A.ptr.assign(m.nc + 1, 0);
    for (int64_t i = 0; i < m.nc; ++i) A.ptr[i + 1] = A.ptr[i] + 1 + m.klen[i];
    A.col.resize(A.ptr[m.nc]);
    A.val.resize(A.ptr[m.nc]);
    // rows are independent: sorted by column in parallel chunks
    for_chunks(m.nc, setup_threads(m.nc), [&](int, int64_t lo, int64_t hi) {
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t sl = i >> 6, lane = i & 63;
            row.clear();
            row.emplace_back(int32_t(i), diag[i]);
            for (int32_t k = 0; k < m.klen[i]; ++k) {
                const int64_t at = m.kmat.off[sl] + int64_t(k) * 64 + lane;
                row.emplace_back(m.kmat.idx[at], val[at]);
            }
            std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
            int64_t at = A.ptr[i];
            for (auto& e : row) {
                A.col[at] = e.first;
                A.val[at] = e.second;
                ++at;
            }
        }
    });
    return MIFVM_OK;
}

}  // namespace

namespace mifvm_api {

void amg_release(State& s) {
    if (s.amg_exec) (void)hipGraphExecDestroy(s.amg_exec);
    s.amg_exec = nullptr;
    delete s.amg;
    s.amg = nullptr;
    delete s.amg_host;
    s.amg_host = nullptr;
}

int amg_phase(State& s, double tol, int maxit, int chunk, int restart, bool use_graph, bool matrix_free,
              bool learned, hipStream_t hs, const std::function<int()>& pull, int& restarts) {
    const Dev& d = s.d;
    const AmgDev& a = *s.amg;
    const BcTable& bc = s.bc[1];
    KernelTimer& tm = s.timer;
    // the attached network as the finest level's smoother
    const AmgSmoother nn = [&s](const double* in, double* out, hipStream_t q) { return nn_apply_vec(s, in, out, q); };
    const AmgSmoother* fine = learned ? &nn : nullptr;
    auto open = [&](bool fresh) -> int {
        HIPCHK(timed(tm, MIFVM_K_CG_SETUP, hs,
                     [&] { return launch_amg_open(d, bc, a, tol, maxit, restart, fresh, hs, fine); }));
        return pull();
    };
    const int key = chunk + (matrix_free ? 1 << 20 : 0) + (learned ? 1 << 21 : 0);
    if (use_graph && (s.amg_exec == nullptr || s.amg_exec_key != key)) {
        HIPCHK(capture_graph(s, &s.amg_exec, [&](hipStream_t q) -> hipError_t {
            for (int c = 0; c < chunk; ++c) {
                hipError_t e = launch_amg_iteration(d, bc, a, matrix_free, q, fine);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }));
        s.amg_exec_key = key;
    }
    auto running = [&]() { return hsc(s, 0, SC_DONE) == 0.0; };
    int rc = open(true);
    if (rc) return rc;
    while (running()) {
        while (running()) {
            if (use_graph) {
                HIPCHK(hipGraphLaunch(s.amg_exec, hs));
            } else {
                for (int c = 0; c < chunk; ++c)
                    HIPCHK(timed(tm, MIFVM_K_CG_SPMV, hs,
                                 [&] { return launch_amg_iteration(d, bc, a, matrix_free, hs, fine); }));
            }
            if ((rc = pull())) return rc;
        }
        // the recurrence converged, hit its limit or is due a restart: reopen
        // from the true residual
        if ((rc = open(false))) return rc;
        if (running()) ++restarts;
    }
    return MIFVM_OK;
}

}  // namespace mifvm_api

extern "C" {

int mifvm_amg_build(mifvm_state* st, const mifvm_amg_opts* opts, mifvm_amg_info* info, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    if (!s.assembled) return fail(MIFVM_E_STATE, "poisson system not assembled");
    if (s.d.nm != 1) return fail(MIFVM_E_ARG, "the multigrid preconditioner needs a single-mesh state");
    if (opts && (opts->cycle < 0 || opts->cycle > 2)) return fail(MIFVM_E_ARG, "cycle must be 0 or 1 (V) or 2 (W)");
    double theta, omega;
    int levels;
    int64_t cmax;
    read_opts(opts, theta, levels, cmax, omega);
    const auto t0 = std::chrono::steady_clock::now();
    AmgCsr A;
    int rc = state_matrix(s, S(stream), A);
    if (rc) return rc;
    auto h = std::make_unique<AmgHierarchy>();
    std::string err;
    rc = amg_build(std::move(A), theta, levels, cmax, omega, *h, err);
    if (rc) return fail(rc, err);
    h->gamma = opts && opts->cycle == 2 ? 2 : 1;
    amg_release(s);
    s.amg_host = h.release();
    if (info) {
        fill_info(*s.amg_host, info);
        info->ws_bytes = amg_layout(*s.amg_host, s.d.nc, nullptr, nullptr);
        info->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return MIFVM_OK;
}

int mifvm_amg_attach(mifvm_state* st, void* d_ws, size_t ws_bytes, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    if (!d_ws) {
        if (s.amg_exec) (void)hipGraphExecDestroy(s.amg_exec);
        s.amg_exec = nullptr;
        delete s.amg;
        s.amg = nullptr;
        return MIFVM_OK;
    }
    if (!s.amg_host) return fail(MIFVM_E_STATE, "no hierarchy: call mifvm_amg_build first");
    const AmgHierarchy& h = *s.amg_host;
    const size_t need = amg_layout(h, s.d.nc, nullptr, nullptr);
    if (ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) & 255))
        return fail(MIFVM_E_WORKSPACE, "multigrid workspace too small or misaligned: need " + std::to_string(need));
    auto a = std::make_unique<AmgDev>();
    amg_layout(h, s.d.nc, static_cast<char*>(d_ws), a.get());
    hipStream_t hs = S(stream);
    for (int l = 0; l < a->nl; ++l) {
        const AmgLevel& L = h.lv[l];
        AmgLevelDev& D = a->lv[l];
        if (l >= 1) {
            Sell64 sl;
            std::vector<double> diag;
            amg_pack(L.A, sl, diag);
            std::vector<double> dinv(diag.size());
            for (size_t i = 0; i < diag.size(); ++i) {
                if (!(diag[i] != 0.0) || !std::isfinite(diag[i]))
                    return fail(MIFVM_E_STATE, "zero or non-finite diagonal on a coarse level");
                dinv[i] = 1.0 / diag[i];
            }
            HIPCHK(up(D.off, sl.off, hs));
            HIPCHK(up(D.w, sl.width, hs));
            HIPCHK(up(D.idx, sl.idx, hs));
            HIPCHK(up(D.val, sl.val, hs));
            HIPCHK(up(D.diag, diag, hs));
            HIPCHK(up(D.dinv, dinv, hs));
            HIPCHK(hipStreamSynchronize(hs));       // the packed host vectors are freed here
        }
        if (l + 1 < a->nl) {
            std::vector<int64_t> mptr(L.ncoarse + 1, 0);
            for (int32_t g : L.agg) mptr[g + 1]++;
            for (int64_t k = 0; k < L.ncoarse; ++k) mptr[k + 1] += mptr[k];
            std::vector<int32_t> midx(L.A.n);
            std::vector<int64_t> pos(mptr.begin(), mptr.end() - 1);
            for (int64_t i = 0; i < L.A.n; ++i) midx[pos[L.agg[i]]++] = int32_t(i);
            HIPCHK(up(D.agg, L.agg, hs));
            HIPCHK(up(D.mptr, mptr, hs));
            HIPCHK(up(D.midx, midx, hs));
            HIPCHK(hipStreamSynchronize(hs));
        }
    }
    HIPCHK(up(a->cinv, h.cinv, hs));
    HIPCHK(hipStreamSynchronize(hs));
    if (s.amg_exec) (void)hipGraphExecDestroy(s.amg_exec);
    s.amg_exec = nullptr;
    delete s.amg;
    s.amg = a.release();
    return MIFVM_OK;
}

int mifvm_amg_apply(mifvm_state* st, int32_t learned_smoother, const double* d_r, double* d_z, void* stream) {
    if (!st || !d_r || !d_z) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    if (!s.amg) return fail(MIFVM_E_STATE, "no multigrid attached");
    if (learned_smoother && (!s.nn || !s.nn_state)) return fail(MIFVM_E_STATE, "no network attached");
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    const AmgSmoother nn = [&s](const double* in, double* out, hipStream_t q) { return nn_apply_vec(s, in, out, q); };
    if (int rc = ensure_mf_tables(s, hs)) return rc;      // the finest level's matrix-free product
    HIPCHK(launch_to_internal(d.cell_perm, d.nc, d.nc, d.nc, 1, d_r, d.r, hs));
    HIPCHK(launch_amg_cycle(d, s.bc[1], *s.amg, d.r, d.z, nullptr, hs, learned_smoother ? &nn : nullptr));
    HIPCHK(launch_to_user(d.cell_perm, d.nc, d.nc, d.nc, 1, d.z, d_z, hs));
    return MIFVM_OK;
}

int mifvm_amg_host_build(int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                         const mifvm_amg_opts* opts, mifvm_amg_host** out) {
    if (!ptr || !col || !val || !out || n < 1) return fail(MIFVM_E_ARG, "null or empty argument");
    *out = nullptr;
    AmgCsr A;
    A.n = n;
    A.ptr.assign(ptr, ptr + n + 1);
    if (A.ptr[0] != 0) return fail(MIFVM_E_ARG, "row pointer must start at 0");
    for (int64_t i = 0; i < n; ++i)
        if (A.ptr[i + 1] < A.ptr[i]) return fail(MIFVM_E_ARG, "row pointer not ascending");
    A.col.assign(col, col + A.ptr[n]);
    A.val.assign(val, val + A.ptr[n]);
    for (int32_t c : A.col)
        if (c < 0 || c >= n) return fail(MIFVM_E_ARG, "column index out of range");
    double theta, omega;
    int levels;
    int64_t cmax;
    read_opts(opts, theta, levels, cmax, omega);
    auto h = std::make_unique<mifvm_amg_host>();
    std::string err;
    const int rc = amg_build(std::move(A), theta, levels, cmax, omega, h->h, err);
    if (rc) return fail(rc, err);
    *out = h.release();
    return MIFVM_OK;
}

int mifvm_amg_host_info(const mifvm_amg_host* h, mifvm_amg_info* info) {
    if (!h || !info) return fail(MIFVM_E_ARG, "null argument");
    fill_info(h->h, info);
    return MIFVM_OK;
}

int mifvm_amg_host_export(const mifvm_amg_host* h, int32_t level, int32_t what, void* dst, size_t bytes) {
    if (!h || !dst) return fail(MIFVM_E_ARG, "null argument");
    if (level < 0 || level >= int32_t(h->h.lv.size())) return fail(MIFVM_E_ARG, "no such level");
    const AmgLevel& L = h->h.lv[level];
    const void* src = nullptr;
    size_t n = 0;
    switch (what) {
        case 0: src = L.agg.data(); n = L.agg.size() * 4; break;
        case 1: src = L.A.ptr.data(); n = L.A.ptr.size() * 8; break;
        case 2: src = L.A.col.data(); n = L.A.col.size() * 4; break;
        case 3: src = L.A.val.data(); n = L.A.val.size() * 8; break;
        case 4:
            if (level != int32_t(h->h.lv.size()) - 1) return fail(MIFVM_E_ARG, "the inverse is on the coarsest level");
            src = h->h.cinv.data(); n = h->h.cinv.size() * 8; break;
        default: return fail(MIFVM_E_ARG, "unknown export id");
    }
    if (bytes != n) return fail(MIFVM_E_ARG, "size mismatch: expected " + std::to_string(n) + " bytes");
    if (n) std::memcpy(dst, src, n);
    return MIFVM_OK;
}

void mifvm_amg_host_destroy(mifvm_amg_host* h) { delete h; }

}  // extern "C"
