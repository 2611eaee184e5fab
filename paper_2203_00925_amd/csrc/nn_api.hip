// C ABI of the learned preconditioner (declared in include/mifvm_nn.h) and
// the flexible-CG phase of mifvm_poisson_solve with method LEARNED.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <random>
#include <vector>

#include "../../include/mifvm.h"
#include "../../include/mifvm_nn.h"
#include "api_util.h"
#include "fcg_monitor.h"
#include "nn.h"

static_assert(MIFVM_NN_PARAMS == mifvm::kNnParams, "parameter count of the ABI and the kernels");

struct mifvm_nn {
    mifvm::NnDev n;
    int64_t adam_steps = 0;
};

using namespace mifvm_api;

namespace mifvm {

size_t nn_layout(char* base, NnDev& n) {
    size_t off = 0;
    n.params = carve<float>(base, off, kNnParams);
    n.grad = carve<float>(base, off, kNnParams);
    n.adam_m = carve<float>(base, off, kNnParams);
    n.adam_v = carve<float>(base, off, kNnParams);
    n.pack = carve<NnPack>(base, off, 1);
    n.partial = carve<float>(base, off, size_t(kNnGridMax) * kNnParams);
    n.partial2 = carve<float>(base, off, size_t(kNnGradChunks) * kNnParams);
    n.loss = carve<double>(base, off, kNnLossRing);
    return (off + 255) & ~size_t(255);
}

namespace {
// the tiles of size T; false if a limit of the fused kernel is exceeded
bool build_tiles(const Mesh& m, int T, NnTiles& out) {
    const int64_t nc = m.nc;
    out = NnTiles{};
    out.tile_rows = T;
    out.ntiles = (nc + T - 1) / T;
    out.ext_off.assign(out.ntiles + 1, 0);
    out.ring.assign(4 * out.ntiles, 0);
    out.nb_off.assign(out.ntiles + 1, 0);
    out.cell.reserve(size_t(nc) * 4);
    out.nb.reserve(size_t(nc) * 12);
    std::vector<int64_t> stamp(nc, -1);
    std::vector<int32_t> loc(nc, 0), list, next;
    for (int64_t t = 0; t < out.ntiles; ++t) {
        list.clear();
        const int64_t c0 = t * T, c1 = std::min<int64_t>(nc, c0 + T);
        for (int64_t c = c0; c < c1; ++c) {
            stamp[c] = t;
            list.push_back(int32_t(c));
        }
        out.ring[4 * t] = int32_t(list.size());
        size_t begin = 0;
        for (int k = 1; k < 4; ++k) {
            const size_t end = list.size();
            next.clear();
            for (size_t idx = begin; idx < end; ++idx)
                for (int f = 0; f < 4; ++f) {
                    const int64_t j = m.c2n[f * nc + list[idx]];
                    if (j < nc && stamp[j] != t) {
                        stamp[j] = t;
                        next.push_back(int32_t(j));
                    }
                }
            std::sort(next.begin(), next.end());
            list.insert(list.end(), next.begin(), next.end());
            begin = end;
            out.ring[4 * t + k] = int32_t(list.size());
        }
        if (list.size() > 65535) return false;
        for (size_t e = 0; e < list.size(); ++e) loc[list[e]] = int32_t(e);
        out.ext_max = std::max(out.ext_max, int32_t(list.size()));
        out.r2_max = std::max(out.r2_max, out.ring[4 * t + 2]);
        out.cell.insert(out.cell.end(), list.begin(), list.end());
        out.ext_off[t + 1] = int64_t(out.cell.size());
        for (int e = 0; e < out.ring[4 * t + 2]; ++e)
            for (int f = 0; f < 4; ++f) {
                const int64_t j = m.c2n[f * nc + list[e]];
                out.nb.push_back(j < nc ? uint16_t(loc[j]) : uint16_t(0xFFFF));
            }
        out.nb_off[t + 1] = int64_t(out.nb.size() / 4);
    }
    return out.r2_max <= kNnFusedMaxGroups * kNnFusedWaves * 16 &&
           out.ext_max <= kNnFusedEntriesPerThread * 256 && nn_fused_lds(out) <= kNnFusedLdsMax;
}
}  // namespace

const NnTiles* nn_tiles(const Mesh& m) {
    if (m.nn_tiles) return m.nn_tiles.get();
    for (int T : {256, 192, 128, 64}) {
        auto t = std::make_shared<NnTiles>();
        if (build_tiles(m, T, *t)) {
            m.nn_tiles = t;
            return t.get();
        }
    }
    return nullptr;
}

size_t nn_state_layout(const Mesh& m, bool training, char* base, NnStateDev& a) {
    size_t off = 0;
    const int64_t nc = m.nc;
    a = NnStateDev{};
    a.nbr = carve<int4>(base, off, nc);
    a.h1 = carve<u32x4>(base, off, 4 * nc);
    a.h2 = carve<u32x4>(base, off, 4 * nc);
    a.r_old = carve<double>(base, off, nc);
    a.x_bak = carve<double>(base, off, nc);
    a.flag = carve<int32_t>(base, off, 1);
    if (training) {
        a.h3 = carve<u32x4>(base, off, 4 * nc);
        a.base = carve<float>(base, off, 32 * nc);
        a.dam0 = carve<float>(base, off, 32 * nc);
        a.dam1 = carve<float>(base, off, 32 * nc);
        a.kt_val = carve<double>(base, off, m.kmat.idx.size());
    }
    a.training = training;
    a.tiles = nn_tiles(m);
    if (a.tiles) {
        const NnTiles& t = *a.tiles;
        a.t_ext_off = carve<int64_t>(base, off, t.ext_off.size());
        a.t_ring = carve<int4>(base, off, size_t(t.ntiles));
        a.t_cell = carve<int32_t>(base, off, t.cell.size());
        a.t_nb_off = carve<int64_t>(base, off, t.nb_off.size());
        a.t_nb = carve<ushort4>(base, off, t.nb.size() / 4);
        a.t_partial = carve<double>(base, off, 2 * size_t(t.ntiles));
    }
    return (off + 255) & ~size_t(255);
}

}  // namespace mifvm

namespace {

std::vector<float> initial_params(uint64_t seed, double scale) {
    std::vector<float> p(kNnParams, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> N(0.0, 1.0);
    auto fill = [&](int at, int count, int fan_in) {
        const double sd = scale * std::sqrt(2.0 / fan_in);
        for (int k = 0; k < count; ++k) p[at + k] = float(sd * N(rng));
    };
    fill(kNnOffWe, 64, 2);
    for (int l = 0; l < kNnLayers; ++l) {
        fill(kNnOffLayer + l * kNnLayerSize + kNnW1, 32 * 64, 64);
        fill(kNnOffLayer + l * kNnLayerSize + kNnW2, 32 * 32, 32);
    }
    return p;
}

// upload a full parameter set, clear the Adam state, repack the operands
int put_params(mifvm_nn* nn, const float* p, hipStream_t hs) {
    for (int k = 0; k < kNnParams; ++k)
        if (!std::isfinite(p[k])) return fail(MIFVM_E_ARG, "non-finite parameter " + std::to_string(k));
    const NnDev& n = nn->n;
    HIPCHK(hipMemcpyAsync(n.params, p, kNnParams * sizeof(float), hipMemcpyHostToDevice, hs));
    HIPCHK(hipMemsetAsync(n.adam_m, 0, kNnParams * sizeof(float), hs));
    HIPCHK(hipMemsetAsync(n.adam_v, 0, kNnParams * sizeof(float), hs));
    HIPCHK(launch_nn_pack(n, hs));
    HIPCHK(hipStreamSynchronize(hs));                 // p may be freed by the caller
    nn->adam_steps = 0;
    return MIFVM_OK;
}

int need_attached(const State& s, bool training) {
    if (!s.nn || !s.nn_state) return fail(MIFVM_E_STATE, "no network attached to this state");
    if (training && !s.nn_state->training) return fail(MIFVM_E_STATE, "the network is attached without training buffers");
    // inference reads D^-1 only; training reads K
    if (training ? !s.assembled : !(s.assembled || s.consts_ready))
        return fail(MIFVM_E_STATE, "poisson system not assembled");
    return MIFVM_OK;
}

// values of K^T, once per assembly
int ensure_transpose(State& s, hipStream_t hs) {
    if (s.kt_ready) return MIFVM_OK;
    const NnStateDev& a = *s.nn_state;
    HIPCHK(hipMemsetAsync(a.flag, 0, sizeof(int32_t), hs));
    HIPCHK(launch_nn_transpose(s.d, a, hs));
    int32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, a.flag, sizeof(int32_t), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    if (flag) return fail(MIFVM_E_STATE, "the pattern of K is not symmetric: K^T cannot share it");
    s.kt_ready = true;
    return MIFVM_OK;
}

struct AdamCfg {
    int loss;
    bool apply;
    float lr, c1, c2, beta1, beta2, eps;
};

// one forward + backward on a sample; with apply, one Adam step
hipError_t train_step(State& s, const NnDev& n, const float* r32, double* loss_slot, const AdamCfg& c,
                      hipStream_t hs) {
    const Dev& d = s.d;
    const NnStateDev& a = *s.nn_state;
    hipError_t e = launch_nn_scale(d, nullptr, r32, hs);
    for (int l = 0; e == hipSuccess && l < kNnLayers; ++l) e = launch_nn_layer(d, n, a, l, nullptr, r32, d.z, true, false, hs);
    if (e == hipSuccess) e = launch_nn_backward(d, n, a, r32, c.loss, loss_slot, hs);
    if (e == hipSuccess)
        e = launch_nn_adam(n, nn_backward_grid(d.nc), c.apply ? 1 : 0, c.lr, c.c1, c.c2, c.beta1, c.beta2, c.eps, hs);
    return e;
}

// the network inside the flexible CG (z from d.r, dots with r, r_old): the
// fused forward when it is the state's chosen form, else layer by layer
hipError_t fcg_forward(State& s, hipStream_t q, bool timing) {
    const Dev& d = s.d;
    const NnStateDev& a = *s.nn_state;
    KernelTimer& tm = s.timer;
    if (a.tiles && a.fused) {
        auto fn = [&] { return launch_nn_fused(d, *s.nn, a, d.r, d.z, true, q); };
        return timing ? timed(tm, MIFVM_K_NN_FUSED, q, fn) : fn();
    }
    for (int l = 0; l < kNnLayers; ++l) {
        auto fn = [&] { return launch_nn_layer(d, *s.nn, a, l, d.r, nullptr, d.z, false, true, q); };
        hipError_t e = timing ? timed(tm, MIFVM_K_NN_LAYER1 + l, q, fn) : fn();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t enqueue_fcg_chunk(State& s, int n, hipStream_t q) {
    const Dev& d = s.d;
    for (int c = 0; c < n; ++c) {
        hipError_t e = s.mf ? launch_mf_cg_spmv(d, s.bc[1], q) : launch_cg_spmv(d, q);
        if (e == hipSuccess) e = launch_fcg_axpy(d, *s.nn_state, q);
        if (e == hipSuccess) e = fcg_forward(s, q, false);
        if (e == hipSuccess) e = launch_fcg_beta(d, *s.nn_state, q);
        if (e == hipSuccess) e = launch_cg_dir(d, q);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

namespace mifvm_api {

int learned_phase(State& s, double tol, int maxit, int chunk, int restart, int stall_window, int learned_maxit,
                  bool use_graph, hipStream_t hs, const std::function<int()>& pull, LearnedRun& out) {
    const Dev& d = s.d;
    const NnStateDev& a = *s.nn_state;
    KernelTimer& tm = s.timer;
    const int limit = learned_maxit > 0 ? std::min(learned_maxit, maxit) : maxit;
    const int window = stall_window > 0 ? stall_window : 200;
    out = LearnedRun{};
    auto setup = [&](bool fresh) -> int {
        HIPCHK(timed(tm, MIFVM_K_CG_SETUP, hs, [&]() -> hipError_t {
            if (s.mf) {                               // K x by the matrix-free product
                hipError_t e = launch_mf_apply(d, s.bc[1], d.x, d.tmp, hs);
                if (e != hipSuccess) return e;
            }
            return launch_fcg_setup(d, tol, limit, restart, fresh, hs, s.mf ? d.tmp : nullptr);
        }));
        HIPCHK(fcg_forward(s, hs, true));
        HIPCHK(timed(tm, MIFVM_K_FCG_VEC, hs, [&] { return launch_fcg_setup_tail(d, a, hs); }));
        return pull();
    };
    const int graph_key = chunk + (s.mf ? 1 << 20 : 0);
    if (use_graph && (s.fcg_exec == nullptr || s.fcg_exec_chunk != graph_key)) {
        HIPCHK(capture_graph(s, &s.fcg_exec, [&](hipStream_t q) { return enqueue_fcg_chunk(s, chunk, q); }));
        s.fcg_exec_chunk = graph_key;
    }
    auto run_chunk = [&]() -> int {
        if (use_graph) {
            HIPCHK(hipGraphLaunch(s.fcg_exec, hs));
            return MIFVM_OK;
        }
        for (int c = 0; c < chunk; ++c) {
            HIPCHK(timed(tm, MIFVM_K_CG_SPMV, hs,
                         [&] { return s.mf ? launch_mf_cg_spmv(d, s.bc[1], hs) : launch_cg_spmv(d, hs); }));
            HIPCHK(timed(tm, MIFVM_K_FCG_VEC, hs, [&] { return launch_fcg_axpy(d, a, hs); }));
            HIPCHK(fcg_forward(s, hs, true));
            HIPCHK(timed(tm, MIFVM_K_FCG_VEC, hs, [&] { return launch_fcg_beta(d, a, hs); }));
            HIPCHK(timed(tm, MIFVM_K_CG_DIR, hs, [&] { return launch_cg_dir(d, hs); }));
        }
        return MIFVM_OK;
    };
    auto fall_back = [&](bool restore) -> int {
        if (restore) HIPCHK(launch_fcg_backup(d, a, true, hs));
        out.fell_back = true;
        return MIFVM_OK;
    };
    HIPCHK(launch_fcg_backup(d, a, false, hs));
    FcgMonitor mon;
    mon.window = window;
    mon.limit_is_learned = limit < maxit;
    auto act = [&](FcgMonitor::Action x) -> int {
        switch (x) {
            case FcgMonitor::FALL_BACK_RESTORE: return fall_back(true);
            case FcgMonitor::FALL_BACK_KEEP: return fall_back(false);
            default: return MIFVM_OK;
        }
    };
    int rc = setup(true);
    if (rc) return rc;
    FcgMonitor::Action x = mon.open(hsc(s, 0, SC_TRUE_RR), hsc(s, 0, SC_RZ), hsc(s, 0, SC_RR));
    if (x != FcgMonitor::CONTINUE) return act(x);
    for (;;) {
        while (hsc(s, 0, SC_DONE) == 0.0) {
            if ((rc = run_chunk())) return rc;
            if ((rc = pull())) return rc;
            out.iterations = int(hsc(s, 0, SC_IT));
            x = mon.after_chunk(hsc(s, 0, SC_RR), hsc(s, 0, SC_RZ), hsc(s, 0, SC_BETA), hsc(s, 0, SC_IT));
            if (x != FcgMonitor::CONTINUE) return act(x);
            HIPCHK(launch_fcg_backup(d, a, false, hs));
        }
        // converged by the recurrence, at the limit, or a restart is due:
        // the true residual decides
        if ((rc = setup(false))) return rc;
        out.iterations = int(hsc(s, 0, SC_IT));
        x = mon.after_reopen(hsc(s, 0, SC_TRUE_RR), hsc(s, 0, SC_RZ), hsc(s, 0, SC_DONE));
        if (x != FcgMonitor::CONTINUE) return act(x);
        ++out.restarts;
    }
}

hipError_t nn_apply_vec(State& s, const double* in, double* out, hipStream_t q) {
    const Dev& d = s.d;
    const NnStateDev& a = *s.nn_state;
    hipError_t e = launch_nn_scale(d, in, nullptr, q);
    if (e == hipSuccess && a.tiles && a.fused) return launch_nn_fused(d, *s.nn, a, in, out, false, q);
    for (int l = 0; e == hipSuccess && l < kNnLayers; ++l)
        e = launch_nn_layer(d, *s.nn, a, l, in, nullptr, out, false, false, q);
    return e;
}

// captured chunks that launch the network (flexible CG; the multigrid cycle
// with the learned smoother) hold its buffers and form: dropped whenever
// those change
void drop_nn_graphs(State& s) {
    if (s.fcg_exec) (void)hipGraphExecDestroy(s.fcg_exec);
    s.fcg_exec = nullptr;
    if (s.amg_exec) (void)hipGraphExecDestroy(s.amg_exec);
    s.amg_exec = nullptr;
}

// Times one application of each form (the second of two, on the cell
// volumes as input; d.z is scratch here) and keeps the faster.  The forms
// give bitwise the same z, so the choice changes only the speed.
hipError_t choose_form(State& s, const NnDev& n, NnStateDev& a, hipStream_t q) {
    const Dev& d = s.d;
    hipEvent_t ev[3];
    for (auto& x : ev)
        if (hipError_t e = hipEventCreate(&x); e != hipSuccess) return e;
    auto run = [&](bool fused) {
        hipError_t e = launch_nn_scale(d, d.vol, nullptr, q);
        if (e == hipSuccess && fused) return launch_nn_fused(d, n, a, d.vol, d.z, false, q);
        for (int l = 0; e == hipSuccess && l < kNnLayers; ++l)
            e = launch_nn_layer(d, n, a, l, d.vol, nullptr, d.z, false, false, q);
        return e;
    };
    float ms[2] = {0.f, 0.f};
    hipError_t e = hipSuccess;
    for (int f = 0; f < 2 && e == hipSuccess; ++f) {
        e = run(f == 1);
        if (e == hipSuccess) e = hipEventRecord(ev[0], q);
        if (e == hipSuccess) e = run(f == 1);
        if (e == hipSuccess) e = hipEventRecord(ev[1], q);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[f], ev[0], ev[1]);
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return e;
    a.ms_layers = ms[0];
    a.ms_fused = ms[1];
    a.fused = ms[1] < ms[0];
    return hipSuccess;
}

}  // namespace mifvm_api

extern "C" {

size_t mifvm_nn_workspace_bytes(void) {
    NnDev probe{};
    return nn_layout(nullptr, probe);
}

int mifvm_nn_create(const mifvm_nn_opts* opts, void* d_ws, size_t ws_bytes, void* stream, mifvm_nn** out) {
    if (!out || !d_ws) return fail(MIFVM_E_ARG, "null argument");
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(MIFVM_E_WORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < mifvm_nn_workspace_bytes())
        return fail(MIFVM_E_WORKSPACE, "workspace too small: need " + std::to_string(mifvm_nn_workspace_bytes()));
    const double scale = opts && opts->init_scale > 0 ? opts->init_scale : 1.0;
    if (!std::isfinite(scale)) return fail(MIFVM_E_ARG, "bad init_scale");
    auto* nn = new (std::nothrow) mifvm_nn();
    if (!nn) return fail(MIFVM_E_ARG, "out of host memory");
    nn_layout(static_cast<char*>(d_ws), nn->n);
    const std::vector<float> p = initial_params(opts ? opts->seed : 0, scale);
    const int rc = put_params(nn, p.data(), S(stream));
    if (rc) {
        delete nn;
        return rc;
    }
    *out = nn;
    return MIFVM_OK;
}

void mifvm_nn_destroy(mifvm_nn* nn) { delete nn; }

int mifvm_nn_get_params(const mifvm_nn* nn, float* out, int64_t n, void* stream) {
    if (!nn || !out) return fail(MIFVM_E_ARG, "null argument");
    if (n != kNnParams) return fail(MIFVM_E_ARG, "need MIFVM_NN_PARAMS values");
    hipStream_t hs = S(stream);
    HIPCHK(hipMemcpyAsync(out, nn->n.params, kNnParams * sizeof(float), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    return MIFVM_OK;
}

int mifvm_nn_set_params(mifvm_nn* nn, const float* in, int64_t n, void* stream) {
    if (!nn || !in) return fail(MIFVM_E_ARG, "null argument");
    if (n != kNnParams) return fail(MIFVM_E_ARG, "need MIFVM_NN_PARAMS values");
    return put_params(nn, in, S(stream));
}

namespace {
constexpr char kTag[8] = {'M', 'I', 'F', 'V', 'M', 'N', 'N', '1'};
constexpr size_t kBlobBytes = 16 + sizeof(float) * size_t(kNnParams);
}  // namespace

int mifvm_nn_save(const mifvm_nn* nn, void* buf, size_t* bytes, void* stream) {
    if (!nn || !bytes) return fail(MIFVM_E_ARG, "null argument");
    if (!buf) {
        *bytes = kBlobBytes;
        return MIFVM_OK;
    }
    if (*bytes < kBlobBytes) return fail(MIFVM_E_ARG, "buffer too small: need " + std::to_string(kBlobBytes));
    std::vector<float> p(kNnParams);
    const int rc = mifvm_nn_get_params(nn, p.data(), kNnParams, stream);
    if (rc) return rc;
    char* o = static_cast<char*>(buf);
    const uint32_t version = 1, count = kNnParams;
    std::memcpy(o, kTag, 8);
    std::memcpy(o + 8, &version, 4);
    std::memcpy(o + 12, &count, 4);
    std::memcpy(o + 16, p.data(), sizeof(float) * p.size());
    *bytes = kBlobBytes;
    return MIFVM_OK;
}

int mifvm_nn_load(mifvm_nn* nn, const void* buf, size_t bytes, void* stream) {
    if (!nn || !buf) return fail(MIFVM_E_ARG, "null argument");
    if (bytes != kBlobBytes) return fail(MIFVM_E_ARG, "blob size " + std::to_string(bytes) + " != " + std::to_string(kBlobBytes));
    const char* b = static_cast<const char*>(buf);
    uint32_t version = 0, count = 0;
    std::memcpy(&version, b + 8, 4);
    std::memcpy(&count, b + 12, 4);
    if (std::memcmp(b, kTag, 8) != 0) return fail(MIFVM_E_ARG, "not a network blob (tag)");
    if (version != 1 || count != uint32_t(kNnParams)) return fail(MIFVM_E_ARG, "unsupported version or parameter count");
    std::vector<float> p(kNnParams);
    std::memcpy(p.data(), b + 16, sizeof(float) * p.size());
    return put_params(nn, p.data(), S(stream));
}

int mifvm_nn_attach_bytes(const mifvm_state* st, int32_t training, size_t* out) {
    if (!st || !out) return fail(MIFVM_E_ARG, "null argument");
    NnStateDev probe;
    *out = nn_state_layout(*st->s.mesh, training != 0, nullptr, probe);
    return MIFVM_OK;
}

int mifvm_nn_attach(mifvm_state* st, mifvm_nn* nn, int32_t training, void* d_ws, size_t ws_bytes, void* stream) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    if (!nn) {                                        // detach
        delete s.nn_state;
        s.nn_state = nullptr;
        s.nn = nullptr;
        s.nn_handle = nullptr;
        s.kt_ready = false;
        drop_nn_graphs(s);
        return MIFVM_OK;
    }
    if (!d_ws) return fail(MIFVM_E_ARG, "null workspace");
    if (s.d.nm != 1) return fail(MIFVM_E_ARG, "the learned preconditioner needs a single-mesh state");
    if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(MIFVM_E_WORKSPACE, "workspace not 256-byte aligned");
    NnStateDev probe;
    const size_t need = nn_state_layout(*s.mesh, training != 0, nullptr, probe);
    if (ws_bytes < need) return fail(MIFVM_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
    auto* a = new (std::nothrow) NnStateDev();
    if (!a) return fail(MIFVM_E_ARG, "out of host memory");
    nn_state_layout(*s.mesh, training != 0, static_cast<char*>(d_ws), *a);
    hipStream_t hs = S(stream);
    hipError_t e = launch_nn_neighbours(s.d, *a, hs);
    if (e == hipSuccess && a->tiles) {                // the fused forward's tiles
        const NnTiles& t = *a->tiles;
        e = hipMemcpyAsync(a->t_ext_off, t.ext_off.data(), t.ext_off.size() * 8, hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(a->t_ring, t.ring.data(), t.ring.size() * 4, hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(a->t_cell, t.cell.data(), t.cell.size() * 4, hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(a->t_nb_off, t.nb_off.data(), t.nb_off.size() * 8, hipMemcpyHostToDevice, hs);
        if (e == hipSuccess) e = hipMemcpyAsync(a->t_nb, t.nb.data(), t.nb.size() * 2, hipMemcpyHostToDevice, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
    }
    if (e == hipSuccess && a->tiles) e = setup_nn_fused(nn_fused_lds(*a->tiles));
    if (e == hipSuccess && a->tiles) e = choose_form(s, nn->n, *a, hs);
    if (e != hipSuccess) {
        delete a;
        return hip_fail(e, "attach");
    }
    delete s.nn_state;
    s.nn_state = a;
    s.nn = &nn->n;
    s.nn_handle = nn;
    s.kt_ready = false;
    drop_nn_graphs(s);
    return MIFVM_OK;
}

}  // extern "C"

namespace {
int nn_apply_impl(mifvm_state* st, const double* d_r, double* d_z, void* stream, bool layers) {
    if (!st || !d_r || !d_z) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    int rc = need_attached(s, false);
    if (rc) return rc;
    const Dev& d = s.d;
    const NnStateDev& a = *s.nn_state;
    hipStream_t hs = S(stream);
    HIPCHK(launch_to_internal(d.cell_perm, d.nc, d.nc, d.nc, 1, d_r, d.r, hs));
    HIPCHK(launch_nn_scale(d, d.r, nullptr, hs));
    if (a.tiles && a.fused && !layers) {
        HIPCHK(timed(s.timer, MIFVM_K_NN_FUSED, hs, [&] { return launch_nn_fused(d, *s.nn, a, d.r, d.z, false, hs); }));
    } else {
        for (int l = 0; l < kNnLayers; ++l)
            HIPCHK(timed(s.timer, MIFVM_K_NN_LAYER1 + l, hs,
                         [&] { return launch_nn_layer(d, *s.nn, a, l, d.r, nullptr, d.z, false, false, hs); }));
    }
    HIPCHK(launch_to_user(d.cell_perm, d.nc, d.nc, d.nc, 1, d.z, d_z, hs));
    return MIFVM_OK;
}
}  // namespace

extern "C" {

int mifvm_nn_apply(mifvm_state* st, const double* d_r, double* d_z, void* stream) {
    return nn_apply_impl(st, d_r, d_z, stream, false);
}

int mifvm_nn_apply_layers(mifvm_state* st, const double* d_r, double* d_z, void* stream) {
    return nn_apply_impl(st, d_r, d_z, stream, true);
}

int mifvm_nn_form(mifvm_state* st, int32_t form, int32_t* chosen, float* ms_layers, float* ms_fused) {
    if (!st) return fail(MIFVM_E_ARG, "null state");
    State& s = st->s;
    int rc = need_attached(s, false);
    if (rc) return rc;
    NnStateDev& a = *s.nn_state;
    if (form == MIFVM_NN_FORM_FUSED && !a.tiles)
        return fail(MIFVM_E_STATE, "the mesh's tiles exceed the fused forward's limits");
    if (form == MIFVM_NN_FORM_AUTO) a.fused = a.tiles && a.ms_fused < a.ms_layers;
    else if (form == MIFVM_NN_FORM_LAYERS) a.fused = false;
    else if (form == MIFVM_NN_FORM_FUSED) a.fused = true;
    else if (form != -1) return fail(MIFVM_E_ARG, "unknown network form");
    drop_nn_graphs(s);                                          // captured chunks hold the old form
    if (chosen) *chosen = a.fused ? MIFVM_NN_FORM_FUSED : MIFVM_NN_FORM_LAYERS;
    if (ms_layers) *ms_layers = a.ms_layers;
    if (ms_fused) *ms_fused = a.ms_fused;
    return MIFVM_OK;
}

int mifvm_nn_sample(mifvm_state* st, float* d_out, double* rms, void* stream) {
    if (!st || !d_out || !rms) return fail(MIFVM_E_ARG, "null argument");
    State& s = st->s;
    if (!s.assembled) return fail(MIFVM_E_STATE, "poisson system not assembled");
    if (!s.b_ready) return fail(MIFVM_E_STATE, "no right-hand side yet (solve or mifvm_poisson_rhs first)");
    if (s.d.nm != 1) return fail(MIFVM_E_ARG, "samples are taken from single-mesh states");
    hipStream_t hs = S(stream);
    HIPCHK(launch_nn_sample(s.d, d_out, hs));
    const int rc = pull_scalars(s, hs);
    if (rc) return rc;
    *rms = std::sqrt(hsc(s, 0, SC_NN_RR) / double(s.d.nc));
    return MIFVM_OK;
}

int mifvm_nn_loss_grad(mifvm_state* st, const float* d_sample, int32_t loss_kind, double* loss, float* grad,
                       void* stream) {
    if (!st || !d_sample || !loss || !grad) return fail(MIFVM_E_ARG, "null argument");
    if (loss_kind != MIFVM_NN_LOSS_RESIDUAL && loss_kind != MIFVM_NN_LOSS_ENERGY) return fail(MIFVM_E_ARG, "unknown loss");
    State& s = st->s;
    int rc = need_attached(s, true);
    if (rc) return rc;
    hipStream_t hs = S(stream);
    if ((rc = ensure_transpose(s, hs))) return rc;
    const NnDev& n = *s.nn;
    const AdamCfg none{loss_kind, false, 0.f, 1.f, 1.f, 0.9f, 0.999f, 1e-8f};
    HIPCHK(train_step(s, n, d_sample, n.loss, none, hs));
    HIPCHK(hipMemcpyAsync(loss, n.loss, sizeof(double), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipMemcpyAsync(grad, n.grad, kNnParams * sizeof(float), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    return MIFVM_OK;
}

int mifvm_nn_train(mifvm_nn* nn, mifvm_state* const* states, int32_t n_states, const float* const* d_samples,
                   const int32_t* state_of_sample, int32_t n_samples, const mifvm_train_opts* opts,
                   mifvm_train_info* info, double* epoch_loss, void* stream) {
    if (!nn || !states || !d_samples || !state_of_sample || !opts) return fail(MIFVM_E_ARG, "null argument");
    if (n_states <= 0 || n_samples <= 0 || opts->epochs <= 0) return fail(MIFVM_E_ARG, "nothing to train on");
    if (!(opts->lr > 0) || !(opts->lr_min >= 0) || opts->lr_min > opts->lr) return fail(MIFVM_E_ARG, "bad lr / lr_min");
    const float beta1 = opts->beta1 > 0 ? float(opts->beta1) : 0.9f;
    const float beta2 = opts->beta2 > 0 ? float(opts->beta2) : 0.999f;
    const float eps = opts->eps > 0 ? float(opts->eps) : 1e-8f;
    if (!(beta1 < 1.f) || !(beta2 < 1.f)) return fail(MIFVM_E_ARG, "beta1, beta2 must be < 1");
    if (opts->loss != MIFVM_NN_LOSS_RESIDUAL && opts->loss != MIFVM_NN_LOSS_ENERGY) return fail(MIFVM_E_ARG, "unknown loss");
    hipStream_t hs = S(stream);
    for (int k = 0; k < n_states; ++k) {
        if (!states[k]) return fail(MIFVM_E_ARG, "null state");
        State& s = states[k]->s;
        int rc = need_attached(s, true);
        if (rc) return rc;
        if (s.nn_handle != nn) return fail(MIFVM_E_STATE, "a state is attached to another network");
        if ((rc = ensure_transpose(s, hs))) return rc;
    }
    for (int k = 0; k < n_samples; ++k) {
        if (state_of_sample[k] < 0 || state_of_sample[k] >= n_states) return fail(MIFVM_E_ARG, "state_of_sample out of range");
        if (!d_samples[k]) return fail(MIFVM_E_ARG, "null sample");
    }
    const NnDev& n = nn->n;
    auto t0 = std::chrono::steady_clock::now();
    std::mt19937_64 rng(opts->seed);
    std::vector<int32_t> order(n_samples);
    for (int k = 0; k < n_samples; ++k) order[k] = k;
    const int64_t total = int64_t(opts->epochs) * n_samples;
    int64_t step = 0;
    std::vector<double> losses;
    double first = 0.0, last = 0.0;
    for (int ep = 0; ep < opts->epochs; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        double sum = 0.0;
        for (int k0 = 0; k0 < n_samples; k0 += kNnLossRing) {
            const int k1 = std::min<int>(n_samples, k0 + kNnLossRing);
            for (int k = k0; k < k1; ++k) {
                const int idx = order[k];
                State& s = states[state_of_sample[idx]]->s;
                const double frac = double(step) / double(total);
                const float lr = float(opts->lr_min + 0.5 * (opts->lr - opts->lr_min) * (1.0 + std::cos(3.14159265358979323846 * frac)));
                ++nn->adam_steps;
                const double t = double(nn->adam_steps);
                const AdamCfg c{opts->loss, true, lr, float(1.0 / (1.0 - std::pow(double(beta1), t))),
                                float(1.0 / std::sqrt(1.0 - std::pow(double(beta2), t))), beta1, beta2, eps};
                HIPCHK(timed(s.timer, MIFVM_K_NN_TRAIN, hs,
                             [&] { return train_step(s, n, d_samples[idx], n.loss + (k - k0), c, hs); }));
                ++step;
            }
            losses.resize(k1 - k0);
            HIPCHK(hipMemcpyAsync(losses.data(), n.loss, losses.size() * sizeof(double), hipMemcpyDeviceToHost, hs));
            HIPCHK(hipStreamSynchronize(hs));
            for (double v : losses) sum += v;
        }
        for (int k = 0; k < n_states; ++k) HIPCHK(timer_flush(states[k]->s.timer));
        const double mean = sum / n_samples;
        if (epoch_loss) epoch_loss[ep] = mean;
        if (ep == 0) first = mean;
        last = mean;
    }
    if (info) {
        info->steps = step;
        info->loss_first = first;
        info->loss_last = last;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return MIFVM_OK;
}

}  // extern "C"
