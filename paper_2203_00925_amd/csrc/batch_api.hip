// C ABI of the batched form: the persistent solve of every mesh of a
// multi-mesh state, the captured run of steps and solves, and the schedule
// autotuner (item size, grid, queue policy) with a JSON cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mifvm.h"
#include "api_util.h"
#include "batch.h"
#include "state.h"

using namespace mifvm;
using namespace mifvm_api;

struct mifvm_batch {
    mifvm_state* st = nullptr;
    BatchDev b{};
    std::vector<BatchRange> range;
    std::vector<int64_t> cells;
    int32_t* d_scan = nullptr;                // device scan lists [8][nm]
    int grid = 0, item_rows = 0, policy = 0, vb = 8, chunk = 32;
    hipGraphExec_t exec = nullptr;            // captured run
    int exec_steps = 0, exec_every = 0, exec_maxit = 0, exec_restart = 0;
    double exec_tol = 0.0;
    int64_t exec_gen = -1;
};

namespace {

constexpr int kDefaultItemRows = 4096, kDefaultGrid = 1024, kDefaultPolicy = BQ_XCD;
constexpr long long kSpinLimit = 1ll << 20;

template <class T>
T* carve_b(char* base, size_t& off, size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
}

int64_t pstride_of(int64_t cells) { return (cells + kBatchMinItemRows - 1) / kBatchMinItemRows; }

// mesh order per XCD for a queue policy (meshes by cell count, largest first)
std::vector<int32_t> scan_lists(const std::vector<int64_t>& cells, int policy) {
    const int nm = int(cells.size());
    std::vector<int32_t> desc(nm);
    std::iota(desc.begin(), desc.end(), 0);
    std::stable_sort(desc.begin(), desc.end(), [&](int a, int b) { return cells[a] > cells[b]; });
    std::vector<int32_t> out(size_t(8) * nm);
    if (policy == BQ_LARGEST) {
        for (int x = 0; x < 8; ++x) std::copy(desc.begin(), desc.end(), out.begin() + size_t(x) * nm);
    } else if (policy == BQ_ROTATE) {
        for (int x = 0; x < 8; ++x)
            for (int k = 0; k < nm; ++k) out[size_t(x) * nm + k] = desc[(k + x * nm / 8) % nm];
    } else {
        // each mesh to the XCD with the least load so far (largest first);
        // an XCD takes its own meshes first, then the others
        std::vector<int64_t> load(8, 0);
        std::vector<int> home(nm, 0);
        for (int m : desc) {
            const int x = int(std::min_element(load.begin(), load.end()) - load.begin());
            home[m] = x;
            load[x] += cells[m];
        }
        for (int x = 0; x < 8; ++x) {
            size_t k = size_t(x) * nm;
            for (int m : desc)
                if (home[m] == x) out[k++] = m;
            for (int m : desc)
                if (home[m] != x) out[k++] = m;
        }
    }
    return out;
}

size_t layout_b(const Dev& d, const std::vector<int64_t>& cells, char* base, BatchDev& b) {
    const int nm = int(cells.size());
    int64_t ptot = 0;
    for (int64_t c : cells) ptot += 3 * pstride_of(c);
    size_t off = 0;
    b.nm = nm;
    b.range = carve_b<BatchRange>(base, off, nm);
    b.q = carve_b<unsigned long long>(base, off, nm);
    b.done = carve_b<unsigned int>(base, off, nm);
    b.fresh = carve_b<int32_t>(base, off, nm);
    b.poff = carve_b<int64_t>(base, off, nm);
    b.pstride = carve_b<int64_t>(base, off, nm);
    b.partial = carve_b<double>(base, off, size_t(ptot));
    b.scan = carve_b<int32_t>(base, off, size_t(8) * nm);
    b.glob = carve_b<unsigned int>(base, off, BG_COUNT);
    b.rel_max = carve_b<double>(base, off, nm);
    b.it_total = carve_b<int64_t>(base, off, nm);
    return (off + 255) & ~size_t(255);
}

// contiguous ranges of each mesh: cells, vertices (numbered by their lowest
// cell), interior faces (sorted by their lower cell), boundary faces (by
// their cell); checks that no vertex list reaches into another mesh
int mesh_ranges(const Mesh& m, std::vector<BatchRange>& out) {
    const int nm = int(m.mesh_start.size()) - 1;
    out.assign(nm, BatchRange{});
    auto vmin = [&](int64_t v) { return int64_t(m.nidx[m.nptr[v]]); };
    auto flo = [&](int64_t f) { return int64_t(std::min(m.fL[f], m.fR[f])); };
    for (int k = 0; k < nm; ++k) {
        const int64_t c0 = m.mesh_start[k], c1 = m.mesh_start[k + 1];
        auto first_v = [&](int64_t c) {
            int64_t lo = 0, hi = m.nv;
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                if (vmin(mid) < c) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        };
        auto first_fi = [&](int64_t c) {
            int64_t lo = 0, hi = m.nfi;
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                if (flo(mid) < c) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        };
        auto first_fb = [&](int64_t c) {
            int64_t lo = m.nfi, hi = m.nf;
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                if (m.fL[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        };
        BatchRange& r = out[k];
        r.c0 = c0;
        r.c1 = c1;
        r.v0 = first_v(c0);
        r.v1 = first_v(c1);
        r.fi0 = first_fi(c0);
        r.fi1 = first_fi(c1);
        r.fb0 = first_fb(c0);
        r.fb1 = first_fb(c1);
        for (int64_t v = r.v0; v < r.v1; ++v)
            for (int64_t e = m.nptr[v]; e < m.nptr[v + 1]; ++e) {
                const int64_t c = m.nidx[e] < m.nc ? m.nidx[e] : m.gowner[m.nidx[e] - m.nc];
                if (c < c0 || c >= c1) return fail(MIFVM_E_ARG, "meshes of a batch share a vertex");
            }
        for (int64_t f = r.fi0; f < r.fi1; ++f)
            if (std::max(m.fL[f], m.fR[f]) >= c1) return fail(MIFVM_E_ARG, "a face joins two meshes of the batch");
    }
    return MIFVM_OK;
}

int upload_schedule(mifvm_batch* h, hipStream_t hs) {
    const std::vector<int32_t> scan = scan_lists(h->cells, h->policy);
    HIPCHK(hipMemcpyAsync(h->d_scan, scan.data(), scan.size() * sizeof(int32_t), hipMemcpyHostToDevice, hs));
    HIPCHK(hipStreamSynchronize(hs));          // scan is freed at return
    h->b.item_rows = h->item_rows;
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    h->exec = nullptr;
    return MIFVM_OK;
}

int check_schedule(int item_rows, int grid, int policy, int vb, int chunk) {
    if (item_rows < kBatchMinItemRows || item_rows % kBatchBlock != 0 || item_rows > (1 << 20))
        return fail(MIFVM_E_ARG, "item_rows must be a multiple of 256 in [256, 2^20]");
    if (grid < 1 || grid > 65536) return fail(MIFVM_E_ARG, "grid must be in [1, 65536]");
    if (policy < BQ_ROTATE || policy > BQ_LAUNCHES) return fail(MIFVM_E_ARG, "unknown queue policy");
    if (vb != 8 && vb != 24) return fail(MIFVM_E_ARG, "vertex_batch must be 8 or 24");
    if (chunk < 1 || chunk > 4096) return fail(MIFVM_E_ARG, "chunk must be in [1, 4096]");
    return MIFVM_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// the solve's device work on q (no host interaction)
hipError_t enqueue_solve(const mifvm_batch* h, double tol, int maxit, int restart, bool zero_run, hipStream_t q) {
    const State& s = h->st->s;
    hipError_t e = launch_rhs(s.d, s.d.u, q);                  // b = -mu u + c
    if (e == hipSuccess) e = launch_batch_init(s.d, h->b, maxit, restart, zero_run, q);
    if (e == hipSuccess) e = launch_batch_solve(s.d, h->b, h->grid, h->vb, tol, q);
    return e;
}

// LAUNCHES: the state's per-launch matrix-free CG (b = -mu U + c from the
// current U); run totals added into it / rel
int solve_launches(mifvm_batch* h, double tol, int maxit, int restart, hipStream_t hs, std::vector<int64_t>& it,
                   std::vector<double>& rel) {
    mifvm_solve_opts o{};
    o.tol = tol;
    o.maxit = maxit;
    o.chunk = h->chunk;
    o.restart = restart;
    o.method = MIFVM_SOLVE_PLAIN;
    o.graph = 1;
    o.matrix_free = 1;
    mifvm_solve_info si{};
    const int rc = mifvm_poisson_solve(h->st, nullptr, &o, &si, hs);
    if (rc < 0) return rc;
    const State& s = h->st->s;
    for (int m = 0; m < h->b.nm; ++m) {
        it[m] += s.last_iters[m];
        rel[m] = std::fmax(rel[m], s.last_rel[m]);
    }
    return MIFVM_OK;
}

// the outcome of LAUNCHES solves, in the form collect() reports
int report_launches(mifvm_batch* h, const std::vector<int64_t>& it, const std::vector<double>& rel,
                    mifvm_batch_info* info, double t0_ms, int solves) {
    const State& s = h->st->s;
    mifvm_batch_info out{};
    bool all = true;
    for (int m = 0; m < h->b.nm; ++m) {
        out.iterations_max = std::max<int64_t>(out.iterations_max, it[m]);
        out.iterations_sum += it[m];
        out.rel_residual_max = std::fmax(out.rel_residual_max, rel[m]);
        all = all && hsc(s, m, SC_DONE) == 1.0;
    }
    out.solves = solves;
    out.iterations_mean = h->b.nm > 0 ? double(out.iterations_sum) / h->b.nm : 0.0;
    out.ms = now_ms() - t0_ms;
    if (info) *info = out;
    return all ? MIFVM_OK : MIFVM_NOT_CONVERGED;
}

int solve_opts(const mifvm_batch_solve_opts* o, double& tol, int& maxit, int& restart, int& every) {
    tol = o && o->tol > 0 ? o->tol : 1e-10;
    maxit = o && o->maxit > 0 ? o->maxit : 20000;
    restart = o ? o->restart : 500;
    every = o && o->solve_every > 0 ? o->solve_every : 1;
    if (!(tol > 0) || restart < 0) return fail(MIFVM_E_ARG, "bad tol or restart");
    return MIFVM_OK;
}

// per-mesh outcome after the device work: scalars, the run accumulators,
// the abort flag
int collect(mifvm_batch* h, hipStream_t hs, mifvm_batch_info* info, double t0_ms, int solves) {
    State& s = h->st->s;
    const int nm = h->b.nm;
    std::vector<int64_t> it(nm);
    std::vector<double> rel(nm);
    unsigned int glob[BG_COUNT];
    HIPCHK(hipMemcpyAsync(it.data(), h->b.it_total, nm * sizeof(int64_t), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipMemcpyAsync(rel.data(), h->b.rel_max, nm * sizeof(double), hipMemcpyDeviceToHost, hs));
    HIPCHK(hipMemcpyAsync(glob, h->b.glob, sizeof(glob), hipMemcpyDeviceToHost, hs));
    int rc = pull_scalars(s, hs);
    if (rc) return rc;
    const double ms = now_ms() - t0_ms;
    if (glob[BG_ABORT] != 0u)
        return fail(MIFVM_E_STATE, "persistent batch solve stopped: no progress within the spin limit");
    s.last_iters.assign(nm, 0);
    s.last_rel.assign(nm, 0.0);
    bool all = true;
    mifvm_batch_info out{};
    for (int m = 0; m < nm; ++m) {
        s.last_iters[m] = int(hsc(s, m, SC_IT));
        const double bb = hsc(s, m, SC_BB);
        s.last_rel[m] = bb > 0 ? std::sqrt(hsc(s, m, SC_TRUE_RR) / bb) : 0.0;
        all = all && hsc(s, m, SC_DONE) == 1.0;
        out.iterations_max = std::max<int64_t>(out.iterations_max, it[m]);
        out.iterations_sum += it[m];
        out.rel_residual_max = std::fmax(out.rel_residual_max, rel[m]);
    }
    out.solves = solves;
    out.iterations_mean = nm > 0 ? double(out.iterations_sum) / nm : 0.0;
    out.ms = ms;
    if (info) *info = out;
    return all ? MIFVM_OK : MIFVM_NOT_CONVERGED;
}

}  // namespace

extern "C" {

int mifvm_batch_bytes(const mifvm_state* st, size_t* out) {
    if (!st || !out) return fail(MIFVM_E_ARG, "null argument");
    const Mesh& m = *st->s.mesh;
    std::vector<int64_t> cells(m.mesh_start.size() - 1);
    for (size_t k = 0; k < cells.size(); ++k) cells[k] = m.mesh_start[k + 1] - m.mesh_start[k];
    BatchDev probe{};
    *out = layout_b(st->s.d, cells, nullptr, probe);
    return MIFVM_OK;
}

int mifvm_batch_create(mifvm_state* st, const mifvm_batch_opts* opts, void* d_ws, size_t ws_bytes, void* stream,
                       mifvm_batch** out) {
    if (!st || !d_ws || !out) return fail(MIFVM_E_ARG, "null argument");
    *out = nullptr;
    State& s = st->s;
    if (s.fp32) return fail(MIFVM_E_STATE, "the batched solve runs on FP64 states");
    if (s.d.nm > kBatchMaxMeshes) return fail(MIFVM_E_ARG, "at most 4096 meshes in a batch");
    if (reinterpret_cast<uintptr_t>(d_ws) & 255) return fail(MIFVM_E_WORKSPACE, "workspace not 256-byte aligned");
    const int item_rows = opts && opts->item_rows > 0 ? opts->item_rows : kDefaultItemRows;
    const int grid = opts && opts->grid > 0 ? opts->grid : kDefaultGrid;
    const int policy = opts && opts->policy >= 0 ? opts->policy : kDefaultPolicy;
    const int vb = opts && opts->vertex_batch > 0 ? opts->vertex_batch : 8;
    const int chunk = opts && opts->chunk > 0 ? opts->chunk : 32;
    int rc = check_schedule(item_rows, grid, policy, vb, chunk);
    if (rc) return rc;
    auto* h = new (std::nothrow) mifvm_batch();
    if (!h) return fail(MIFVM_E_ARG, "out of host memory");
    h->st = st;
    const Mesh& m = *s.mesh;
    if ((rc = mesh_ranges(m, h->range))) {
        delete h;
        return rc;
    }
    h->cells.resize(h->range.size());
    for (size_t k = 0; k < h->range.size(); ++k) h->cells[k] = h->range[k].c1 - h->range[k].c0;
    BatchDev probe{};
    const size_t need = layout_b(s.d, h->cells, nullptr, probe);
    if (ws_bytes < need) {
        delete h;
        return fail(MIFVM_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
    }
    layout_b(s.d, h->cells, static_cast<char*>(d_ws), h->b);
    h->d_scan = const_cast<int32_t*>(h->b.scan);
    h->b.spin_limit = opts && opts->spin_limit > 0 ? opts->spin_limit : kSpinLimit;
    h->item_rows = item_rows;
    h->grid = grid;
    h->policy = policy;
    h->vb = vb;
    h->chunk = chunk;
    hipStream_t hs = S(stream);
    std::vector<int64_t> poff(h->cells.size()), pstride(h->cells.size());
    int64_t at = 0;
    for (size_t k = 0; k < h->cells.size(); ++k) {
        pstride[k] = pstride_of(h->cells[k]);
        poff[k] = at;
        at += 3 * pstride[k];
    }
    auto fail_hip = [&](hipError_t e, const char* what) {
        delete h;
        return hip_fail(e, what);
    };
    hipError_t e = hipMemcpyAsync(const_cast<BatchRange*>(h->b.range), h->range.data(),
                                  h->range.size() * sizeof(BatchRange), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<int64_t*>(h->b.poff), poff.data(), poff.size() * 8, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<int64_t*>(h->b.pstride), pstride.data(), pstride.size() * 8,
                           hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);     // host vectors are freed at return
    if (e != hipSuccess) return fail_hip(e, "batch upload");
    if ((rc = upload_schedule(h, hs))) {
        delete h;
        return rc;
    }
    *out = h;
    return MIFVM_OK;
}

void mifvm_batch_destroy(mifvm_batch* h) {
    if (!h) return;
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    delete h;
}

int mifvm_batch_set_schedule(mifvm_batch* h, const mifvm_batch_opts* opts, void* stream) {
    if (!h || !opts) return fail(MIFVM_E_ARG, "null argument");
    const int item_rows = opts->item_rows > 0 ? opts->item_rows : h->item_rows;
    const int grid = opts->grid > 0 ? opts->grid : h->grid;
    const int policy = opts->policy >= 0 ? opts->policy : h->policy;
    const int vb = opts->vertex_batch > 0 ? opts->vertex_batch : h->vb;
    const int chunk = opts->chunk > 0 ? opts->chunk : h->chunk;
    int rc = check_schedule(item_rows, grid, policy, vb, chunk);
    if (rc) return rc;
    h->item_rows = item_rows;
    h->grid = grid;
    h->policy = policy;
    h->vb = vb;
    h->chunk = chunk;
    if (opts->spin_limit > 0) h->b.spin_limit = opts->spin_limit;
    return upload_schedule(h, S(stream));
}

int mifvm_batch_get_schedule(const mifvm_batch* h, mifvm_batch_opts* out) {
    if (!h || !out) return fail(MIFVM_E_ARG, "null argument");
    *out = mifvm_batch_opts{};
    out->item_rows = h->item_rows;
    out->grid = h->grid;
    out->policy = h->policy;
    out->spin_limit = int32_t(h->b.spin_limit);
    out->vertex_batch = h->vb;
    out->chunk = h->chunk;
    return MIFVM_OK;
}

int mifvm_batch_solve(mifvm_batch* h, const mifvm_batch_solve_opts* opts, mifvm_batch_info* info, void* stream) {
    if (!h) return fail(MIFVM_E_ARG, "null batch");
    double tol;
    int maxit, restart, every;
    int rc = solve_opts(opts, tol, maxit, restart, every);
    if (rc) return rc;
    State& s = h->st->s;
    hipStream_t hs = S(stream);
    const double t0 = now_ms();
    if ((rc = ensure_consts(s, hs))) return rc;
    if (h->policy == BQ_LAUNCHES) {
        std::vector<int64_t> it(h->b.nm, 0);
        std::vector<double> rel(h->b.nm, 0.0);
        if ((rc = solve_launches(h, tol, maxit, restart, hs, it, rel))) return rc;
        return report_launches(h, it, rel, info, t0, 1);
    }
    HIPCHK(enqueue_solve(h, tol, maxit, restart, true, hs));
    s.b_ready = true;
    return collect(h, hs, info, t0, 1);
}

int mifvm_batch_run(mifvm_batch* h, int32_t n_steps, const mifvm_batch_solve_opts* opts, mifvm_batch_info* info,
                    void* stream) {
    if (!h) return fail(MIFVM_E_ARG, "null batch");
    if (n_steps < 1) return fail(MIFVM_E_ARG, "n_steps must be >= 1");
    double tol;
    int maxit, restart, every;
    int rc = solve_opts(opts, tol, maxit, restart, every);
    if (rc) return rc;
    State& s = h->st->s;
    if (!(s.cfl > 0)) return fail(MIFVM_E_STATE, "the run takes each mesh's CFL step: call mifvm_cfl_dt first");
    hipStream_t hs = S(stream);
    const double t0 = now_ms();
    if ((rc = ensure_consts(s, hs))) return rc;
    if (h->policy == BQ_LAUNCHES) {             // a step graph and the chunked solve per step
        std::vector<int64_t> it(h->b.nm, 0);
        std::vector<double> rel(h->b.nm, 0.0);
        int solves = 0;
        for (int k = 0; k < n_steps; ++k) {
            if ((rc = mifvm_step_graph(h->st, 1, 0.0, stream))) return rc;
            if ((k + 1) % every == 0) {
                if ((rc = solve_launches(h, tol, maxit, restart, hs, it, rel))) return rc;
                ++solves;
            }
        }
        return report_launches(h, it, rel, info, t0, solves);
    }
    if (!h->exec || h->exec_steps != n_steps || h->exec_every != every || h->exec_tol != tol ||
        h->exec_maxit != maxit || h->exec_restart != restart || h->exec_gen != s.graph_gen) {
        HIPCHK(capture_graph(s, &h->exec, [&](hipStream_t q) -> hipError_t {
            bool first = true;
            for (int k = 0; k < n_steps; ++k) {
                hipError_t e = enqueue_steps(s, 1, 0.0, q);
                if (e != hipSuccess) return e;
                if ((k + 1) % every == 0) {
                    if ((e = enqueue_solve(h, tol, maxit, restart, first, q)) != hipSuccess) return e;
                    first = false;
                }
            }
            return hipSuccess;
        }));
        h->exec_steps = n_steps;
        h->exec_every = every;
        h->exec_tol = tol;
        h->exec_maxit = maxit;
        h->exec_restart = restart;
        h->exec_gen = s.graph_gen;
    }
    HIPCHK(hipGraphLaunch(h->exec, hs));
    s.b_ready = true;
    return collect(h, hs, info, t0, n_steps / every);
}

}  // extern "C"

namespace {

using TuneEntry = std::array<int, 5>;       // item_rows, grid, policy, vertex_batch, chunk

std::map<std::string, TuneEntry> read_batch_cache(const char* path) {
    std::map<std::string, TuneEntry> out;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        char key[256];
        TuneEntry e{};
        if (std::sscanf(line.c_str(),
                        " \"%255[^\"]\": {\"item_rows\": %d, \"grid\": %d, \"policy\": %d, \"vertex_batch\": %d, "
                        "\"chunk\": %d}",
                        key, &e[0], &e[1], &e[2], &e[3], &e[4]) == 6)
            out[key] = e;
    }
    return out;
}

void write_batch_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
    std::ofstream o(path);
    o << "{\n";
    size_t k = 0;
    for (auto& kv : m)
        o << "  \"" << kv.first << "\": {\"item_rows\": " << kv.second[0] << ", \"grid\": " << kv.second[1]
          << ", \"policy\": " << kv.second[2] << ", \"vertex_batch\": " << kv.second[3]
          << ", \"chunk\": " << kv.second[4] << "}" << (++k < m.size() ? "," : "") << "\n";
    o << "}\n";
}

}  // namespace

extern "C" int mifvm_batch_autotune(mifvm_batch* h, const char* cache_path, int32_t iterations,
                                    mifvm_batch_tune_info* out, void* stream) {
    if (!h) return fail(MIFVM_E_ARG, "null batch");
    State& s = h->st->s;
    const Dev& d = s.d;
    hipStream_t hs = S(stream);
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= d.nc) ++lg;
    const std::string key = "gfx950/batch/" + std::to_string(d.nm) + "/" + std::to_string(lg);
    mifvm_batch_tune_info info{};
    std::map<std::string, TuneEntry> cache;
    auto apply = [&](const TuneEntry& e) -> int {
        mifvm_batch_opts o{};
        o.item_rows = e[0];
        o.grid = e[1];
        o.policy = e[2];
        o.vertex_batch = e[3];
        o.chunk = e[4];
        return mifvm_batch_set_schedule(h, &o, stream);
    };
    if (cache_path) {
        cache = read_batch_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            int rc = apply(it->second);
            if (rc) return rc;
            info.item_rows = h->item_rows;
            info.grid = h->grid;
            info.policy = h->policy;
            info.vertex_batch = h->vb;
            info.chunk = h->chunk;
            info.from_cache = 1;
            if (out) *out = info;
            return MIFVM_OK;
        }
    }
    const int iters = iterations > 0 ? iterations : 24;
    int rc = ensure_consts(s, hs);
    if (rc) return rc;
    // every trial runs `iters` iterations of every mesh from the current P,
    // which is restored afterwards (kept in the scratch array's last third:
    // the per-launch solve's true residual uses its first)
    double* saved_x = d.tmp + 2 * (d.nc + d.nb);
    HIPCHK(hipMemcpyAsync(saved_x, d.x, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
    auto trial = [&](const TuneEntry& e, double* ms) -> int {
        int r = apply(e);
        if (r) return r;
        HIPCHK(hipMemcpyAsync(d.x, saved_x, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
        HIPCHK(hipStreamSynchronize(hs));
        const double t0 = now_ms();
        if (h->policy == BQ_LAUNCHES) {
            std::vector<int64_t> it(h->b.nm, 0);
            std::vector<double> rel(h->b.nm, 0.0);
            if ((r = solve_launches(h, 1e-300, iters, 0, hs, it, rel))) return r;
        } else {
            HIPCHK(enqueue_solve(h, 1e-300, iters, 0, true, hs));   // never converged: exactly iters each
        }
        HIPCHK(hipStreamSynchronize(hs));
        *ms = now_ms() - t0;
        if (h->policy != BQ_LAUNCHES) {
            unsigned int glob[BG_COUNT];
            HIPCHK(hipMemcpy(glob, h->b.glob, sizeof(glob), hipMemcpyDeviceToHost));
            if (glob[BG_ABORT]) return fail(MIFVM_E_STATE, "persistent batch solve stopped during autotuning");
        }
        return MIFVM_OK;
    };
    double ms = 0.0;
    TuneEntry best_p = {kDefaultItemRows, kDefaultGrid, kDefaultPolicy, 8, h->chunk};
    if ((rc = trial(best_p, &ms))) return rc;                      // warm-up
    double tp = 1e300;
    int n = 0;
    for (int policy : {BQ_ROTATE, BQ_XCD, BQ_LARGEST})
        for (int grid : {512, 1024, 2048}) {
            const TuneEntry e = {kDefaultItemRows, grid, policy, 8, h->chunk};
            if ((rc = trial(e, &ms))) return rc;
            ++n;
            if (ms < tp) {
                tp = ms;
                best_p = e;
            }
        }
    for (int item_rows : {1024, 2048, 8192, 16384, 32768, 65536}) {
        TuneEntry e = best_p;
        e[0] = item_rows;
        if ((rc = trial(e, &ms))) return rc;
        ++n;
        if (ms < tp) {
            tp = ms;
            best_p = e;
        }
    }
    {
        TuneEntry e = best_p;
        e[3] = 24;
        if ((rc = trial(e, &ms))) return rc;
        ++n;
        if (ms < tp) {
            tp = ms;
            best_p = e;
        }
    }
    double tl = 1e300;
    TuneEntry best_l = best_p;
    for (int chunk : {16, 32, 64}) {
        TuneEntry e = best_p;
        e[2] = BQ_LAUNCHES;
        e[4] = chunk;
        if ((rc = trial(e, &ms))) return rc;
        ++n;
        if (ms < tl) {
            tl = ms;
            best_l = e;
        }
    }
    HIPCHK(hipMemcpyAsync(d.x, saved_x, d.nc * sizeof(double), hipMemcpyDeviceToDevice, hs));
    const TuneEntry best = tl < tp ? best_l : best_p;
    if ((rc = apply(best))) return rc;
    info.item_rows = best[0];
    info.grid = best[1];
    info.policy = best[2];
    info.vertex_batch = best[3];
    info.chunk = best[4];
    info.trials = n;
    info.ms_best = std::fmin(tp, tl);
    info.ms_persistent = tp;
    info.ms_launches = tl;
    info.p_item_rows = best_p[0];
    info.p_grid = best_p[1];
    info.p_policy = best_p[2];
    info.p_vertex_batch = best_p[3];
    info.iterations = iters;
    if (cache_path) {
        cache[key] = best;
        write_batch_cache(cache_path, cache);
    }
    if (out) *out = info;
    return MIFVM_OK;
}
