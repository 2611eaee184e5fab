// Helpers shared by the translation units that implement the C ABI: error
// reporting, workspace carving, timed launches, graph capture, scalar pulls.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/mifvm.h"
#include "mesh.h"
#include "state.h"

struct mifvm_mesh {
    mifvm::Mesh m;
};
struct mifvm_state {
    mifvm::State s;
};

namespace mifvm_api {
inline thread_local std::string g_err;

inline int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
inline int hip_fail(hipError_t e, const char* where) {
    return fail(MIFVM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}
#define HIPCHK(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

inline hipStream_t S(void* p) { return reinterpret_cast<hipStream_t>(p); }

template <class T>
T* carve(char* base, size_t& off, size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
}

template <class T>
inline hipError_t up(T* dst, const std::vector<T>& src, hipStream_t s) {
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

inline int reduce_blocks(int64_t n) {
    int64_t b = (n + mifvm::kBlock - 1) / mifvm::kBlock;
    return int(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

// Launch `fn` on `s`; with timing on, bracket it with an event pair.
template <class F>
hipError_t timed(mifvm::KernelTimer& t, int kid, hipStream_t s, F fn) {
    if (!t.on || !((t.mask >> kid) & 1u)) return fn();
    while (t.pool.size() < t.used + 2) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        t.pool.push_back(e);
    }
    const size_t at = t.used;
    t.used += 2;
    hipError_t err = hipEventRecord(t.pool[at], s);
    if (err != hipSuccess) return err;
    err = fn();
    if (err != hipSuccess) return err;
    err = hipEventRecord(t.pool[at + 1], s);
    if (err != hipSuccess) return err;
    t.pending.emplace_back(kid, at);
    return hipSuccess;
}

// After the stream has been synchronised: fold pending pairs into totals.
inline hipError_t timer_flush(mifvm::KernelTimer& t) {
    for (auto& pr : t.pending) {
        float ms = 0.f;
        hipError_t err = hipEventElapsedTime(&ms, t.pool[pr.second], t.pool[pr.second + 1]);
        if (err != hipSuccess) return err;
        t.total_ms[pr.first] += ms;
        t.count[pr.first] += 1;
    }
    t.pending.clear();
    t.used = 0;
    return hipSuccess;
}

using namespace mifvm;

// Capture the launches `enqueue` makes on the library's capture stream into
// an executable graph (the kernels take their arguments by value, so the
// graph can be replayed on any stream).
template <class F>
inline hipError_t capture_graph(State& s, hipGraphExec_t* exec, F enqueue) {
    hipError_t e = hipSuccess;
    if (!s.cap_stream) {
        e = hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    e = hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue(s.cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s.cap_stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess) return e;
    if (*exec) (void)hipGraphExecDestroy(*exec);
    *exec = nullptr;
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

// n RK3 steps without timing events (api.hip)
hipError_t enqueue_steps(const mifvm::State& s, int n, double dt, hipStream_t q);
// the matrix-free product's per-cell tables of the current potential BC
// kinds, built if stale (api.hip)
int ensure_mf_tables(mifvm::State& s, hipStream_t hs);
// the diagonal, D^-1 and c of the current potential BCs, computed if stale,
// and the per-cell tables (api.hip)
int ensure_consts(mifvm::State& s, hipStream_t hs);

// copy every mesh's scalars to the pinned host mirror and wait
inline int pull_scalars(State& s, hipStream_t hs) {
    HIPCHK(hipMemcpyAsync(s.h_scal, s.d.scal, size_t(s.d.nm) * SC_COUNT_ * sizeof(double),
                          hipMemcpyDeviceToHost, hs));
    HIPCHK(hipStreamSynchronize(hs));
    return MIFVM_OK;
}
inline double hsc(const State& s, int m, int slot) { return s.h_scal[size_t(m) * SC_COUNT_ + slot]; }

// Flexible-CG phase of a learned solve (nn_api.hip): runs until the true
// residual meets tol, the iteration limit is reached, or a fallback to the
// plain solver is due (non-finite residual, stall, learned_maxit).
struct LearnedRun {
    int iterations = 0;
    int restarts = 0;
    bool fell_back = false;
};
int learned_phase(State& s, double tol, int maxit, int chunk, int restart, int stall_window, int learned_maxit,
                  bool use_graph, hipStream_t hs, const std::function<int()>& pull, LearnedRun& out);

// Multigrid-preconditioned flexible CG (amg_api.hip): runs until the true
// residual meets tol or the iteration limit; restarts counted.
// learned: the attached network replaces the finest level's Jacobi sweeps.
int amg_phase(State& s, double tol, int maxit, int chunk, int restart, bool use_graph, bool matrix_free,
              bool learned, hipStream_t hs, const std::function<int()>& pull, int& restarts);
// out = z(in) of the attached network (input scales, then the 3 layers;
// nn_api.hip), launches only
hipError_t nn_apply_vec(State& s, const double* in, double* out, hipStream_t q);
// free the hierarchy, its device record and graph of a state
void amg_release(State& s);

}  // namespace mifvm_api
