// Persistent batched solve (the batched form of the Poisson solves): every
// mesh of a multi-mesh state runs its own matrix-free Jacobi-CG, reopened
// from the true residual at convergence of the recurrence, at the iteration
// limit and every `restart` iterations, in one kernel launch.  The item
// bodies compute what the single-mesh kernels compute, in the same order:
// vertex values of Algorithm 2 with homogeneous ghosts, the diamond flux of
// eq. (diamond) on interior and Dirichlet faces, the gather over each cell's
// faces (the matrix-free product of eqs. (7), (laplace)), and the CG vector
// updates.
#include "batch.h"
#include "mf_cell.h"
#include "reduce.h"
#include "seg.h"
#include "state.h"

namespace mifvm {
namespace {

__device__ inline int64_t phase_rows(const BatchRange& r, uint32_t ph) {
    switch (ph) {
        case BP_OV:
        case BP_V: return r.v1 - r.v0;
        case BP_IDLE: return 0;
        default: return r.c1 - r.c0;
    }
}

__device__ inline int64_t phase_items(const BatchDev& b, const BatchRange& r, uint32_t ph) {
    return (phase_rows(r, ph) + b.item_rows - 1) / b.item_rows;
}

// queue word: item index in bits 0-31, phase in 32-39, phase epoch (counts
// the mesh's phase changes) in 40-63
__device__ inline uint32_t q_phase(unsigned long long w) { return uint32_t(w >> 32) & 0xffu; }
__device__ inline int64_t q_item(unsigned long long w) { return int64_t(w & 0xffffffffull); }
__device__ inline unsigned long long q_word(uint32_t epoch, uint32_t phase) {
    return ((unsigned long long)(epoch & 0xffffffu) << 40) | ((unsigned long long)phase << 32);
}
// fences at device (agent) scope: a release writes back what this
// workgroup stored, an acquire drops stale cached copies; each is paid only
// where the queue protocol needs it
__device__ inline void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ inline void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ inline unsigned long long ld_q(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned int ld_u(const unsigned int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// x_v = sum alpha_{v,e} src_e over the vertex list, each ghost entry folded
// onto its owner (the operator's list, mf_nidx).  Entries in batches of VB (a schedule choice: 24, the
// single-mesh vertex kernel's, keeps more gathers in flight; 8 needs fewer
// registers, so more waves stay resident), the indices and weights of a
// batch loaded before its values, summed in list order (so the values are
// the single-mesh kernel's bits).
template <int kVb>
__device__ inline double vertex_value(const Dev& d, const BatchDev& b, const double* __restrict__ src, int64_t v) {
    const int64_t sl = v >> 6;
    const int64_t base = d.n_off[sl] + (v & 63);
    const int w = d.n_w[sl];
    double s = 0.0;
    for (int k0 = 0; k0 < w; k0 += kVb) {
        int e[kVb];
        double al[kVb];
#pragma unroll
        for (int j = 0; j < kVb; ++j) {
            const bool in = k0 + j < w;
            const int64_t at = base + int64_t(k0 + j) * 64;
            e[j] = in ? d.mf_nidx[at] : 0;            // padding entries carry weight 0
            al[j] = in ? d.n_alpha[at] : 0.0;
        }
        double xe[kVb];
#pragma unroll
        for (int j = 0; j < kVb; ++j) {              // a ghost folded onto its owner, as ~owner for -x
            const double xo = src[e[j] >= 0 ? e[j] : ~e[j]];
            xe[j] = e[j] >= 0 ? xo : -xo;
        }
#pragma unroll
        for (int j = 0; j < kVb; ++j) s += al[j] * xe[j];
    }
    return s;
}

// one item: rows [lo, hi) of the phase's range; partial sums of the item
// into its slots
template <int VB>
__device__ void run_item(const Dev& d, const BatchDev& b, const BatchRange& r, uint32_t ph, int m, int64_t item,
                         double* lds) {
    const int64_t lo = item * b.item_rows;
    const int64_t hi = min(lo + int64_t(b.item_rows), phase_rows(r, ph));
    const int tid = threadIdx.x;
    const double* sc = msc(d, m);
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    switch (ph) {
        case BP_OV:
        case BP_V: {
            const double* src = ph == BP_OV ? d.x : d.p;
#pragma unroll 1
            for (int64_t k = lo + tid; k < hi; k += kBatchBlock) d.mf_xv[r.v0 + k] = vertex_value<VB>(d, b, src, r.v0 + k);
            break;
        }
        case BP_OG:
#pragma unroll 1
            for (int64_t k = lo + tid; k < hi; k += kBatchBlock) {
                const int64_t i = r.c0 + k;
                const double bi = d.b[i];
                const double ri = bi - cell_row(d, d.x, d.mf_xv, i);
                const double zi = d.k_dinv[i] * ri;
                d.r[i] = ri;
                d.z[i] = zi;
                d.p[i] = zi;
                v0 += ri * zi;
                v1 += ri * ri;
                v2 += bi * bi;
            }
            break;
        case BP_G:
#pragma unroll 1
            for (int64_t k = lo + tid; k < hi; k += kBatchBlock) {
                const int64_t i = r.c0 + k;
                const double y = cell_row(d, d.p, d.mf_xv, i);
                d.q[i] = y;
                v0 += d.p[i] * y;
            }
            break;
        case BP_AX: {
            const double alpha = sc[SC_ALPHA];
#pragma unroll 1
            for (int64_t k = lo + tid; k < hi; k += kBatchBlock) {
                const int64_t i = r.c0 + k;
                d.x[i] += alpha * d.p[i];
                const double ri = d.r[i] - alpha * d.q[i];
                const double zi = d.k_dinv[i] * ri;
                d.r[i] = ri;
                d.z[i] = zi;
                v0 += ri * zi;
                v1 += ri * ri;
            }
            break;
        }
        case BP_DIR: {
            const double beta = sc[SC_BETA];
#pragma unroll 1
            for (int64_t k = lo + tid; k < hi; k += kBatchBlock) {
                const int64_t i = r.c0 + k;
                d.p[i] = d.z[i] + beta * d.p[i];
            }
            break;
        }
        case BP_ZX:
#pragma unroll 1
            for (int64_t k = lo + tid; k < hi; k += kBatchBlock) d.x[r.c0 + k] = 0.0;
            break;
        default: break;
    }
    const int nsum = ph == BP_OG ? 3 : (ph == BP_AX ? 2 : (ph == BP_G ? 1 : 0));
    double* part = b.partial + b.poff[m];
    const int64_t stride = b.pstride[m];
    if (nsum > 0) {
        const double s0 = block_sum256(v0, lds);
        if (tid == 0) part[item] = s0;
    }
    if (nsum > 1) {
        const double s1 = block_sum256(v1, lds);
        if (tid == 0) part[stride + item] = s1;
    }
    if (nsum > 2) {
        const double s2 = block_sum256(v2, lds);
        if (tid == 0) part[2 * stride + item] = s2;
    }
}

// sum of partial slot s over n items, in item order per thread, then the
// threads in a fixed order (deterministic)
__device__ inline double sum_items(const BatchDev& b, int m, int s, int64_t n, double* lds) {
    const double* part = b.partial + b.poff[m] + s * b.pstride[m];
    double acc = 0.0;
    for (int64_t it = threadIdx.x; it < n; it += kBatchBlock) acc += part[it];
    return block_sum256(acc, lds);
}

// the phase after `ph` of mesh m has completed (every item); updates the
// mesh's scalars (thread 0 writes); returns the next phase
__device__ uint32_t finish_phase(const Dev& d, const BatchDev& b, const BatchRange& r, uint32_t ph, int m,
                                 double tol, double* lds) {
    double* sc = msc(d, m);
    const int64_t n = phase_items(b, r, ph);
    const bool t0 = threadIdx.x == 0;
    switch (ph) {
        case BP_OV: return BP_OG;
        case BP_V: return BP_G;
        case BP_DIR: return BP_V;
        case BP_ZX: return BP_IDLE;
        case BP_G: {
            const double pq = sum_items(b, m, 0, n, lds);
            if (t0) {
                sc[SC_PQ] = pq;
                sc[SC_ALPHA] = sc[SC_RZ] / pq;
            }
            return BP_AX;
        }
        case BP_AX: {
            const double trz = sum_items(b, m, 0, n, lds);
            const double trr = sum_items(b, m, 1, n, lds);
            const double rz_old = sc[SC_RZ];
            const double it = sc[SC_IT] + 1.0, since = sc[SC_SINCE] + 1.0;
            __syncthreads();                       // every thread has read the old scalars
            if (t0) {
                sc[SC_BETA] = trz / rz_old;
                sc[SC_RZ] = trz;
                sc[SC_RR] = trr;
                sc[SC_IT] = it;
                sc[SC_SINCE] = since;
            }
            // the recurrence converged, the limit or a restart is due: the
            // true residual decides
            const bool reopen = trr <= sc[SC_TOL2BB] || it >= sc[SC_MAXIT] ||
                                (sc[SC_RESTART] > 0.0 && since >= sc[SC_RESTART]);
            return reopen ? BP_OV : BP_DIR;
        }
        case BP_OG: {
            const double trz = sum_items(b, m, 0, n, lds);
            const double trr = sum_items(b, m, 1, n, lds);
            const double tbb = sum_items(b, m, 2, n, lds);
            const bool fresh = b.fresh[m] != 0;
            const double tol2bb = fresh ? tol * tol * tbb : sc[SC_TOL2BB];
            const double it = sc[SC_IT], maxit = sc[SC_MAXIT];
            __syncthreads();
            uint32_t next;
            double done = 0.0;
            if (tbb == 0.0) {                      // b = 0: the solution is 0
                next = BP_ZX;
                done = 1.0;
            } else if (trr <= tol2bb) {
                next = BP_IDLE;
                done = 1.0;
            } else if (it >= maxit) {
                next = BP_IDLE;
                done = 2.0;
            } else {
                next = BP_V;
            }
            if (t0) {
                sc[SC_RZ] = trz;
                sc[SC_RR] = trr;
                sc[SC_TRUE_RR] = trr;
                sc[SC_BB] = tbb;
                sc[SC_TOL2BB] = tol2bb;
                sc[SC_SINCE] = 0.0;
                sc[SC_DONE] = done;
                b.fresh[m] = 0;
                if (done != 0.0) {
                    b.it_total[m] += int64_t(it);
                    const double rel = tbb > 0.0 ? sqrt(trr / tbb) : 0.0;
                    if (rel > b.rel_max[m]) b.rel_max[m] = rel;
                }
            }
            return next;
        }
        default: return BP_IDLE;
    }
}

template <int VB>
__global__ __launch_bounds__(kBatchBlock) void k_batch_solve(Dev d, BatchDev b, double tol) {
    __shared__ double lds[4];
    __shared__ long long s_cmd[4];           // phase (-1 none, -2 exit), mesh, item, epoch
    __shared__ int s_last;
    const int tid = threadIdx.x;
    const int nm = b.nm;
    const int32_t* scan = b.scan + int64_t(blockIdx.x % 8) * nm;
    unsigned int seen = 0xffffffffu;
    long long idle = 0;
    long long last_m = -1, last_ep = -1;     // wave 0: the epoch last acquired
    for (;;) {
        if (tid < 64) {                       // wave 0 looks for an item
            long long cph = -1, cm = 0, ci = 0, cep = 0;
            // the global words as lane 0 reads them (one value for the wave)
            const unsigned int gdone = __shfl(ld_u(&b.glob[BG_DONE]), 0, 64);
            const unsigned int gabort = __shfl(ld_u(&b.glob[BG_ABORT]), 0, 64);
            if (gdone >= unsigned(nm) || gabort != 0u) {
                cph = -2;
            } else {
                for (int c0 = 0; c0 < nm && cph == -1; c0 += 64) {
                    const int k = c0 + tid;
                    int m = 0;
                    bool avail = false;
                    if (k < nm) {
                        m = scan[k];
                        const unsigned long long w = ld_q(&b.q[m]);
                        avail = q_item(w) < phase_items(b, b.range[m], q_phase(w));
                    }
                    unsigned long long mask = __ballot(avail);
                    while (mask != 0ull && cph == -1) {
                        const int lane = __ffsll((long long)mask) - 1;
                        int ok = 0;
                        unsigned long long w2 = 0ull;
                        if (tid == lane) {
                            w2 = atomicAdd(&b.q[m], 1ull);
                            ok = q_item(w2) < phase_items(b, b.range[m], q_phase(w2));
                        }
                        ok = __shfl(ok, lane, 64);
                        if (ok) {
                            const unsigned lo32 = __shfl(unsigned(w2 & 0xffffffffull), lane, 64);
                            const unsigned hi32 = __shfl(unsigned(w2 >> 32), lane, 64);
                            cph = hi32 & 0xffu;
                            cep = hi32 >> 8;
                            cm = __shfl(m, lane, 64);
                            ci = lo32;
                        }
                        mask &= mask - 1ull;
                    }
                }
                if (cph == -1) {                  // nothing to take: count polls without progress
                    const unsigned int pr = __shfl(ld_u(&b.glob[BG_PROGRESS]), 0, 64);
                    if (pr != seen) {
                        seen = pr;
                        idle = 0;
                    } else if (++idle > b.spin_limit) {
                        if (tid == 0) atomicExch(&b.glob[BG_ABORT], 1u);
                        cph = -2;
                    }
                }
            }
            // acquire the phase's inputs (written by other workgroups) once
            // per phase epoch: later items of the same epoch read the same data
            if (cph >= 0 && (cm != last_m || cep != last_ep)) {
                fence_acquire();
                last_m = cm;
                last_ep = cep;
            }
            if (tid == 0) {
                s_cmd[0] = cph;
                s_cmd[1] = cm;
                s_cmd[2] = ci;
                s_cmd[3] = cep;
            }
            if (cph == -1) __builtin_amdgcn_s_sleep(2);
        }
        __syncthreads();
        const long long ph = s_cmd[0];
        if (ph == -2) return;
        if (ph == -1) {
            __syncthreads();                    // s_cmd is rewritten only after every wave read it
            continue;
        }
        const int m = int(s_cmd[1]);
        const int64_t item = s_cmd[2];
        const BatchRange r = b.range[m];
        run_item<VB>(d, b, r, uint32_t(ph), m, item, lds);
        fence_release();                        // every wave releases its stores of the item
        __syncthreads();                        // ... before the item is counted
        if (tid == 0) {
            const unsigned int old = atomicAdd(&b.done[m], 1u);
            s_last = int64_t(old) + 1 == phase_items(b, r, uint32_t(ph)) ? 1 : 0;
            if (s_last) fence_acquire();        // every other item's results
        }
        __syncthreads();
        if (s_last) {
            const uint32_t next = finish_phase(d, b, r, uint32_t(ph), m, tol, lds);
            __syncthreads();                    // scalars written before they are released
            if (tid == 0) {
                atomicExch(&b.done[m], 0u);
                fence_release();                // scalars and the reset before the new phase
                atomicExch(&b.q[m], q_word(uint32_t(s_cmd[3]) + 1u, next));
                atomicAdd(&b.glob[BG_PROGRESS], 1u);
                if (next == BP_IDLE) atomicAdd(&b.glob[BG_DONE], 1u);
            }
        }
        __syncthreads();                        // s_cmd and s_last are reused
    }
}

__global__ void k_batch_init(Dev d, BatchDev b, int maxit, int restart, int zero_run) {
    const int m = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (m == 0)
        for (int k = 0; k < BG_COUNT; ++k) b.glob[k] = 0u;
    if (m >= b.nm) return;
    b.q[m] = q_word(0u, BP_OV);
    b.done[m] = 0u;
    b.fresh[m] = 1;
    double* sc = msc(d, m);
    sc[SC_IT] = 0.0;
    sc[SC_MAXIT] = double(maxit);
    sc[SC_RESTART] = double(restart);
    sc[SC_SINCE] = 0.0;
    sc[SC_DONE] = 0.0;
    if (zero_run) {
        b.it_total[m] = 0;
        b.rel_max[m] = 0.0;
    }
}


}  // namespace

hipError_t launch_batch_init(const Dev& d, const BatchDev& b, int maxit, int restart, bool zero_run,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_batch_init, dim3(unsigned((b.nm + 255) / 256)), dim3(256), 0, s, d, b, maxit, restart,
                       zero_run ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_solve(const Dev& d, const BatchDev& b, int grid, int vertex_batch, double tol,
                              hipStream_t s) {
    if (vertex_batch == 24)
        hipLaunchKernelGGL(k_batch_solve<24>, dim3(unsigned(grid)), dim3(kBatchBlock), 0, s, d, b, tol);
    else
        hipLaunchKernelGGL(k_batch_solve<8>, dim3(unsigned(grid)), dim3(kBatchBlock), 0, s, d, b, tol);
    return hipGetLastError();
}


}  // namespace mifvm
