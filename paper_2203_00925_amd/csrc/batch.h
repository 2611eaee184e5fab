// Batched form: the Poisson solves of many independent meshes of one state
// run in one persistent kernel.  Each mesh's matrix-free Jacobi-CG is a
// sequence of phases (vertex values, the per-cell product, update,
// direction; and the opening from the true residual); a phase is split into
// items of consecutive rows.  Workgroups pull (mesh, phase, item) from
// per-mesh device queues; the workgroup that completes a phase's last item
// reduces its partial sums in item order (deterministic), updates the
// mesh's CG scalars and publishes the next phase.  No workgroup waits while
// holding an item, so the kernel drains whatever the grid's residency; a
// workgroup that sees no progress anywhere for a bounded number of polls
// raises an abort flag and every workgroup exits.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "state.h"

namespace mifvm {

constexpr int kBatchBlock = 256;          // threads per workgroup
constexpr int kBatchMinItemRows = 256;    // smallest item (partials are sized for it)
constexpr int kBatchMaxMeshes = 4096;

// phases of one mesh's solve (the queue word holds the phase in its high
// 32 bits and the next unclaimed item in its low 32 bits)
enum BatchPhase : uint32_t {
    BP_OV = 0,   // open: vertex values of x
    BP_OG,       // open: r = b - K x (per-cell product), z = D^-1 r, p = z; partial rz, rr, bb
    BP_V,        // vertex values of p
    BP_G,        // q = K p (per-cell product); partial p.q  -> alpha
    BP_AX,       // x += alpha p, r -= alpha q, z = D^-1 r; partial rz, rr -> beta, tests
    BP_DIR,      // p = z + beta p
    BP_ZX,       // b = 0: x = 0
    BP_IDLE      // finished
};

// global words
enum BatchGlob { BG_DONE = 0, BG_PROGRESS = 1, BG_ABORT = 2, BG_COUNT = 16 };

// queue policies: the order in which a workgroup looks at the meshes
// BQ_LAUNCHES: no persistent kernel - the per-launch matrix-free CG of the
// state (all meshes per launch, chunks of iterations replayed from a graph,
// the host checking between chunks)
enum BatchPolicy { BQ_ROTATE = 0, BQ_XCD = 1, BQ_LARGEST = 2, BQ_LAUNCHES = 3 };

struct BatchRange {
    int64_t c0, c1;     // cells
    int64_t v0, v1;     // vertices (numbered by their lowest cell)
    int64_t fi0, fi1;   // interior faces
    int64_t fb0, fb1;   // boundary faces
};

struct BatchDev {
    int32_t nm;
    int32_t item_rows;                // rows per item: a multiple of kBatchBlock
    const BatchRange* range;          // [nm]
    unsigned long long* q;            // [nm] queue word
    unsigned int* done;               // [nm] items completed in the current phase
    int32_t* fresh;                   // [nm] 1 until the first opening of a solve
    const int64_t* poff;              // [nm] first partial of the mesh: [3][pstride]
    const int64_t* pstride;           // [nm]
    double* partial;
    const int32_t* scan;              // [8][nm] mesh order per XCD
    unsigned int* glob;               // [BG_COUNT]
    double* rel_max;                  // [nm] largest final relative residual of a run
    int64_t* it_total;                // [nm] iterations summed over a run's solves
    long long spin_limit;             // polls without progress before an abort
};

// per-solve reset (queues at BP_OV, scalars, flags); zero_run: also the
// run's accumulators
hipError_t launch_batch_init(const Dev& d, const BatchDev& b, int maxit, int restart, bool zero_run,
                             hipStream_t s);
// the persistent solve of every mesh of the state
hipError_t launch_batch_solve(const Dev& d, const BatchDev& b, int grid, int vertex_batch, double tol,
                              hipStream_t s);
// ghost factors from the potential's boundary kinds

}  // namespace mifvm
