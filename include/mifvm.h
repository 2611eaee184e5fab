/*
 * mifvm.h - C ABI of the MI355X finite-volume library.
 *
 * The library implements the data-parallel hot path of the cell-centred
 * finite-volume method of Kissami & Ratnani (arXiv 2203.00925, "Manapy"):
 * one explicit time step of the convection-diffusion equation (Sec. 2.1,
 * eqs. (1)-(4), (15), (diamond), (6)) on an unstructured tetrahedral mesh,
 * and the assembly and solve of the Poisson system the same discretisation
 * gives (Sec. 2.2, eqs. (7), (laplace)).  The calls mirror the paper's
 * problem statement (annex example): load a mesh, declare a variable with
 * boundary conditions, step, assemble, solve.
 *
 * Conventions, common to every call:
 *  - status: 0 = OK, > 0 = non-fatal outcome, < 0 = error; no exception or
 *    abort crosses the ABI.  mifvm_last_error() returns a thread-local text
 *    for the last failing call on this thread (valid until the next call).
 *  - "d_" pointers are device pointers (HIP device memory on the current
 *    device); every other pointer is host memory.  Host arrays are copied
 *    during the call and may be freed afterwards.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  Device
 *    work is enqueued on that stream only; calls that return a host scalar
 *    synchronise the stream, all others are asynchronous.
 *  - field arrays at the ABI are in the caller's ("user") cell order, the
 *    order of the tets array given to mifvm_mesh_preprocess; the library
 *    renumbers internally.
 *  - handles are owned by the library and freed with the matching
 *    *_destroy; a handle may be used by one thread at a time.
 *  - the device workspace is owned by the caller; it must be at least
 *    mifvm_mesh_info.ws_bytes bytes, 256-byte aligned, and outlive the
 *    state that uses it.
 */
#ifndef MIFVM_H
#define MIFVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mifvm_status {
    MIFVM_OK = 0,
    MIFVM_NOT_CONVERGED = 1,   /* solve hit maxit; info is filled          */
    MIFVM_FELL_BACK = 2,       /* learned solve stalled, switched to plain
                                  Jacobi-CG and converged; info is filled   */
    MIFVM_E_ARG = -1,          /* invalid argument (null, range, size)      */
    MIFVM_E_MESH = -2,         /* degenerate/inverted cell, non-manifold or
                                  untagged boundary face                    */
    MIFVM_E_HIP = -3,          /* a HIP runtime call failed                 */
    MIFVM_E_WORKSPACE = -4,    /* workspace too small or misaligned         */
    MIFVM_E_STATE = -5         /* call out of order (e.g. solve before
                                  assemble)                                 */
};

/* boundary-condition kinds, per boundary tag (the per-name dictionary of the
 * paper's annex).  Ghost value u_g = s*u_owner + t:
 *   ZERO_FLUX  no flux of any kind crosses the face; ghost (1, 0)
 *   NEUMANN    du/dn = value: diffusive flux D*value*|S|, convective upwind
 *              with the ghost value on inflow; ghost (1, value*|x_g - x_L|)
 *   DIRICHLET  u = value on the face: diamond flux with the ghost as the
 *              right cell, convective upwind; ghost (-1, 2*value)          */
enum mifvm_bc_kind { MIFVM_ZERO_FLUX = 0, MIFVM_NEUMANN = 1, MIFVM_DIRICHLET = 2 };

/* variables with their own boundary conditions */
enum mifvm_var { MIFVM_VAR_SCALAR = 0, MIFVM_VAR_POTENTIAL = 1 };

/* element type of a field array at the ABI (mifvm_set_field/get_field) */
enum mifvm_dtype { MIFVM_F64 = 0, MIFVM_F32 = 1 };

/* per-cell fields (user cell order; float64 or float32, see mifvm_dtype) */
enum mifvm_field {
    MIFVM_FIELD_U = 0,        /* transported scalar u                        */
    MIFVM_FIELD_VEL = 1,      /* velocity, 3*Nc values laid out [x..., y..., z...] */
    MIFVM_FIELD_SOURCE = 2,   /* source S_i of eq. (1)                        */
    MIFVM_FIELD_P = 3,        /* Poisson unknown (last solution)              */
    MIFVM_FIELD_ION = 4,      /* positive-ion density n_p of the coupled loop  */
    MIFVM_FIELD_EFIELD = 5    /* E = -grad P of the last coupled step, 3*Nc values
                                 [x..., y..., z...] (get only)                */
};

/* internal cell order: as given, Morton order of the centres, or reverse
 * Cuthill-McKee on the face-adjacency graph (per mesh and component, from a
 * pseudo-peripheral cell); vertices follow their lowest cell              */
enum mifvm_renumber { MIFVM_RENUMBER_NONE = 0, MIFVM_RENUMBER_MORTON = 1, MIFVM_RENUMBER_RCM = 2 };

#define MIFVM_MAX_TAGS 32

typedef struct mifvm_mesh mifvm_mesh;     /* host-side preprocessed mesh     */
typedef struct mifvm_state mifvm_state;   /* device-resident mesh + fields   */

typedef struct {
    int32_t renumber;          /* enum mifvm_renumber                         */
    int32_t nmeshes;           /* independent meshes in the tets array (>=1)  */
    const int64_t* mesh_cell_start;  /* nmeshes+1 offsets into tets; mesh m is
                                  tets[start[m]:start[m+1]]; NULL when
                                  nmeshes <= 1.  Meshes of a batch share no
                                  face; each needs >= 256 cells.             */
    int32_t no_matrix;         /* 1 = do not build the stored Poisson pattern
                                  (no assembly, no stored-matrix solves; the
                                  matrix-free solves need none of it): the
                                  workspace shrinks by about 17 B per matrix
                                  entry (8.7 GB for the 10.4M-cell cube)      */
    int32_t pad_;
} mifvm_mesh_opts;

typedef struct {
    int64_t nc;                /* cells                                       */
    int64_t nv;                /* vertices                                    */
    int64_t nf;                /* faces (interior first, then boundary)       */
    int64_t nf_interior;
    int64_t nb;                /* boundary faces = ghost cells                */
    int32_t nmeshes;           /* independent meshes (batch size)             */
    int32_t pad0_;
    int64_t stencil_entries;   /* node-neighbour entries (unpadded)           */
    int64_t stencil_padded;    /* stored entries after 64-row slicing         */
    int64_t node_entries;      /* vertex->cell/ghost entries (unpadded)       */
    int64_t matrix_nnz;        /* Poisson entries incl. diagonal (pattern)    */
    int64_t matrix_padded;     /* stored off-diagonal entries after slicing   */
    int32_t stencil_max;       /* longest node-neighbour list                 */
    int32_t node_max;          /* longest vertex list                         */
    int32_t row_max;           /* longest off-diagonal matrix row             */
    int32_t tile_rows;         /* cells per LDS tile (256, 128 or 64)         */
    int32_t halo_max;          /* largest tile halo (cells + ghosts)          */
    int32_t tile_vertices_max; /* most vertices the cells of one tile touch   */
    int64_t halo_entries;      /* sum of tile halo sizes                      */
    size_t ws_bytes;           /* device workspace needed by a state          */
    int64_t edge_nbr_entries;  /* entities sharing only an edge with a cell,
                                  summed over cells (unpadded)                */
    int64_t foreign_rows;      /* vertices touched by a tile's cells but owned
                                  by another tile, summed over tiles          */
    int64_t foreign_entries;   /* entries of their vertex lists (unpadded)    */
} mifvm_mesh_info;

typedef struct {
    double diffusivity;        /* D of eq. (1)                                */
    int32_t precision;         /* enum mifvm_precision                        */
    int32_t pad_;
} mifvm_params;

/* FP64: the step in FP64.  FP32: the reduced-precision form - state,
 * gradients, limiter, vertex values, fluxes and the geometry they read in
 * FP32 (positions relative to a nearby cell); the CFL bound and the
 * conservation sum stay FP64.  Fields cross the ABI in either element type
 * (mifvm_dtype) whatever the precision of the state.                       */
enum mifvm_precision { MIFVM_FP64 = 0, MIFVM_FP32 = 1 };

typedef struct {
    double tol;                /* relative true residual ||b-Kx||/||b||       */
    int32_t maxit;             /* iteration limit                             */
    int32_t chunk;             /* iterations enqueued between host checks    */
    int32_t restart;           /* restart from the true residual every this
                                  many iterations (0 = only when the
                                  recurrence residual claims convergence)    */
    int32_t history_cap;       /* capacity of history (0 = none)              */
    double* history;           /* host, optional: recurrence ||r||/||b|| at
                                  every host check                           */
    int32_t method;            /* enum mifvm_solve_method                     */
    int32_t graph;             /* 1: enqueue each chunk by replaying a captured
                                  hipGraph (not while kernel timing is on);
                                  -1: the autotuned choice (else 0)          */
    double inner_tol;          /* IR_FP32: relative reduction asked of each
                                  FP32 inner solve (0 = 1e-4)                */
    int32_t stall_window;      /* LEARNED: fall back when the best residual
                                  norm has not dropped by 1% in this many
                                  iterations (0 = 200)                      */
    int32_t learned_maxit;     /* LEARNED: fall back after this many flexible
                                  CG iterations (0 = maxit)                  */
    int32_t matrix_free;       /* 1 = apply K in the iterations from the
                                  discretisation (vertex values, diamond
                                  fluxes, cell gather) instead of the stored
                                  matrix, the true residual included; needs
                                  no assembly (the diagonal, D^-1 and c are
                                  computed from the discretisation when the
                                  POTENTIAL BCs have changed).  IR_FP32: the
                                  inner CG applies
                                  it in FP32 (FP32 copies of the vertex
                                  weights and diamond coefficients) and the
                                  true residual in FP64                      */
    int32_t learned_smoother;  /* AMG: 1 = the attached network (mifvm_nn.h)
                                  replaces the Jacobi sweeps of the finest
                                  level: x = z(b), then after the coarse
                                  correction x += z(b - K x); E_STATE
                                  without an attached network               */
} mifvm_solve_opts;

/* PLAIN: FP64 Jacobi-CG.  IR_FP32: iterative refinement - the FP64 true
 * residual r = b - K x, an FP32 Jacobi-CG solve of K d = r on an FP32 copy of
 * K or the FP32 matrix-free product (dot products accumulated in FP64),
 * x += d in FP64 - repeated until the FP64 true residual meets tol.        */
enum mifvm_solve_method { MIFVM_SOLVE_PLAIN = 0, MIFVM_SOLVE_IR_FP32 = 1, MIFVM_SOLVE_LEARNED = 2,
                          MIFVM_SOLVE_FGMRES = 3, MIFVM_SOLVE_AMG = 4 };
/* AMG: flexible CG (Polak-Ribiere beta) preconditioned by one V(1,1) cycle
 * of the attached aggregation multigrid (mifvm_amg_build/attach), reopened
 * from the true residual when the recurrence converges or `restart`
 * iterations have passed.  Single-mesh states; matrix_free chooses the
 * product of the outer iteration (the cycle's finest level always applies K
 * matrix-free).                                                            */
/* FGMRES: restarted flexible GMRES(m) with the Jacobi preconditioner, the
 * Krylov method of the paper's solver runs (Sec. 3.4.2): right
 * preconditioning z_j = D^-1 v_j, classical Gram-Schmidt, Givens rotations,
 * and a new cycle from the true residual every m steps (m from
 * mifvm_fgmres_attach; `restart` is not used).  `iterations` counts steps,
 * `outer` cycles.  Needs a single-mesh state with an FGMRES workspace;
 * matrix_free applies.                                                     */
/* LEARNED: flexible CG (Polak-Ribiere beta) preconditioned by the attached
 * message-passing network (mifvm_nn.h), with restarts from the true residual
 * as for PLAIN.  A non-finite residual (the iterate is reset to the last
 * finite one), a stall (stall_window) or learned_maxit switches to PLAIN
 * Jacobi-CG from the current iterate for the remaining iterations; the
 * result is then FELL_BACK (or NOT_CONVERGED).  Needs a single-mesh state
 * with an attached network.                                                 */

typedef struct {
    int32_t iterations;
    int32_t restarts;          /* times the loop was reopened from the true
                                  residual without having converged           */
    int32_t history_len;       /* entries written to opts->history            */
    int32_t outer;             /* IR_FP32: refinement steps                   */
    double rel_residual;       /* final true relative residual (FP64)        */
    double ms;                 /* wall time of the solve call                */
    int32_t fell_back;         /* LEARNED: 1 if the plain solver finished    */
    int32_t learned_iterations;/* LEARNED: flexible-CG iterations            */
} mifvm_solve_info;

/* ---- errors --------------------------------------------------------------- */
const char* mifvm_last_error(void);
const char* mifvm_version(void);

/* ---- load mesh (readmesh + Domain of the paper's annex) --------------------
 * xyz: float64 [nv][3]; tets: int32 [nc][4] (any orientation); btris: int32
 * [nb][3] boundary triangles with tags btags[nb] in [0, MIFVM_MAX_TAGS).
 * Computes, on the host: orientation, volumes, centres of gravity, faces
 * (interior ones have L = the owner with the smaller user index), face
 * vectors S (L -> R), face centroids, ghost cells (owner centre mirrored
 * across the face), the node-neighbour stencil of Algorithm 1 with the
 * inverse of its normal matrix, the vertex lists of Algorithm 2 with their
 * least-squares weights, the diamond coefficients of eq. (diamond), the
 * cell->face table and the sparsity pattern of the Poisson matrix; then
 * renumbers cells by a Morton curve of their centres.
 * Errors: E_ARG (null/negative sizes, index out of range), E_MESH (cell
 * volume <= 1e-14 * mean volume, a face shared by more than two cells, a
 * boundary face without a tag or a tag on an interior face).              */
int mifvm_mesh_preprocess(const double* xyz, int64_t nv, const int32_t* tets, int64_t nc,
                          const int32_t* btris, const int32_t* btags, int64_t nb,
                          const mifvm_mesh_opts* opts, mifvm_mesh** out);
int mifvm_mesh_get_info(const mifvm_mesh* mesh, mifvm_mesh_info* out);
void mifvm_mesh_destroy(mifvm_mesh* mesh);

/* Copy one preprocessed host array out (for inspection and tests; no GPU).
 * what (all internal numbering unless stated):
 *   0 CELL_PERM   int32 [nc]  internal cell -> user cell
 *   1 VERT_PERM   int32 [nv]  internal vertex -> user vertex
 *   2 VOLUME      f64   [nc]
 *   3 CENTRE      f64   [3][nc+nb]  cells then ghosts, SoA
 *   4 FACE_LR     int32 [2][nf]     L, R (R >= nc: ghost R-nc)
 *   5 FACE_ABC    int32 [3][nf]     diamond vertex labels (internal vertices)
 *   6 FACE_COEF   f64   [3][nf]     kAC, kBC, kRL
 *   7 FACE_S      f64   [3][nf]     face vector
 *   8 STENCIL_PTR int64 [nc+1]      CSR over internal cells
 *   9 STENCIL_IDX int32 [stencil_entries]  cell or nc+ghost, ascending
 *  10 NODE_PTR    int64 [nv+1]
 *  11 NODE_IDX    int32 [node_entries]
 *  12 NODE_ALPHA  f64   [node_entries]
 *  13 GHOST_OWNER int32 [nb]
 *  14 GHOST_TAG   int32 [nb]
 *  15 MINV        f64   [6][nc]     xx, xy, xz, yy, yz, zz of M_i^{-1}
 *  16 EDGE_NBR_PTR int64 [nc+1]     CSR over internal cells of the entities
 *  17 EDGE_NBR_IDX int32 [edge_nbr_entries]  sharing exactly two vertices
 *                                    with the cell (cell or nc+ghost, ascending)
 * bytes must equal the array's size exactly (E_ARG otherwise).            */
int mifvm_mesh_export(const mifvm_mesh* mesh, int32_t what, void* dst, size_t bytes);

/* ---- variable + boundary conditions (Variable(domain, BC, values)) ------- */
int mifvm_state_create(const mifvm_mesh* mesh, const mifvm_params* params,
                       void* d_ws, size_t ws_bytes, void* stream, mifvm_state** out);
void mifvm_state_destroy(mifvm_state* st);
/* kind/value for one boundary tag of one variable (Annexes: the per-name
 * dictionary of Variable(domain, BC, values)); default ZERO_FLUX, 0.  The
 * value is written to every ghost of the tag in device memory (the call
 * synchronises the device before and after).  It takes effect at the next
 * step (SCALAR) or solve (POTENTIAL; a stored matrix must be assembled
 * again).  Captured graphs (mifvm_step_graph, graph-replayed solves) are
 * dropped and captured again at their next use.                           */
int mifvm_set_bc(mifvm_state* st, int32_t var, int32_t tag, int32_t kind, double value);
/* Per-face values for one tag of one variable, for data that varies along
 * a boundary (Dirichlet data at each face's foot point, a Neumann flux per
 * face): d_vals holds one float64 per boundary triangle given to
 * mifvm_mesh_preprocess, in that order (nb values); the entries of
 * triangles with another tag are not read.  The kind stays the one set by
 * mifvm_set_bc.  Asynchronous on `stream`; later steps, solves and graph
 * replays read the new values.  POTENTIAL: the ghost constants c change, so
 * a stored matrix must be assembled again (matrix-free solves recompute c).
 * E_ARG for a null pointer, an unknown variable or a tag out of range.     */
int mifvm_set_bc_values(mifvm_state* st, int32_t var, int32_t tag, const double* d_vals, void* stream);
int mifvm_set_diffusivity(mifvm_state* st, double diffusivity);          /* every mesh */
/* one diffusivity per mesh of a batch (n = nmeshes).  Synchronises.        */
int mifvm_set_mesh_diffusivity(mifvm_state* st, const double* D, int32_t n);
/* d_src: nc values (3*nc for VEL, laid out [x..., y..., z...]) in user cell
 * order, of element type dtype (mifvm_dtype).  A value crosses into the
 * state's precision by round to nearest; FIELD_U of an FP32 state from F32
 * data is taken as is.  Setting VEL recomputes the face velocity fluxes
 * phi_f = 1/2 (V_L + V_R) . S_f.  get_field writes the same layout.
 * E_ARG for a null pointer, an unknown field or dtype (and EFIELD to set).  */
int mifvm_set_field(mifvm_state* st, int32_t field, const void* d_src, int32_t dtype, void* stream);
int mifvm_get_field(const mifvm_state* st, int32_t field, void* d_dst, int32_t dtype, void* stream);

/* ---- step (eq. (4) with the Runge-Kutta scheme of eq. (6)) ---------------
 * Per mesh: dt_m = cfl * min_i mu_i / sum_{faces of i not ZERO_FLUX}
 * (|phi_f| + D_m kRL_f); returns the smallest and keeps every dt_m for
 * steps called with dt = 0.  Synchronises.                                 */
int mifvm_cfl_dt(mifvm_state* st, double cfl, double* dt_out, void* stream);
/* n_steps explicit 3-stage steps u^(k) = u^n + a_k dt Res(u^(k-1)),
 * a = (1/2, 1/2, 1); dt > 0 for every mesh, dt = 0 for each mesh's own CFL
 * step (E_STATE before any mifvm_cfl_dt).  Asynchronous.                   */
int mifvm_step(mifvm_state* st, int32_t n_steps, double dt, void* stream);
/* One evaluation of Res(U) and its parts, for inspection; any output may be
 * NULL.  d_res, d_psi [nc], d_grad [3][nc] in user cell order; d_unode [nv]
 * in user vertex order; d_flux [nf] in internal face order (FACE_LR gives
 * each face's cells).                                                      */
int mifvm_residual(mifvm_state* st, double* d_res, double* d_grad, double* d_psi,
                   double* d_unode, double* d_flux, void* stream);
/* sum_i mu_i u_i in FP64 over all meshes (per mesh, deterministic order,
 * then the meshes in order).  Synchronises.                                */
int mifvm_conservation(mifvm_state* st, double* total_out, void* stream);
/* Discrete L2 norm of a field's difference from a given one, as the
 * annex's error report (norml2 with order 1): sqrt(sum_i mu_i (a_i - e_i)^2)
 * over all cells (cell-centre quadrature); field is FIELD_U, FIELD_P or
 * FIELD_ION, d_exact (user cell order) may be NULL for e = 0.  FP64.
 * Synchronises.                                                            */
int mifvm_norm_l2(mifvm_state* st, int32_t field, const double* d_exact, double* out, void* stream);
/* Per-mesh results of the last call that produced them (n = nmeshes):
 * what 0 = dt_m of mifvm_cfl_dt, 1 = conservation total, 2 = iterations of
 * the last solve, 3 = its true relative residual.                          */
int mifvm_mesh_values(const mifvm_state* st, int32_t what, double* out, int32_t n);

/* ---- Poisson (LinearSystem.assembly() / .solve()) ------------------------
 * Assemble K and the ghost-constant vector c of K P = -mu*f + c, from the
 * POTENTIAL boundary conditions (rows without the 1/mu_i factor, sign
 * flipped so that the diagonal is positive).  E_STATE for a mesh
 * preprocessed with no_matrix.  Drops captured graphs.  Asynchronous.      */
int mifvm_poisson_assemble(mifvm_state* st, void* stream);
/* d_y = K d_x, both user order.                                            */
int mifvm_poisson_apply(mifvm_state* st, const double* d_x, double* d_y, void* stream);
/* d_y = K d_x evaluated from the discretisation, without the stored matrix
 * (eqs. (7), (laplace): Algorithm 2 vertex values with homogeneous ghosts,
 * the diamond flux on interior and Dirichlet faces, the sum over each
 * cell's faces), user order; equal to mifvm_poisson_apply up to rounding.
 * Needs only the POTENTIAL boundary kinds (no assembly).                  */
int mifvm_poisson_apply_free(mifvm_state* st, const double* d_x, double* d_y, void* stream);
/* d_b = -mu * d_f + c (user order; d_f NULL = the current U); c is
 * computed first if the POTENTIAL BCs changed since it last was.           */
int mifvm_poisson_rhs(mifvm_state* st, const double* d_f, double* d_b, void* stream);
/* Jacobi-preconditioned CG on K x = b with b from d_f (NULL = current U);
 * starts from the stored P (zero after create, the last solution after a
 * solve: warm start) and stores the result back in P.  Converged when the
 * recomputed FP64 true residual ||b - K x||_2 <= tol ||b||_2.  opts NULL =
 * tol 1e-10, maxit 20000, chunk 32, restart 500.  A restart
 * recomputes r = b - K x and sets p = D^-1 r.  With method IR_FP32,
 * `iterations` counts FP32 inner iterations and every outer step restarts
 * the inner CG.  On a batch every mesh runs its own CG (own scalars and
 * stopping test); info reports the largest iteration count and residual.
 * Returns NOT_CONVERGED at maxit.  Every method but a matrix_free one
 * (and AMG, whose hierarchy is built from K) needs an assembled system:
 * E_STATE otherwise.
 * Synchronises (once per chunk).                                           */
int mifvm_poisson_solve(mifvm_state* st, const double* d_f, const mifvm_solve_opts* opts,
                        mifvm_solve_info* info, void* stream);

/* FGMRES workspace: (2m + 1) vectors of nc doubles and O(m^2) scalars, in a
 * caller-owned 256-byte-aligned device buffer that must outlive its use.
 * 1 <= m <= 64.  attach with d_ws NULL detaches.  E_ARG for a batch.       */
int mifvm_fgmres_bytes(const mifvm_state* st, int32_t m, size_t* out);
int mifvm_fgmres_attach(mifvm_state* st, int32_t m, void* d_ws, size_t ws_bytes);

/* ---- captured replays and the autotuner -----------------------------------
 * mifvm_step_graph: as mifvm_step, but the n_steps x 3 stages are captured
 * once into a hipGraph (per (n_steps, dt, CFL factor of the last
 * mifvm_cfl_dt)) and replayed on `stream`; mifvm_set_bc and
 * mifvm_poisson_assemble drop every captured graph.
 * mifvm_autotune: times the CG schedule (chunk 8/16/32/64, direct launches
 * or graph replay) on short solves of the current system (f = U; P is
 * restored afterwards) and one step direct vs replayed (U restored); keeps
 * the fastest in the state (used by solves with chunk = 0 / graph = -1 and
 * by mifvm_step_graph) and records it in the JSON file cache_path (NULL: no
 * file) under "arch/nmeshes/log2(cells)".  Reads the file first: a recorded
 * entry is used without timing.  Synchronises.                              */
typedef struct {
    int32_t chunk;
    int32_t graph;
    int32_t step_graph;
    int32_t from_cache;
    double ms_per_iteration;   /* of the chosen CG schedule (0 if cached)     */
    double ms_per_step_direct;
    double ms_per_step_graph;
} mifvm_tune_info;
int mifvm_step_graph(mifvm_state* st, int32_t n_steps, double dt, void* stream);
int mifvm_autotune(mifvm_state* st, const char* cache_path, mifvm_tune_info* out, void* stream);

/* ---- batched form: persistent solve of many meshes ---------------------------
 * A batch is a state made of independent meshes (mifvm_mesh_opts.nmeshes;
 * one workspace, one internal numbering, every step kernel launched once
 * for all meshes).  mifvm_batch runs the meshes' Poisson solves - each its
 * own matrix-free Jacobi-CG with the stopping test, restarts and scalars of
 * mifvm_poisson_solve (matrix_free = 1) - in ONE persistent kernel: every
 * mesh's iteration is a sequence of phases (vertex values of Algorithm 2,
 * diamond face fluxes of eq. (diamond), the cell gather with p.q, the
 * update with r.z and r.r, the new direction; and the opening from the true
 * residual), each split into items of `item_rows` consecutive rows;
 * workgroups take (mesh, phase, item) from per-mesh device queues, the
 * workgroup that completes a phase's last item adds its partial sums in item
 * order (deterministic) and publishes the next phase, and a mesh that has
 * converged leaves the queue while the others go on.  A workgroup that sees
 * no progress of any mesh for about 2^20 polls stops the kernel (E_STATE),
 * so it cannot hang.  FP64 states only; no stored matrix needed.
 *
 * Schedule: item_rows (a multiple of 256: 256 threads, item_rows/256 rows per
 * thread; 0 = 4096), grid (workgroups; 0 = 1024), policy (the order in which
 * a workgroup looks for work: 0 ROTATE - meshes by size, rotated per XCD;
 * 1 XCD - meshes assigned to the 8 XCDs by size (longest processing time
 * first), an XCD's workgroups take their own meshes first so that a mesh's
 * data stays in one L2, then steal; 2 LARGEST - the largest mesh first
 * everywhere; 3 LAUNCHES - no persistent kernel: the state's per-launch
 * matrix-free CG, every launch covering all meshes, chunks of iterations
 * replayed from a captured graph and the host checking the meshes between
 * chunks (mifvm_batch_run then replays a step graph and these chunks per
 * step instead of one graph for the whole run); -1 = 1).                   */
typedef struct mifvm_batch mifvm_batch;
typedef struct {
    int32_t item_rows;
    int32_t grid;
    int32_t policy;
    int32_t spin_limit;        /* polls without progress before the kernel
                                  stops (0 = 2^20; for tests of that path)   */
    int32_t vertex_batch;      /* vertex-list entries gathered together per
                                  thread: 8 or 24 (0 = 8)                     */
    int32_t chunk;             /* LAUNCHES: CG iterations per replayed chunk
                                  (0 = 32)                                   */
} mifvm_batch_opts;

typedef struct {
    double tol;                /* relative true residual per mesh (0 = 1e-10)  */
    int32_t maxit;             /* per mesh and solve (0 = 20000)              */
    int32_t restart;           /* reopen from the true residual every this many
                                  iterations (0 = only at convergence)       */
    int32_t solve_every;       /* mifvm_batch_run: a solve after every this many
                                  steps (0 = 1)                              */
    int32_t pad_;
} mifvm_batch_solve_opts;

typedef struct {
    int32_t solves;            /* solves in the call                          */
    int32_t pad_;
    int64_t iterations_max;    /* per mesh, summed over the call's solves: the
                                  largest over the meshes                    */
    int64_t iterations_sum;    /* over meshes and solves                      */
    double iterations_mean;    /* per mesh                                    */
    double rel_residual_max;   /* largest final true relative residual        */
    double ms;                 /* wall time of the call                       */
} mifvm_batch_info;

typedef struct {
    int32_t item_rows, grid, policy;
    int32_t from_cache;
    int32_t trials;
    int32_t iterations;        /* iterations per mesh of each timed trial     */
    double ms_best;            /* the chosen schedule's trial                 */
    int32_t vertex_batch, chunk;
    double ms_persistent;      /* best persistent-kernel trial                */
    double ms_launches;        /* best per-launch trial                       */
    int32_t p_item_rows, p_grid, p_policy, p_vertex_batch;   /* that persistent schedule */
} mifvm_batch_tune_info;

/* Device workspace of a batch (queues, ranges, partial sums, schedule),
 * 256-byte aligned, caller-owned, outliving the batch.                      */
int mifvm_batch_bytes(const mifvm_state* st, size_t* out);
/* Bind a batch to a state.  E_ARG when two meshes share a vertex or a face,
 * or for a bad schedule; E_STATE for an FP32 state.  Synchronises.        */
int mifvm_batch_create(mifvm_state* st, const mifvm_batch_opts* opts, void* d_ws, size_t ws_bytes,
                       void* stream, mifvm_batch** out);
void mifvm_batch_destroy(mifvm_batch* b);
/* Change the schedule (fields <= 0, or -1 for the policy, keep theirs).    */
int mifvm_batch_set_schedule(mifvm_batch* b, const mifvm_batch_opts* opts, void* stream);
int mifvm_batch_get_schedule(const mifvm_batch* b, mifvm_batch_opts* out);
/* Every mesh's Poisson solve of Delta P = U (b = -mu U + c, warm-started
 * from P) in one persistent launch.  Per-mesh iterations and residuals go to
 * mifvm_mesh_values (2, 3).  NOT_CONVERGED if a mesh stopped at maxit.
 * Synchronises.                                                            */
int mifvm_batch_solve(mifvm_batch* b, const mifvm_batch_solve_opts* opts, mifvm_batch_info* info, void* stream);
/* n_steps of the batched configuration: each an RK3 step of every mesh at
 * its own CFL time step (mifvm_cfl_dt first), then, every solve_every steps,
 * the persistent solve - the whole sequence captured once into one hipGraph
 * (per n_steps and options; dropped with the state's graphs) and replayed.
 * info sums the run's solves.  Synchronises.                               */
int mifvm_batch_run(mifvm_batch* b, int32_t n_steps, const mifvm_batch_solve_opts* opts, mifvm_batch_info* info,
                    void* stream);
/* Time `iterations` (0 = 24) iterations of every mesh for queue policy x
 * grid {512, 1024, 2048} at 4096-row items, then item_rows {1024 .. 65536}
 * and vertex_batch {8, 24} at the best, then LAUNCHES with chunk {16, 32,
 * 64}; keep the fastest and record it in the JSON file cache_path (NULL:
 * none) under "gfx950/batch/<meshes>/<log2 cells>"; a recorded entry is used
 * without timing.  ms_persistent / ms_launches: the best trial of each kind.
 * P is restored.  Synchronises.                                           */
int mifvm_batch_autotune(mifvm_batch* b, const char* cache_path, int32_t iterations, mifvm_batch_tune_info* out,
                         void* stream);

/* ---- aggregation multigrid preconditioner ----------------------------------
 * The analogue of the paper's fastest solver configuration (PETSc GAMG,
 * Sec. 3.4.2), as plain aggregation: per level, strong neighbours
 * |a_ij| >= theta max_{k != i} |a_ik|; aggregates in three passes in row
 * order (a row with all strong neighbours free seeds an aggregate with them;
 * a free row joins the aggregate of its strongest aggregated strong
 * neighbour, the smallest index on ties; a row still free seeds one with
 * its free strong neighbours); A_c = P^T A P with the piecewise-constant P;
 * until at most coarse_max rows, inverted densely (LU, partial pivoting).
 * The cycle: x = w D^-1 b; b_c = P^T (b - A x); x += P V(b_c);
 * x += w D^-1 (b - A x); the dense inverse on the coarsest level.  With
 * cycle = 2 (W) the coarse correction of every level whose coarser level is
 * not the dense one is improved once more before it is prolonged:
 * x_c = V(b_c); x_c += V(b_c - A_c x_c).                                  */
typedef struct {
    double theta;              /* 0 = 0.25                                    */
    double omega;              /* Jacobi damping, 0 = 2/3                     */
    int32_t max_levels;        /* 0 = 10 (at most 16)                         */
    int32_t coarse_max;        /* 0 = 1024 (at most 4096)                     */
    int32_t cycle;             /* 0 or 1 = V-cycle, 2 = W-cycle; else E_ARG   */
    int32_t pad_;
} mifvm_amg_opts;

typedef struct {
    int32_t levels;
    int32_t pad_;
    int64_t rows[16];
    int64_t nnz[16];           /* stored entries, diagonal included           */
    double setup_ms;           /* mifvm_amg_build: host setup incl. the copy of K */
    size_t ws_bytes;           /* device workspace for mifvm_amg_attach        */
} mifvm_amg_info;

/* Build the hierarchy of the state's assembled K on the host (copies K from
 * the device; synchronises).  E_ARG for a batch or bad options or when the
 * coarsening stalls; E_STATE without an assembled system.  Replaces an
 * earlier hierarchy and detaches it.                                       */
int mifvm_amg_build(mifvm_state* st, const mifvm_amg_opts* opts, mifvm_amg_info* info, void* stream);
/* Upload the built hierarchy into a caller workspace of info.ws_bytes
 * (256-byte aligned, outliving the attachment; E_WORKSPACE otherwise);
 * d_ws NULL detaches.  Synchronises.                                       */
int mifvm_amg_attach(mifvm_state* st, void* d_ws, size_t ws_bytes, void* stream);
/* d_z = V(d_r), one cycle, user cell order (for inspection and tests);
 * learned_smoother as in mifvm_solve_opts.  Uses the solver's r and z
 * vectors as scratch.                                                     */
int mifvm_amg_apply(mifvm_state* st, int32_t learned_smoother, const double* d_r, double* d_z, void* stream);
/* The same setup for any square CSR matrix (host arrays, diagonal included,
 * any column order), without a GPU, for inspection and tests.             */
typedef struct mifvm_amg_host mifvm_amg_host;
int mifvm_amg_host_build(int64_t n, const int64_t* ptr, const int32_t* col, const double* val,
                         const mifvm_amg_opts* opts, mifvm_amg_host** out);
int mifvm_amg_host_info(const mifvm_amg_host* h, mifvm_amg_info* info);
/* what: 0 AGG int32 [rows] (not on the coarsest level), 1 PTR int64
 * [rows+1], 2 COL int32 [nnz], 3 VAL f64 [nnz] of the level's matrix
 * (columns ascending on coarse levels; level 0 as given), 4 the coarsest
 * level's dense inverse f64 [rows*rows], row-major.  bytes must match.    */
int mifvm_amg_host_export(const mifvm_amg_host* h, int32_t level, int32_t what, void* dst, size_t bytes);
void mifvm_amg_host_destroy(mifvm_amg_host* h);

/* ---- coupled streamer-type loop (Sec. 4, eq. (10)) -------------------------
 * One species in drift-diffusion coupled to the electrostatic potential:
 *     d n_e/dt + div(n_e v_e) - div(D grad n_e) = S_e,   d n_p/dt = S_e,
 *     Delta P = kappa (n_e - n_p),   E = -grad P,
 *     v_e = -mu E,   S_e = alpha(|E|) |v_e| n_e,   alpha(|E|) = a exp(-b/|E|).
 * n_e is FIELD_U with the SCALAR boundary conditions and the state's
 * diffusivity D; P is FIELD_P with the POTENTIAL boundary conditions (the
 * system must be assembled); n_p is FIELD_ION.  The paper's C1, C2 and its
 * ionisation fit are not usable as printed, so the mobility is a constant
 * and alpha a Townsend-type law with caller constants (a = 0: no source).
 * Each step: P from the Poisson solve (warm-started from the last P; PLAIN
 * or, with matrix_free, on the matrix-free product), E = -grad P by the
 * least-squares gradient of Algorithm 1 (ghosts from the POTENTIAL
 * conditions), v_e and S_e per cell, the face velocities (as FIELD_VEL
 * does), dt = cfl times each mesh's CFL bound, one RK3 step of n_e with S_e
 * held over the step, and n_p += dt S_e.  FP64 states only (E_STATE for
 * FP32).  A solve that does not converge ends the call with its status.  */
typedef struct {
    double mobility;           /* mu (>= 0)                                   */
    double charge_scale;       /* kappa (e / epsilon)                         */
    double alpha_a, alpha_b;   /* ionisation law constants (>= 0)             */
    double cfl;                /* > 0                                         */
    double tol;                /* Poisson tolerance (0 = 1e-10)               */
    int32_t maxit;             /* per solve (0 = 20000)                       */
    int32_t restart;           /* as mifvm_solve_opts (0 = 500)               */
    int32_t matrix_free;
    int32_t pad_;
} mifvm_streamer_opts;

typedef struct {
    int32_t steps;             /* steps taken                                 */
    int32_t iterations_max;    /* largest CG iteration count of a step        */
    int64_t iterations_sum;
    double time;               /* sum of the steps' dt (the smallest over the
                                  meshes of a batch)                         */
    double last_dt;
} mifvm_streamer_info;

int mifvm_streamer_step(mifvm_state* st, int32_t n_steps, const mifvm_streamer_opts* opts,
                        mifvm_streamer_info* info, void* stream);

/* ---- without allocation ------------------------------------------------------
 * For callers that cannot allocate device or host memory while they run
 * (code under graph capture, tight serving loops, harnesses that forbid
 * it): the total of mifvm_conservation, bitwise the same, with its
 * reduction scratch (per-block partials, per-mesh totals, the result) in a
 * fixed array of MIFVM_STATIC_SCRATCH_BYTES that the library holds on each
 * GPU it runs on until the process ends, instead of the state's workspace
 * and host mirror.  The call allocates nothing.  At most
 * MIFVM_STATIC_MAX_MESHES meshes (E_ARG beyond).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other threads,
 * other streams) race and must be serialised by the caller.  Synchronises.  */
#define MIFVM_STATIC_MAX_MESHES 1024
#define MIFVM_STATIC_SCRATCH_BYTES ((1024 + MIFVM_STATIC_MAX_MESHES * 32 + 8) * 8)
int mifvm_conservation_static(mifvm_state* st, double* total_out, void* stream);

/* ---- per-kernel timing (HIP events on the launch stream) -----------------
 * enable != 0 starts recording an event pair around every kernel launch of
 * this state and clears the totals; enable == 0 stops.  Kernel ids: */
enum mifvm_kernel {
    MIFVM_K_GHOST_FILL = 0, MIFVM_K_GRAD_LIMITER = 1 /* incl. vertex values */,
    MIFVM_K_NODE_INTERP = 2 /* reserved: computed inside GRAD_LIMITER, never launched */,
    MIFVM_K_FACE_FLUX = 3 /* face fluxes of the residual evaluation */,
    MIFVM_K_UPDATE = 4 /* reserved: the update is part of FV_CELL, never launched */,
    MIFVM_K_CG_SETUP = 5, MIFVM_K_CG_SPMV = 6,
    MIFVM_K_CG_AXPY = 7, MIFVM_K_CG_DIR = 8, MIFVM_K_RHS = 9, MIFVM_K_ASSEMBLE = 10,
    MIFVM_K_NN_LAYER1 = 11, MIFVM_K_NN_LAYER2 = 12, MIFVM_K_NN_LAYER3 = 13 /* network layers
    (the first includes the encoder, the last the decoder) */,
    MIFVM_K_FCG_VEC = 14 /* flexible-CG update and its scalar steps */,
    MIFVM_K_NN_TRAIN = 15 /* one whole training step (all of its launches) */,
    MIFVM_K_MF_VERTEX = 16 /* matrix-free product inside the CG: the vertex values */,
    MIFVM_K_MF_FACE = 17 /* reserved: the face terms are summed per cell inside MF_GATHER,
    never launched */,
    MIFVM_K_MF_GATHER = 18 /* matrix-free product inside the CG: the per-cell product over
    the cell's vertices and faces, with p.q (CG_SPMV counts the stored-matrix product) */,
    MIFVM_K_NN_FUSED = 19 /* the whole network in one launch (encoder, 3 layers, decoder) */,
    MIFVM_K_CG_ALPHA = 20 /* the matrix-free CG's alpha step (its p.q partials summed per mesh) */,
    MIFVM_K_FV_CELL = 21 /* the step: face fluxes and the RK stage update in one pass per cell */,
    MIFVM_K_COUNT = 22
};
int mifvm_kernel_timing(mifvm_state* st, int32_t enable);
/* As mifvm_kernel_timing(st, 1), but only the launches of the kernels whose
 * bit (1 << id) is set in `kernels` get an event pair (and totals); the
 * others launch without events, so a timed run carries fewer event records.
 * With any bit set, solves launch their kernels directly instead of
 * replaying captured chunks (as with all kernels timed).  0 stops timing;
 * E_ARG for a bit at or above MIFVM_K_COUNT; E_STATE as mifvm_kernel_timing. */
int mifvm_kernel_timing_select(mifvm_state* st, uint64_t kernels);
/* Total milliseconds and number of timed launches of one kernel since the
 * last enable.  Synchronises the stream.                                    */
int mifvm_kernel_stats(mifvm_state* st, int32_t kernel, double* total_ms, int64_t* launches,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MIFVM_H */
