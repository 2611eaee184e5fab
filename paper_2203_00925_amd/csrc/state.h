// Device-resident state: the preprocessed mesh and every field, carved out
// of one caller-owned workspace.  Shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "mesh.h"

namespace mifvm {

constexpr int kMaxTags = 32;
constexpr int kBlock = 256;               // threads per block (4 wavefronts)
constexpr int kZeroFlux = 0, kNeumann = 1, kDirichlet = 2;

// Boundary conditions of one variable: the kind per tag (captured by value
// in launches and graphs) and the value per ghost (device memory, read when
// a kernel runs, so a graph replay sees values set after its capture).
struct BcTable {
    int32_t kind[kMaxTags];
    const double* val;                    // [nb] value at each ghost's face
    const float* val32;                   // [nb] FP32 copy (scalar variable only; else null)
};

// the value of ghost g in the precision of the kernel reading it
template <class R> __device__ inline R bc_value(const BcTable& bc, int64_t g);
template <> __device__ inline double bc_value<double>(const BcTable& bc, int64_t g) { return bc.val[g]; }
template <> __device__ inline float bc_value<float>(const BcTable& bc, int64_t g) { return bc.val32[g]; }

// Pointers into the workspace.  Layout: SoA, float64 unless noted, every
// array 256-byte aligned.
struct Dev {
    int64_t nc, nv, nf, nfi, nb;
    int32_t nm;                           // independent meshes (batch size)
    int64_t* mesh_start;                  // nm+1 internal cell offsets
    double* mesh_D;                       // nm diffusivities
    double* mesh_dt;                      // nm time steps
    int64_t ns, nvs;                      // 64-row slices of cells / vertices
    // cells
    double *vol, *xc;                     // xc: 3 x (nc+nb)
    double4* xyz4;                        // nc+nb centres as (x, y, z, 0) records
    double4* fx4;                         // nf face centroids as (x, y, z, 0) records
    double* minv;                         // 6 x nc
    int32_t *c2f, *c2n;                   // 4 x nc
    int64_t* s_off; int32_t* s_w; int32_t* s_idx;
    // faces
    int32_t *fL, *fR, *fA, *fB, *fC;
    double *kAC, *kBC, *kRL, *fx, *S, *area;   // fx, S: 3 x nf
    // ghosts
    int32_t *gowner, *gtag; double* gdist;
    int32_t* gbtri;                       // ghost -> caller's boundary triangle
    double* gval;                         // 2 x nb boundary values (SCALAR, POTENTIAL) per ghost
    float* gval32;                        // nb: the scalar's values in FP32
    // vertices
    int64_t* n_off; int32_t* n_w; int32_t* n_idx; double* n_alpha;
    int32_t* n_len;                       // nv vertex list lengths
    // Poisson pattern and values
    int64_t* k_off; int32_t* k_w; int32_t* k_col; int32_t* k_len;
    double *k_val, *k_diag, *k_dinv, *k_c;
    float *k_val32, *k_diag32, *k_dinv32;  // FP32 copy for the refined solve
    float *d32, *r32, *z32, *p32, *q32;   // FP32 inner-CG vectors
    // LDS tiles: tile_rows consecutive cells and their halo
    int32_t tile_rows, halo_max;
    int64_t ntiles;
    int64_t* h_off; int32_t* h_idx; int32_t* h_self;
    uint16_t *k_lidx, *c2n_l, *n_lidx;
    int64_t* v_off;
    // star-moment gradient: edge-only neighbours (64-row slices, local),
    // tile-local vertex numbers, the foreign vertices of each tile
    int32_t tv_max;
    int64_t* e_off; int32_t* e_w; uint16_t* e_lidx;
    uint16_t* c2v_l;
    int64_t* fv_off; int32_t* fv_len;
    int64_t* f_off; int32_t* f_w; uint16_t* f_lidx;
    // renumbering
    int32_t *cell_perm, *vert_perm;       // internal -> user
    // fields
    double *u, *src, *vel, *phi;     // u: nc+nb (ghosts behind), vel 3 x nc
    double *grad, *psi, *unode, *flux;    // grad 3 x nc
    // FP64 step (per cell): the MUSCL value at each of the cell's four face
    // centroids [4][nc] (gradient kernel -> cell step); the two stage buffers
    // of u (nc+nb each: a stage reads one and writes the other, u^n stays in u)
    double *uf, *u_b, *u_c;
    // per-cell tables of the FP64 step (geometry only): the cell's 4 vertex
    // ids, their diffusion weights and the kRL weights over its interior
    // faces ([4][nc] each), and per face k the slot of the same face among
    // the neighbour's faces (2 bits per face)
    int32_t* fvc_vid;
    double *fvc_w, *fvc_r;
    uint8_t* fvc_slot;
    double* fvc_phi;                      // [4][nc] outward phi of the cell's faces (with phi)
    // the same for the FP32 step: face values, stage buffers, weights, phi
    float *uf32, *u_b32, *u_c32, *fvc_w32, *fvc_r32, *fvc_phi32;
    // solver vectors (P lives in x)
    double *x, *r, *z, *p, *q, *b;
    // reduced-precision (FP32) form of the step
    float *u32, *src32, *phi32, *grad32, *psi32, *unode32, *flux32;
    float *minv32, *kAC32, *kBC32, *kRL32, *area32, *vol32, *n_alpha32, *fx32, *xc32, *gdist32;
    double* tmp;                          // nc+nb scratch (permutation, residual)
    double *np_ion, *efield;              // coupled loop: ion density [nc], E [3][nc]
    double* mf_xv;                        // matrix-free operator: vertex values [nv]
    // the vertex lists' entries for the matrix-free operator (same slots as
    // n_idx, n_entries of them): a cell reads itself, a ghost is folded onto
    // its owner, as ~owner where its homogeneous value is -x_owner (Dirichlet)
    int32_t* mf_nidx;
    int64_t n_entries;
    // matrix-free operator per cell i (from the faces and the potential's
    // boundary kinds): (K x)_i = -(sum_k w[k] x_v[vid[k]] + sum_k r[k] t_k) over
    // the cell's 4 vertices and 4 faces, t_k = x[c2n[k]] - x_i across an
    // interior face and x_i on a boundary face ([4][nc] each; FP32 copies)
    int32_t* mfc_vid;
    double *mfc_w, *mfc_r;
    float *mfc_w32, *mfc_r32;
    double* partial;                      // reduction partials ([k][block], k < 4)
    double* scal;                         // solver scalars, [nm][SC_COUNT_]
};

// The arrays one precision of the step reads and writes.
template <class R>
struct FvArrays {
    R *u, *grad, *psi, *unode, *flux;
    const R *phi, *minv, *kAC, *kBC, *kRL, *area, *vol, *src, *n_alpha, *fx, *xc, *gdist;
    // the per-cell stage: face values [4][nc], vertex and kRL weights, outward phi
    R* uf;
    const R *cw, *cr, *cphi;
};

constexpr int kNumKernels = 22;

struct NnDev;
struct NnStateDev;
struct GmDev;
struct AmgHierarchy;
struct AmgDev;

// Event pairs around kernel launches, resolved into totals at sync points.
struct KernelTimer {
    bool on = false;
    uint64_t mask = ~uint64_t(0);           // kernel ids that get an event pair while on
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<int, size_t>> pending;   // kernel id, index of start event
    double total_ms[kNumKernels] = {};
    int64_t count[kNumKernels] = {};
};

struct State {
    const Mesh* mesh = nullptr;           // host copy kept for sizes
    Dev d{};
    BcTable bc[2]{};                      // SCALAR, POTENTIAL
    double bc_tag_value[2][kMaxTags]{};   // the last per-tag value set (host record)
    double step_exec_cfl = -1.0;          // CFL factor captured in step_exec
    int64_t graph_gen = 0;                // bumped whenever the captured graphs are dropped
    double diffusivity = 0.0;
    bool fp32 = false;                    // reduced-precision form of the step
    double cfl = 0.0;                     // factor of the last CFL evaluation
    std::vector<int> last_iters;          // per mesh, last solve
    std::vector<double> last_rel;
    // captured launch sequences (hipGraph), replayed on the caller's stream
    hipStream_t cap_stream = nullptr;     // library-owned, used only to capture
    hipGraphExec_t cg_exec = nullptr;     // one chunk of CG iterations
    int cg_exec_chunk = 0, cg_exec_method = -1;
    hipGraphExec_t step_exec = nullptr;   // n RK3 steps
    int step_exec_n = 0;
    double step_exec_dt = -1.0;
    // schedule chosen by the autotuner (0 = not tuned)
    int tuned_chunk = 0, tuned_graph = 0, tuned_step_graph = 0;
    bool assembled = false;               // K's stored values, diagonal and c match the BCs
    bool consts_ready = false;            // diagonal, D^-1 and c match the BCs (matrix-free solves)
    bool mfc_ready = false;               // the matrix-free per-cell tables match the potential's BC kinds
    bool k32_ready = false;               // FP32 copy of K matches K
    bool vel_set = false;
    double* h_scal = nullptr;             // pinned host mirror of scalars
    int nblk_cells = 0;                   // grid for per-cell reductions
    KernelTimer timer;
    // attached learned preconditioner (the network is not owned; the
    // per-state buffers live in a caller workspace)
    const NnDev* nn = nullptr;
    const void* nn_handle = nullptr;
    NnStateDev* nn_state = nullptr;       // owned host record
    bool kt_ready = false;                // K^T values match K
    bool mf = false;                      // the running solve applies K matrix-free
    GmDev* gm = nullptr;                  // FGMRES workspace (owned host record)
    hipGraphExec_t gm_exec = nullptr;     // one captured FGMRES cycle
    int gm_exec_key = 0;
    bool b_ready = false;                 // d.b holds a right-hand side
    hipGraphExec_t fcg_exec = nullptr;    // one chunk of flexible-CG iterations
    int fcg_exec_chunk = 0;
    AmgHierarchy* amg_host = nullptr;     // multigrid hierarchy (host, owned)
    AmgDev* amg = nullptr;                // its device form (caller workspace; owned record)
    hipGraphExec_t amg_exec = nullptr;    // one chunk of multigrid-preconditioned iterations
    int amg_exec_key = 0;
};

// destroy every captured graph (their launch arguments hold boundary kinds,
// the CFL factor and chunk sizes by value); the next use captures again
void drop_graphs(State& s);
// value of every ghost of `tag` for variable var: `value`, or, when vals is
// not null, vals[caller's boundary triangle of the ghost]
hipError_t launch_set_bc_values(const Dev& d, int var, int tag, double value, const double* vals, hipStream_t s);

// workspace layout; returns total bytes (and fills d when base != nullptr)
size_t layout(const Mesh& m, char* base, Dev& d);

// launchers (fv_kernels.hip)
hipError_t launch_ghost_fill(const Dev& d, bool fp32, const BcTable& bc, hipStream_t s);
// parts: write the gradient and limiter arrays (the face kernel reads
// them); without parts, the per-face MUSCL values of the cell step instead,
// from u_in (the state's u in the step's precision if null)
hipError_t launch_grad_limiter(const Dev& d, bool fp32, hipStream_t s, bool parts = false,
                               const void* u_in = nullptr);
// once per state: kernel attributes (LDS above 64 KB for large tile halos)
hipError_t setup_fv_kernels(const Dev& d);
hipError_t launch_face_flux(const Dev& d, bool fp32, const BcTable& bc, hipStream_t s);
// RK stage in one pass per cell (face fluxes and update):
// u_out = u + alpha dt Res(u_in), with the ghosts behind the cells (u, u_in
// and u_out in the step's precision: double, or float with fp32)
hipError_t launch_cell_step(const Dev& d, bool fp32, const BcTable& bc, const void* u_in, void* u_out,
                            double alpha, hipStream_t s);
// once per state: the cell step's tables
hipError_t launch_fv_cell_setup(const Dev& d, hipStream_t s);
// the matrix-free per-cell tables (mf_kernels.hip)
hipError_t launch_mf_cell_setup(const Dev& d, const BcTable& bc_pot, hipStream_t s);
hipError_t launch_set_dt(const Dev& d, double dt, double cfl, hipStream_t s);
hipError_t launch_residual_out(const Dev& d, bool fp32, double* res_internal, hipStream_t s);
hipError_t launch_face_phi(const Dev& d, hipStream_t s);
hipError_t launch_make_fp32_geometry(const Dev& d, int64_t node_padded, hipStream_t s);
hipError_t launch_cast_to_f32(int64_t n, const double* src, float* dst, hipStream_t s);
hipError_t launch_cast_to_f64(int64_t n, const float* src, double* dst, hipStream_t s);
hipError_t launch_to_internal(const int32_t* perm, int64_t n, int64_t stride_in, int64_t stride_out,
                              int comps, const double* src, double* dst, hipStream_t s);
hipError_t launch_to_user(const int32_t* perm, int64_t n, int64_t stride_in, int64_t stride_out,
                          int comps, const double* src, double* dst, hipStream_t s);
// the same with the element type chosen per side (n rows, stride n)
hipError_t launch_to_internal_typed(const int32_t* perm, int64_t n, int comps, const void* src, bool src_f32,
                                    void* dst, bool dst_f32, hipStream_t s);
hipError_t launch_to_user_typed(const int32_t* perm, int64_t n, int comps, const void* src, bool src_f32,
                                void* dst, bool dst_f32, hipStream_t s);
hipError_t launch_cfl(const Dev& d, const Mesh& mh, const BcTable& bc, hipStream_t s);
hipError_t launch_conservation(const Dev& d, const Mesh& mh, bool fp32, hipStream_t s);

// launchers (solve_kernels.hip)
hipError_t launch_assemble(const Dev& d, const BcTable& bc, int row_max, hipStream_t s);
// the diagonal of K, D^-1 and the ghost constants c only (no stored matrix)
hipError_t launch_assemble_consts(const Dev& d, const BcTable& bc, hipStream_t s);
hipError_t launch_spmv_plain(const Dev& d, const double* x, double* y, hipStream_t s);
hipError_t launch_rhs(const Dev& d, const double* f_internal, hipStream_t s);
// kx: K x computed by the caller (matrix-free), or null for the stored K
hipError_t launch_cg_setup(const Dev& d, double tol, int maxit, int restart, bool fresh, hipStream_t s,
                           const double* kx = nullptr);
hipError_t launch_cg_spmv(const Dev& d, hipStream_t s);
hipError_t launch_cg_axpy(const Dev& d, hipStream_t s);
hipError_t launch_cg_dir(const Dev& d, hipStream_t s);

// launchers (mf_kernels.hip): y = K x from the discretisation (no stored matrix)
// skip: a device flag; the product is skipped when it is non-zero (nullptr: never)
hipError_t launch_mf_apply(const Dev& d, const BcTable& bc, const double* x, double* y, hipStream_t s,
                           const double* skip = nullptr);
hipError_t launch_mf_cg_spmv(const Dev& d, const BcTable& bc, hipStream_t s);
// the parts of launch_mf_cg_spmv one by one (part 0 ghost and vertex values,
// 1 the per-cell product + p.q partials, 2 alpha), for per-kernel timing
constexpr int kMfParts = 3;
hipError_t launch_mf_cg_part(const Dev& d, const BcTable& bc, int part, hipStream_t s);
// the same product in FP32 for the inner CG of the refined solve: q32 = K p32
// with the FP32 vertex weights and per-cell tables, partial p32.q32 in FP64
hipError_t launch_mf_cg32_spmv(const Dev& d, const BcTable& bc, hipStream_t s);
hipError_t launch_mf_cg32_part(const Dev& d, const BcTable& bc, int part, hipStream_t s);

// launchers (streamer_kernels.hip): the coupled loop's per-step kernels
hipError_t launch_streamer_rhs(const Dev& d, double kappa, double* f, hipStream_t s);
hipError_t launch_streamer_fields(const Dev& d, const BcTable& bc_pot, double mu, double a, double b,
                                  hipStream_t s);
hipError_t launch_ion_update(const Dev& d, hipStream_t s);
// sum_i mu_i (a_i - e_i)^2 over all cells (e null: 0) into scal[SC_NORM] of mesh 0
hipError_t launch_norm_l2(const Dev& d, const double* a, const double* e, hipStream_t s);

// launchers (ir_kernels.hip): FP32 inner CG inside FP64 iterative refinement
hipError_t launch_cast_matrix(const Dev& d, int64_t padded, hipStream_t s);
// kx: K x computed by the caller (matrix-free), or null for the stored K
hipError_t launch_ir_residual(const Dev& d, double tol, double tol_in, int maxit, int restart, bool fresh,
                              const double* kx, hipStream_t s);
hipError_t launch_cg32_spmv(const Dev& d, hipStream_t s);
hipError_t launch_cg32_axpy(const Dev& d, hipStream_t s);
hipError_t launch_cg32_dir(const Dev& d, hipStream_t s);
hipError_t launch_ir_update(const Dev& d, hipStream_t s);

// scalar slots in Dev::scal
enum Scal {
    SC_RZ = 0, SC_PQ, SC_ALPHA, SC_BETA, SC_RR, SC_BB, SC_TOL2BB, SC_DONE, SC_IT, SC_MAXIT,
    SC_TRUE_RR, SC_CONS, SC_DT_INV, SC_RESTART, SC_SINCE, SC_TOL2BB_OUT,
    // learned preconditioner: input scales and flexible-CG dot products
    SC_NN_INV_SR, SC_NN_INV_SD, SC_NN_SD, SC_NN_RR, SC_NN_DD, SC_ZR, SC_ZRO, SC_NN_RDR, SC_NN_DSCALE,
    SC_NORM,                              // mifvm_norm_l2 (mesh 0's slots)
    SC_COUNT_ = 32
};

}  // namespace mifvm
