// Message-passing network used as a learned preconditioner for the Poisson
// solve (not part of the paper's method; an added form of the solver).
//
//   x_i  = [r_i / s_r, (D^-1 r)_i / s_d]          s_r, s_d: RMS of r, D^-1 r
//   h0_i = We x_i + be
//   3 x: m_i = 1/4 sum_{j face neighbour of i} h_j
//        u_i = relu(W1 [h_i; m_i] + b1),  h_i <- h_i + W2 u_i + b2
//   y_i  = wd . h_i + bd,   z_i = (D^-1 r)_i + s_d y_i
//
// Hidden width 32.  Weights, h, m and u are bfloat16 (matrix-core operands),
// accumulation FP32, z FP64.  Parameters are kept in FP32 (master copy) in
// the order We[32][2], be, then per layer W1[32][64], b1, W2[32][32], b2,
// then wd, bd.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "state.h"

namespace mifvm {

constexpr int kNnH = 32;
constexpr int kNnLayers = 3;
constexpr int kNnLayerSize = 32 * 64 + 32 + 32 * 32 + 32;   // 3136
constexpr int kNnOffWe = 0, kNnOffBe = 64, kNnOffLayer = 96;
constexpr int kNnW1 = 0, kNnB1 = 2048, kNnW2 = 2080, kNnB2 = 3104;  // within a layer
constexpr int kNnOffWd = kNnOffLayer + kNnLayers * kNnLayerSize;    // 9504
constexpr int kNnOffBd = kNnOffWd + 32;
constexpr int kNnParams = kNnOffBd + 1;                             // 9537
constexpr int kNnGridMax = 1024;          // blocks of the weight-gradient kernels
constexpr int kNnGradChunks = 32;         // first stage of the block-gradient sum

// Storage order of a 32-feature row (h, and the per-cell backward rows):
// slot q = 8g + j holds feature pi(q) = 4g + j (j < 4) or 16 + 4g + j - 4.
// Lane group g (lanes 16g..16g+15) of a wave owns slots 8g..8g+7, which are
// exactly the features a 16x16 matrix-core result tile leaves in its lanes
// (rows 4g..4g+3 of both 16-row tiles), so every row is loaded and stored as
// one 16-byte vector per lane.
__host__ __device__ inline int nn_pi(int q) {
    const int g = q >> 3, j = q & 7;
    return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Weights rearranged as matrix-core A operands (one 16-byte fragment per
// lane) and per-slot vectors; rebuilt from the master copy after every update.
struct NnPackLayer {
    bf16x8 w1[2][2][64];    // W1 rows 16t.., k = 32s + pi(8g + j)
    bf16x8 w2[2][64];       // W2 rows 16t.., k = pi(8g + j)
    bf16x8 w2t[2][64];      // W2^T: row = input feature 16t + lane%16, k = output pi(8g + j)
    bf16x8 w1t[4][64];      // W1^T: row = input 16t + lane%16 (0..63), k = output pi(8g + j)
    float b1[32], b2[32];   // slot order
};
struct NnPack {
    float we0[32], we1[32], be[32];   // bf16-rounded encoder columns, slot order
    float wd[32];                     // slot order (FP32, not rounded)
    float bd, pad_[63];
    NnPackLayer layer[kNnLayers];
};

// Device memory of one network (carved from the caller's workspace).
struct NnDev {
    float* params;          // [kNnParams] FP32 master copy
    float* grad;            // [kNnParams]
    float* adam_m;          // [kNnParams]
    float* adam_v;          // [kNnParams]
    NnPack* pack;
    float* partial;         // [kNnGridMax][kNnParams] per-block gradient sums
    float* partial2;        // [kNnGradChunks][kNnParams] their sums by chunk
    double* loss;           // [kNnLossRing] loss of each training step
};
constexpr int kNnLossRing = 65536;

// Tiles of the fused forward: tile t holds `tile_rows` consecutive cells
// (ring 0) and the cells within three face-neighbour steps of them (rings
// 1-3), each ring in ascending cell order; the face neighbours of rings 0-2
// as indices into the tile's list (0xFFFF: a boundary face).  Three layers
// of the network at the tile's own cells read the first layer's output on
// rings 0-2, which reads the encoding on rings 0-3.
struct NnTiles {
    int32_t tile_rows = 0;
    int32_t ext_max = 0;              // most cells of one tile's list
    int32_t r2_max = 0;               // most cells of rings 0-2 of one tile
    int64_t ntiles = 0;
    std::vector<int64_t> ext_off;     // [ntiles + 1]
    std::vector<int32_t> ring;        // [ntiles][4] cumulative ring sizes
    std::vector<int32_t> cell;        // the lists
    std::vector<int64_t> nb_off;      // [ntiles + 1]
    std::vector<uint16_t> nb;         // [entries of rings 0-2][4]
};
constexpr int kNnFusedMaxGroups = 16;           // 16-cell groups per wave and layer (registers)
constexpr int kNnFusedWaves = 4;
constexpr int kNnFusedEntriesPerThread = 5;    // list entries per thread (256 threads) in the prologue
constexpr size_t kNnFusedLdsMax = 78 * 1024;    // two workgroups per CU
// the tiles of a mesh (largest tile size <= 256 that fits the limits;
// computed once per mesh and kept with it); null if none fits
const NnTiles* nn_tiles(const Mesh& m);
inline size_t nn_fused_lds(const NnTiles& t) { return size_t(t.ext_max) * 64 + size_t(t.r2_max) * 8; }

// Per-state buffers of an attached network.
struct NnStateDev {
    int4* nbr;              // [nc] face neighbours (internal numbering, -1: none)
    u32x4* h1;              // [nc][4] bf16 rows (16-byte chunks)
    u32x4* h2;
    u32x4* h3;              // training only
    double* r_old;          // [nc] previous residual (flexible CG)
    double* x_bak;          // [nc] iterate saved at the last good check
    float* base;            // [nc][32] training: dh + dh through the self half
    float* dam0;            // [nc][32] training: gradient reaching m (ping)
    float* dam1;            //                                        (pong)
    double* kt_val;         // [matrix_padded] values of K^T in K's pattern
    int32_t* flag;          // [1] pattern check of the transpose (0 = ok)
    bool training;
    // fused forward (null tables: the three-launch forward is used)
    const NnTiles* tiles = nullptr;
    int64_t* t_ext_off;
    int4* t_ring;
    int32_t* t_cell;
    int64_t* t_nb_off;
    ushort4* t_nb;
    double* t_partial;      // [2][ntiles] z.r, z.r_old per tile
    // the form in use (both give bitwise the same z): fused when the tiles
    // exist and it was chosen; the attach-time timings of one application
    bool fused = false;
    float ms_layers = 0.f, ms_fused = 0.f;
};

size_t nn_layout(char* base, NnDev& n);
size_t nn_state_layout(const Mesh& m, bool training, char* base, NnStateDev& a);

// launchers (nn_kernels.hip)
hipError_t launch_nn_pack(const NnDev& n, hipStream_t s);
hipError_t launch_nn_neighbours(const Dev& d, const NnStateDev& a, hipStream_t s);
hipError_t launch_nn_transpose(const Dev& d, const NnStateDev& a, hipStream_t s);
// RMS scales of r (r64 or r32 is the input) into the mesh-0 scalar slots
hipError_t launch_nn_scale(const Dev& d, const double* r64, const float* r32, hipStream_t s);
// one forward layer (0, 1, 2); the last writes z (FP64).  fcg: skipped once
// the solve is done, and the last layer writes partial z.r and z.r_old.
// keep_h3: the last layer also stores its rows (training).
hipError_t launch_nn_layer(const Dev& d, const NnDev& n, const NnStateDev& a, int layer, const double* r64,
                           const float* r32, double* z, bool keep_h3, bool fcg, hipStream_t s);
int nn_forward_grid(int64_t nc);
// the whole forward in one launch on the state's tiles (z from r64); fcg:
// skipped once the solve is done, per-tile partial z.r and z.r_old
hipError_t launch_nn_fused(const Dev& d, const NnDev& n, const NnStateDev& a, const double* r64, double* z,
                           bool fcg, hipStream_t s);
// kernel attribute for dynamic LDS above 64 KB (once per tile set)
hipError_t setup_nn_fused(size_t lds);
// partial sums the forward leaves for the flexible CG's z.r and z.r_old
int64_t nn_forward_parts(const Dev& d, const NnStateDev& a);
int nn_backward_grid(int64_t nc);
// training, after the forward on r32 (z in d.z): the loss (kind 0 residual,
// 1 energy) into *loss_slot, its gradient w.r.t. z, the backward and the
// per-block parameter gradients
hipError_t launch_nn_backward(const Dev& d, const NnDev& n, const NnStateDev& a, const float* r32, int kind,
                              double* loss_slot, hipStream_t s);
// gradient = sum of the per-block sums (nblocks); apply: one Adam update
// (c1 = 1/(1-beta1^t), c2 = 1/sqrt(1-beta2^t)) and a repack of the operands
hipError_t launch_nn_adam(const NnDev& n, int nblocks, int apply, float lr, float c1, float c2, float beta1,
                          float beta2, float eps, hipStream_t s);
// r = b - K x, its scales, out = r / s_r in FP32 (a training sample)
hipError_t launch_nn_sample(const Dev& d, float* out, hipStream_t s);
// flexible CG steps
// kx: K x computed matrix-free by the caller, or null for the stored K
hipError_t launch_fcg_setup(const Dev& d, double tol, int maxit, int restart, bool fresh, hipStream_t s,
                            const double* kx = nullptr);
hipError_t launch_fcg_setup_tail(const Dev& d, const NnStateDev& a, hipStream_t s);
hipError_t launch_fcg_axpy(const Dev& d, const NnStateDev& a, hipStream_t s);
hipError_t launch_fcg_beta(const Dev& d, const NnStateDev& a, hipStream_t s);
hipError_t launch_fcg_backup(const Dev& d, const NnStateDev& a, bool restore, hipStream_t s);

}  // namespace mifvm
