/*
 * mifvm_nn.h - learned preconditioner of the Poisson solve (C ABI).
 *
 * Not part of the paper's method: an added form of the solve of the system
 * of Sec. 2.2 (eqs. (7), (laplace)).  A message-passing network over the
 * cell-face graph (each tetrahedron's up to 4 face neighbours) maps a
 * residual r to a correction
 *
 *     x_i  = [r_i / s_r, (D^-1 r)_i / s_d]      s_r, s_d = RMS of r, D^-1 r
 *     h0_i = We x_i + be
 *     3 layers:  m_i = 1/4 sum_{j face neighbour of i} h_j
 *                u_i = relu(W1 [h_i; m_i] + b1),   h_i <- h_i + W2 u_i + b2
 *     y_i  = wd . h_i + bd,        z_i = (D^-1 r)_i + s_d y_i
 *
 * with D = diag(K) and hidden width 32 (MIFVM_NN_PARAMS parameters).  z is
 * 1-homogeneous in r; with wd = bd = 0 it is Jacobi.  Weights, h, m and u
 * are bfloat16 (round to nearest even) and feed bf16 matrix-core products
 * with FP32 accumulation; z is FP64.  mifvm_poisson_solve with method
 * MIFVM_SOLVE_LEARNED runs flexible CG with z as the preconditioner.
 *
 * Training minimises one of two losses per sample r with Adam (one sample
 * per step):
 *   RESIDUAL  L = ||r - K z||^2 / ||r||^2
 *   ENERGY    L = (z^T K z - 2 z^T r) / (r^T D^-1 r)
 * The energy functional is ||z - e||^2 in the norm of K_s = (K + K^T)/2,
 * e = K_s^-1 r, minus a constant: the norm conjugate gradients minimise; the
 * residual loss weights the error by K^2.  Both need K^T, whose values the
 * library builds in K's (symmetric) pattern.  The samples are true residuals
 * b - K x_k of iterates of the library's own solver (mifvm_nn_sample), i.e.
 * r = K e_k with e_k = x* - x_k.  The gradient is the chain rule of the
 * rounded forward with each rounding taken as the identity.
 *
 * Parameter order (FP32, as get/set/save): We[32][2], be[32], then for each
 * of the 3 layers W1[32][64] (columns: h then m), b1[32], W2[32][32],
 * b2[32], then wd[32], bd.  Conventions as in mifvm.h (status codes, "d_"
 * device pointers, streams, caller-owned 256-byte-aligned workspaces).
 */
#ifndef MIFVM_NN_H
#define MIFVM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "mifvm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MIFVM_NN_PARAMS 9537

enum mifvm_nn_loss { MIFVM_NN_LOSS_RESIDUAL = 0, MIFVM_NN_LOSS_ENERGY = 1 };

typedef struct mifvm_nn mifvm_nn;

typedef struct {
    uint64_t seed;             /* initial weights: N(0, init_scale^2 * 2/fan_in) */
    double init_scale;         /* 0 = 1; biases, wd and bd start at 0            */
} mifvm_nn_opts;

/* Device bytes of a network (parameters, Adam moments, operand copies,
 * per-block gradient sums).                                                */
size_t mifvm_nn_workspace_bytes(void);
/* Create a network in the caller's workspace (E_WORKSPACE if too small or
 * misaligned).  Synchronises.                                               */
int mifvm_nn_create(const mifvm_nn_opts* opts, void* d_ws, size_t ws_bytes, void* stream, mifvm_nn** out);
/* The network must outlive every state it is attached to.                  */
void mifvm_nn_destroy(mifvm_nn* nn);
/* FP32 parameters in the order above, n = MIFVM_NN_PARAMS (host arrays).
 * set: E_ARG on a non-finite value; resets the Adam moments and step count.
 * Synchronise.                                                              */
int mifvm_nn_get_params(const mifvm_nn* nn, float* out, int64_t n, void* stream);
int mifvm_nn_set_params(mifvm_nn* nn, const float* in, int64_t n, void* stream);
/* Serialised parameters: an 8-byte tag "MIFVMNN1", uint32 version (1),
 * uint32 count, then the FP32 parameters.  save with buf NULL sets *bytes to
 * the size; otherwise *bytes must be at least that size and receives it.
 * load: E_ARG on a wrong tag, version, count or size, or a non-finite value
 * (the network is left unchanged).  Synchronise.                           */
int mifvm_nn_save(const mifvm_nn* nn, void* buf, size_t* bytes, void* stream);
int mifvm_nn_load(mifvm_nn* nn, const void* buf, size_t bytes, void* stream);

/* Per-state buffers of an attached network: face neighbours, two (training:
 * three) bf16 activation rows per cell, flexible-CG vectors; for training
 * also FP32 backward rows and the values of K^T.                           */
int mifvm_nn_attach_bytes(const mifvm_state* st, int32_t training, size_t* out);
/* Attach nn to a single-mesh state (E_ARG for a batch); nn NULL detaches.
 * The workspace must outlive the attachment.  When the mesh has tiles for the
 * one-launch forward (below), attaching times one application of each form on
 * the given stream (the cell volumes as input) and keeps the faster; the
 * state's scratch vectors are overwritten.  Synchronises in that case.      */
int mifvm_nn_attach(mifvm_state* st, mifvm_nn* nn, int32_t training, void* d_ws, size_t ws_bytes,
                    void* stream);
/* d_z = z(d_r), both FP64 in user cell order (for inspection and tests), in
 * the form the state uses (mifvm_nn_form), as inside the flexible CG and the
 * multigrid smoother.  E_STATE without an attached network or an assembled
 * system (or, for matrix-free use, the diagonal of a solve).               */
int mifvm_nn_apply(mifvm_state* st, const double* d_r, double* d_z, void* stream);
/* The same network layer by layer: three launches with the activation rows
 * going through device memory (the form training uses).  Bitwise the same
 * z as the one-launch form.                                                */
int mifvm_nn_apply_layers(mifvm_state* st, const double* d_r, double* d_z, void* stream);
/* Forms of the forward.  LAYERS: three launches, rows through device memory.
 * FUSED: one launch per tile of consecutive cells; the encoding of the cells
 * within three face-neighbour steps of the tile kept in LDS and each layer
 * evaluated where the next reads it (so the rings are evaluated more than
 * once).  A mesh whose tiles exceed the fused kernel's LDS or register limits
 * has LAYERS only.  Both give bitwise the same z.                          */
#define MIFVM_NN_FORM_AUTO 0
#define MIFVM_NN_FORM_LAYERS 1
#define MIFVM_NN_FORM_FUSED 2
/* Select the form (AUTO: the faster of the attach-time timings; -1: leave
 * it) and report the one in use (*chosen, LAYERS or FUSED) and the timings
 * of one application of each (ms, 0 if not timed); outputs may be NULL.
 * E_STATE without an attached network or for FUSED without tiles; E_ARG for
 * an unknown form.  Drops captured chunks that launch the network.         */
int mifvm_nn_form(mifvm_state* st, int32_t form, int32_t* chosen, float* ms_layers, float* ms_fused);
/* A training sample from the state's current solve: the true residual
 * r = b - K x of the stored P against the right-hand side of the last solve
 * (or mifvm_poisson_rhs), scaled to unit RMS, written as FP32 in the
 * library's internal cell order (d_out: nc floats; opaque to the caller,
 * valid for this state).  *rms receives the RMS of r (0: d_out is 0).
 * Synchronises.                                                            */
int mifvm_nn_sample(mifvm_state* st, float* d_out, double* rms, void* stream);
/* Loss L of one sample (internal order, as from mifvm_nn_sample) and its
 * gradient (host, MIFVM_NN_PARAMS floats, parameter order), without an
 * update.  Needs a training attachment.  Synchronises.                    */
int mifvm_nn_loss_grad(mifvm_state* st, const float* d_sample, int32_t loss_kind, double* loss, float* grad,
                       void* stream);

typedef struct {
    int32_t epochs;
    int32_t loss;              /* enum mifvm_nn_loss                          */
    uint64_t seed;             /* order of the samples in each epoch          */
    double lr;                 /* Adam step, cosine-decayed to lr_min         */
    double lr_min;
    double beta1, beta2, eps;  /* 0 = 0.9, 0.999, 1e-8                        */
} mifvm_train_opts;

typedef struct {
    int64_t steps;
    double loss_first;         /* mean loss over the first epoch              */
    double loss_last;          /* mean loss over the last epoch               */
    double ms;
} mifvm_train_info;

/* Train on n_samples samples; sample k is d_samples[k] from
 * states[state_of_sample[k]], each state attached to nn for training with
 * its system assembled.  One Adam step per sample, in a seeded random order
 * each epoch.  epoch_loss (host, optional, epochs entries) receives each
 * epoch's mean loss.  Synchronises once per epoch.                         */
int mifvm_nn_train(mifvm_nn* nn, mifvm_state* const* states, int32_t n_states, const float* const* d_samples,
                   const int32_t* state_of_sample, int32_t n_samples, const mifvm_train_opts* opts,
                   mifvm_train_info* info, double* epoch_loss, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MIFVM_NN_H */
