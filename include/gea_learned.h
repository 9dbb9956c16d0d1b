/*
 * gea_learned.h -- C ABI of the small convolutional network that supplies
 * the learned initial guess and preconditioner of the pressure solve
 * (GEA_LEARNED_MIXED in gea.h).  The pressure equation it serves is the SPD
 * system of Step 3 (GEA, arXiv:2303.10499, Sec. 3, eq. p_prime_sd re-derived,
 * see gea.h); the network itself is not from the paper.
 *
 * Network: 3-level encoder-decoder with skip concatenation, channels
 * 16/32/64, 3x3 (2D) or 3x3x3 (3D) zero-padded convolutions, ReLU, 2x
 * average pooling, 2x nearest upsampling:
 *     e0 = relu(conv(x, W0, b0))            2 -> 16   full resolution
 *     e1 = relu(conv(pool(e0), W1, b1))    16 -> 32   1/2
 *     e2 = relu(conv(pool(e1), W2, b2))    32 -> 64   1/4
 *     d1 = relu(conv([up(e2), e1], W3, b3)) 96 -> 32  1/2
 *     d0 = relu(conv([up(d1), e0], W4, b4)) 48 -> 16  full
 *     y  =       conv(d0, W5, b5)           16 -> 1   full
 * Input channels: the scaled residual r/s (s = max |r|) and c/diag, the
 * operator's mass coefficient relative to its diagonal.  Output: the
 * scaled correction, so that x0 + s*y approximates A^{-1} b.
 *
 * Arithmetic: weights and activations in bfloat16 (round to nearest even),
 * products on the matrix cores (v_mfma bf16, FP32 accumulation), FP32
 * gradients, FP32 master weights with Adam.
 *
 * Layout: tensors are channels-last over the cells in mesh order (index
 * i + nx*(j + ny*k)).  Packed parameters (FP32): for each layer 0..5 in
 * order, W[c_out][tap][c_in] then b[c_out]; tap t enumerates the offsets
 * (dz, dx) (2D) or (dz, dy, dx) (3D) over {-1, 0, 1} lexicographically, and
 * output cell p reads input cell p + offset (zero outside the mesh).
 * Every dimension must be a positive multiple of 4.  Memory: the caller
 * owns all arrays and the workspace; errors as in gea.h.
 */
#ifndef GEA_LEARNED_H
#define GEA_LEARNED_H
#include "gea.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gea_cnn gea_cnn;

/* Number of packed FP32 parameters of the 2D (ndim = 2) or 3D network. */
gea_status gea_cnn_param_count(int32_t ndim, int64_t* count);

/* Device workspace for a network instance on an nx x ny x nz grid (ny = 1
 * in 2D); train = 1 adds the buffers of the backward pass and Adam. */
gea_status gea_cnn_workspace_bytes(int32_t ndim, int32_t nx, int32_t ny, int32_t nz,
                                   int32_t train, size_t* bytes);

gea_status gea_cnn_create(int32_t ndim, int32_t nx, int32_t ny, int32_t nz, int32_t train,
                          void* hip_stream, void* workspace, size_t workspace_bytes,
                          gea_cnn** out);

/* Copy packed FP32 parameters in / out (in also resets Adam's moments). */
gea_status gea_cnn_set_params(gea_cnn* net, const float* params, gea_ptr_kind kind);
gea_status gea_cnn_get_params(gea_cnn* net, float* params, gea_ptr_kind kind);

/* y = net(x); x: npix x 2 FP32 (channels last), y: npix FP32.  Returns
 * after the work completed. */
gea_status gea_cnn_forward(gea_cnn* net, const float* x, float* y, gea_ptr_kind kind);

/* Gradient of L = sum (y - t)^2 / (2 npix) for the last forward pass
 * (train instances only); accumulate = 1 adds to the stored gradient.
 * loss (nullable) receives L. */
gea_status gea_cnn_backward(gea_cnn* net, const float* target, gea_ptr_kind kind,
                            int32_t accumulate, double* loss);

/* Packed FP32 gradient (same layout as the parameters). */
gea_status gea_cnn_get_grads(gea_cnn* net, float* grads, gea_ptr_kind kind);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the stored gradient
 * scaled by grad_scale; step counts from 1. */
gea_status gea_cnn_adam(gea_cnn* net, float lr, float grad_scale, int32_t step);

/* Test support: an activation of the last forward pass as FP32, channels
 * last: which = 0 input (8 channels, 2 used), 1 e0, 2 pool(e0), 3 e1,
 * 4 pool(e1), 5 e2, 6 [up(e2), e1], 7 d1, 8 [up(d1), e0], 9 d0, 10 y.
 * Inference instances (train = 0) keep neither the padded input nor the
 * concatenations: which = 0, 6 and 8 return GEA_ERR_STATE there. */
gea_status gea_cnn_activation(gea_cnn* net, int32_t which, float* out, gea_ptr_kind kind);

void gea_cnn_destroy(gea_cnn* net);

/* Learned solver: give a solver context the network weights (packed FP32,
 * the network of the context's dimension).  Required before a step or solve
 * with GEA_LEARNED_MIXED; the mesh dimensions must be multiples of 4. */
gea_status gea_load_weights(gea_ctx* ctx, const float* params, gea_ptr_kind kind);

/* Training pair from the current state (Sec. 3, Step 3): assemble the
 * first-corrector pressure system, r0 = b - A p', solve A x = b to rel_tol
 * with FP64 Jacobi-PCG, delta = x - p'; s = max |r0|.  Outputs (npix each,
 * FP32): in_r = r0/s, in_a = c/diag, out_d = delta/s; *scale = s. */
gea_status gea_make_pair(gea_ctx* ctx, double rel_tol, float* in_r, float* in_a, float* out_d,
                         double* scale, gea_ptr_kind kind);

/* Test support: the learned solver's network application exactly as its
 * flexible CG makes it, on the pressure system of the context's last
 * assembly (gea_pressure_solve or a step): r is an FP32 residual of npix
 * values; the library forms s = max |r| (*scale, host) and
 * z = s * net(r/s, c/diag) (npix FP32 values) with the loaded weights.
 * GEA_ERR_STATE without weights or an assembled system.  Overwrites the
 * solver's inner FP32 work vectors. */
gea_status gea_learned_apply(gea_ctx* ctx, const float* r, float* z, double* scale,
                             gea_ptr_kind kind);

/* Test support: an activation of the context's network after its last
 * application, as gea_cnn_activation (which = 1..9); which = 0 gives the two
 * input channels (r/s, c/diag) per cell; the output y is not kept. */
gea_status gea_learned_activation(gea_ctx* ctx, int32_t which, float* out, gea_ptr_kind kind);

#ifdef __cplusplus
}
#endif
#endif
