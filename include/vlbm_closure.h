/*
 * vlbm_closure.h -- C ABI of the learned-closure network (gfx950, BF16 MFMA).
 *
 * A three-layer 3x3 convolutional network corrects the moments of a coarse
 * vLBM run (arXiv:2504.15574 solves the flow; the closure is an extension that
 * the paper does not contain).  Convolution taps that leave the grid continue
 * across a pole to phi + pi, the mapping the populations' ghost rows use
 * (Sec. III.E, eqs. (bcs_phi), (bcs_theta)); vector channels (the orthonormal
 * velocity components) change sign there.
 *
 * Conventions
 *  - A context fixes the grid n_theta x n_phi (n_theta >= 2; n_phi even and a
 *    multiple of 16) and the largest batch.  Tensors are NHWC: index
 *    ((b * n_theta + r) * n_phi + c) * C + ch; P = batch * n_theta * n_phi.
 *  - bf16 tensors are arrays of uint16 (IEEE bfloat16 bits); float tensors are
 *    FP32; field tensors are FP64 [batch][n_theta][n_phi].
 *  - Layer shapes: CIN in {8, 32} input channels, COUT in {16, 32} output
 *    channels (the 4 input and 3 output channels of the network are padded
 *    to 8 and 16 with zeros).  Weights in three layouts:
 *      master  FP32 [COUT][9 * CIN]      (k = tap * CIN + ci, tap = 3 (dy+1) + dx+1)
 *      w       bf16 [COUT][KP]           (KP = 9 * CIN rounded up to 32, zero padded)
 *      wt      bf16 [9][CIN][COUT]       (transposed, for the data gradient)
 *  - Every pointer is device memory; every call is asynchronous on the
 *    context's stream and validates only its arguments.  Returns a vlbm_status
 *    (include/vlbm.h); vlbm_last_error() holds the reason of a failure.
 */
#ifndef VLBM_CLOSURE_H
#define VLBM_CLOSURE_H

#include <stddef.h>
#include <stdint.h>

#include "vlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vlbm_clo vlbm_clo;

/* Device workspace bytes for a grid and batch (0 if invalid): stencil tables
 * and the partial sums of the weight gradients and of the loss. */
size_t vlbm_clo_workspace_bytes(int n_theta, int n_phi, int max_batch);

/* Create a context on the current device; builds the tap tables (for each cell
 * and tap the cell it reads and whether it crosses a pole; for each cell the
 * nine (cell, tap) pairs that read it) and uploads them, synchronising the
 * stream once.  Errors: VLBM_ERR_ARG, VLBM_ERR_ALLOC (workspace too small),
 * VLBM_ERR_DEVICE. */
vlbm_status vlbm_clo_create(int n_theta, int n_phi, int max_batch, void* hip_stream,
                            void* workspace, size_t workspace_bytes, vlbm_clo** out);
vlbm_status vlbm_clo_destroy(vlbm_clo* c);

/* z = conv(x; w, bias) (FP32, [P][COUT], may be NULL) and a = relu(z) (relu =
 * 1) or a = z, rounded to bf16 [P][COUT].  x: bf16 [P][CIN].  vector_mask: bit
 * ch set for the input channels that are vector components.  MFMA 16x16x32
 * BF16 with FP32 accumulation. */
vlbm_status vlbm_clo_conv_forward(vlbm_clo* c, int cin, int cout, int batch, const void* x,
                                  const void* w, const float* bias, uint32_t vector_mask,
                                  int relu, float* z, void* a);

/* Data gradient through a layer whose input is a hidden (scalar) activation:
 * dx = conv^T(dz; wt), then dx_masked = dx * (z_in > 0) (the ReLU of the layer
 * below) rounded to bf16 [P][CIN].  dz: bf16 [P][COUT]; z_in: FP32 [P][CIN]. */
vlbm_status vlbm_clo_conv_backward_data(vlbm_clo* c, int cin, int cout, int batch,
                                        const void* dz, const void* wt, const float* z_in,
                                        void* dx_masked);

/* Weight and bias gradients dw = sum_p dz x_tap (FP32 [COUT][9 * CIN]) and db =
 * sum_p dz (FP32 [COUT]); deterministic two-pass reduction over cells. */
vlbm_status vlbm_clo_conv_backward_weight(vlbm_clo* c, int cin, int cout, int batch,
                                          const void* x, const void* dz, uint32_t vector_mask,
                                          float* dw, float* db);

/* Loss of the network output z (FP32 [P][16], channels 0..2 used) against
 * target (FP32 [P][3]): L = sum_p w(row) |z - t|^2 / (3 * batch * n_phi * sum w),
 * w = sin(theta).  Writes dL/dz as bf16 [P][16] (zero in channels 3..15) and
 * per-block partial sums of L to loss_partials (FP32, *n_partials entries,
 * summed by the caller). */
vlbm_status vlbm_clo_loss(vlbm_clo* c, int batch, const float* z, const float* target,
                          void* dz, float* loss_partials, int* n_partials);

/* Adam (Kingma and Ba, 2015) with bias correction on n FP32 parameters; step
 * counts from 1. */
vlbm_status vlbm_clo_adam(vlbm_clo* c, int n, float* param, const float* grad, float* m,
                          float* v, int step, float lr, float beta1, float beta2, float eps);

/* Round the FP32 master weights [COUT][9 CIN] to the bf16 layouts w and wt. */
vlbm_status vlbm_clo_pack_weights(vlbm_clo* c, int cin, int cout, const float* master, void* w,
                                  void* wt);

/* Network input from moment fields: x[p] = ((rho - 1) s_rho, u_theta s_u,
 * u_phi s_u, (T - 1) s_T, 0 x 4) as bf16 [P][8].  T may be NULL (channel 3
 * is then 0). */
vlbm_status vlbm_clo_pack_input(vlbm_clo* c, int batch, const double* rho, const double* u_theta,
                                const double* u_phi, const double* T, double s_rho, double s_u,
                                double s_T, void* x);

/* Moment corrections from the network output z (FP32 [P][16]): d_rho = z0 o_rho,
 * d_u_theta = z1 o_u, d_u_phi = z2 o_u (FP64 fields). */
vlbm_status vlbm_clo_unpack_output(vlbm_clo* c, int batch, const float* z, double o_rho,
                                   double o_u, double* d_rho, double* d_u_theta, double* d_u_phi);

/* Training target from two sets of moment fields (a: reference, b: prediction):
 * target[p] = ((rho_a - rho_b) / o_rho, (u_theta_a - u_theta_b) / o_u,
 * (u_phi_a - u_phi_b) / o_u) as FP32 [P][3]. */
vlbm_status vlbm_clo_pack_target(vlbm_clo* c, int batch, const double* rho_a, const double* ut_a,
                                 const double* up_a, const double* rho_b, const double* ut_b,
                                 const double* up_b, double o_rho, double o_u, float* target);

/* Coarse graining of fine FP64 fields [batch][n_theta_f][n_phi_f] by boxes of
 * factor x factor cells, with the area weight sin(theta): rho by area average,
 * u by momentum average (sum w rho u / sum w rho).  Needs no context. */
vlbm_status vlbm_box_filter(int n_theta_f, int n_phi_f, int factor, int batch, const double* rho,
                            const double* u_theta, const double* u_phi, double* rho_c,
                            double* u_theta_c, double* u_phi_c, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* VLBM_CLOSURE_H */
