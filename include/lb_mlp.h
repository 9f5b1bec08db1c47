/*
 * lb_mlp.h -- C ABI of the MLP surrogate of the time-averaged acoustic
 * radiation force (BF16 MFMA forward, backward and Adam on gfx950).
 *
 * The network maps four normalised inputs (k R, the position phase k h, the
 * contrast c_p/c0 and the lattice resolution 1/R in inverse cells, each
 * mapped to [-1, 1] by the caller) to the force
 * normalised by the small-sphere scale F0 = pi R^3 Pa^2 k / (3 rho0 c0^2) of
 * eq. ARF_Gorkov_3D (with it F/F0 tends to f1 sin 2kh as kR -> 0).  It is
 * trained on forces computed by the wave lattice Boltzmann library
 * (lb_wave.h), which stays the reference and the fallback outside the
 * training box.  The resolution is an input because the lattice's answer at
 * a given (k R, k h, c_p/c0) still depends on how many cells span the
 * radius, by up to a few percent over R = 4 .. 16 cells.
 *
 * Architecture (fixed): 4 -> 256 -> 256 -> 256 -> 256 -> 1, exact-erf GELU
 * after each hidden layer, linear output.  Parameters are FP32 masters, laid
 * out layer by layer as W_l (out x in, row-major) followed by b_l; the
 * matrix products run on MFMA with BF16 operands (weights, activations and
 * back-propagated errors rounded to BF16) and FP32 accumulation; biases,
 * pre-activations, the loss and Adam are FP32, the loss sum FP64.  Weight
 * gradients are summed over the batch in fixed chunks and the chunk sums
 * added in a fixed order, so gradients and training are deterministic.
 *
 * Conventions as in lb_wave.h: C linkage, lb_status return codes,
 * lb_last_error(), pointers are host pointers unless named dev_*, the caller
 * owns one 256-byte aligned device workspace and a HIP stream, the library
 * never allocates device memory, a handle is not thread-safe.
 */
#ifndef LB_MLP_H
#define LB_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_mlp lb_mlp;

/* Number of FP32 parameters (198913). */
int32_t lb_mlp_num_params(void);

/* Workspace bytes for training batches of up to max_batch samples (0 unless
 * 1 <= max_batch <= 2^24). */
size_t lb_mlp_workspace_bytes(int32_t max_batch);

/* Create a handle on the caller's workspace and stream.  Parameters and the
 * Adam state start at zero; load parameters with lb_mlp_set_params.
 * LB_EINVAL unless 1 <= max_batch <= 2^24; LB_ENOMEM if the workspace is
 * smaller than lb_mlp_workspace_bytes(max_batch) or not 256-byte aligned. */
int lb_mlp_create(int32_t max_batch, void *dev_workspace, size_t workspace_bytes,
                  void *hip_stream, lb_mlp **out);
int lb_mlp_destroy(lb_mlp *h);  /* NULL-safe */

/* Copy FP32 parameters in (also zeroes the Adam moments and step count) or
 * out; both synchronise the stream. */
int lb_mlp_set_params(lb_mlp *h, const float *host_params);
int lb_mlp_get_params(lb_mlp *h, float *host_params);

/* y = net(x) for 1 <= B <= 2^30 samples (independent of max_batch: inference
 * keeps no activations in the workspace): dev_x B x 4 FP32, dev_y B FP32.  One fused launch carries
 * 128 samples per workgroup through every layer with the activations in LDS;
 * operand roundings as in the training forward (BF16 weights and
 * activations, FP32 accumulation and bias).  Asynchronous on the handle's
 * stream. */
int lb_mlp_forward(lb_mlp *h, const float *dev_x, int32_t B, float *dev_y);

/* The training forward (one MFMA GEMM launch per layer, activations kept in
 * the workspace for the backward pass) for B <= max_batch samples; same
 * arguments as lb_mlp_forward.  Both run the same MFMA sequence per output
 * (sums starting at the bias, K in the same 32-wide steps) and the same
 * roundings, so their outputs agree bit for bit.  Asynchronous. */
int lb_mlp_forward_layered(lb_mlp *h, const float *dev_x, int32_t B, float *dev_y);

/* Gradient of the mean squared error L = (1/B) sum (y - t)^2 with respect to
 * every parameter, without updating (host_grads: lb_mlp_num_params() floats;
 * host_loss may be NULL).  Synchronises the stream. */
int lb_mlp_grad(lb_mlp *h, const float *dev_x, const float *dev_t, int32_t B, float *host_grads,
                double *host_loss);

/* One Adam step on the mean squared error of the batch (asynchronous);
 * lb_mlp_last_loss() returns that batch's loss (synchronises).  LB_EINVAL
 * for a batch outside 1 .. max_batch, a NULL pointer, or hyper-parameters
 * outside lr > 0, 0 <= beta < 1, eps > 0. */
int lb_mlp_train_step(lb_mlp *h, const float *dev_x, const float *dev_t, int32_t B, float lr,
                      float beta1, float beta2, float eps);

/* n_steps Adam steps on the same batch, step s with learning rate host_lr[s]
 * (host array of n_steps floats, copied before return): the same kernels as
 * n_steps calls of lb_mlp_train_step, enqueued from one call.  Asynchronous;
 * every learning rate is checked before anything is enqueued. */
int lb_mlp_train_steps(lb_mlp *h, const float *dev_x, const float *dev_t, int32_t B,
                       int32_t n_steps, const float *host_lr, float beta1, float beta2,
                       float eps);
int lb_mlp_last_loss(lb_mlp *h, double *loss);

/* One 16x16x32 BF16 MFMA tile D = A B (A 16 x 32, B 32 x 16, row-major BF16
 * bits; D 16 x 16 row-major FP32), computed by the same fragment mapping as
 * the network's products: a check of the matrix-core lane layout. */
int lb_mlp_mfma_probe(const uint16_t *dev_A, const uint16_t *dev_B, float *dev_D,
                      void *hip_stream);

/* The network's activation applied elementwise: out = g(z) = z Phi(z), the
 * exact (erf) GELU, or with derivative != 0 its derivative g'(z) = Phi(z) +
 * z phi(z), in the FP32 form every layer uses (Phi from Hastings' rational-
 * exponential erf, within 3e-7 of the exact value).  dev_z and dev_out hold n
 * FP32 values (0 <= n <= 2^31; they may alias).  Asynchronous on hip_stream.
 * LB_EINVAL for a negative or too large n or a NULL pointer with n > 0. */
int lb_mlp_activation(const float *dev_z, int64_t n, int32_t derivative, float *dev_out,
                      void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LB_MLP_H */
