/*
 * sdpdem_mlp.h -- C ABI of the viscosity surrogate: a 4-64-64-64-1 SiLU
 * multilayer perceptron mapping (volume fraction, sphere diameter / dx,
 * kT, log shear rate) to log(eta_eff / eta), trained on the viscosities
 * that the batched Lees-Edwards viscometer (sdpdem_create_batch,
 * sdpdem_box_stress) measures.  Not part of the paper: it is the learned
 * part of the viscometer workflow, with the plain simulation as its
 * fallback and the reference its error is measured against.
 *
 * Numerics: parameters kept as float32 masters and used as bfloat16
 * (round to nearest even) in the forward and backward passes; activations
 * and all sums in float32 on the matrix cores (16x16x4 float32 MFMA);
 * loss = mean squared error; Adam with bias correction on the masters.
 *
 * Memory: the caller owns a device workspace of sdpdem_mlp_workspace_bytes
 * bytes and keeps it alive until sdpdem_mlp_destroy; inputs and outputs of
 * predict and train_step are device pointers; init/read use host memory.
 * Every call takes a hipStream_t (as void*); predict and train_step only
 * enqueue work, read synchronises.  Return 0 or a negative SDPDEM_E_* code
 * of sdpdem.h.
 */
#ifndef SDPDEM_MLP_H
#define SDPDEM_MLP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SDPDEM_MLP_PARAMS = 8705, SDPDEM_MLP_MAX_BATCH = 256 };

typedef struct sdpdem_mlp_config {
  float norm_mean[4];  /* inputs are normalised as (x - mean) / std         */
  float norm_std[4];
  float lr, beta1, beta2, eps; /* Adam                                       */
  int32_t max_batch;   /* training batch limit, 1..SDPDEM_MLP_MAX_BATCH      */
  int32_t reserved;    /* 0 */
} sdpdem_mlp_config;

typedef struct sdpdem_mlp sdpdem_mlp;

/* Bytes of device workspace for the network that stands in for the
 * viscosity measurement of Secs. 4.1 and 4.3 (Eq. poiseuave): parameters,
 * bfloat16 copies, gradients, Adam moments and a batch of activations.
 * Touches no device. */
int sdpdem_mlp_workspace_bytes(const sdpdem_mlp_config* cfg, size_t* bytes);

/* Create the surrogate of the effective viscosity of Secs. 4.1 and 4.3.
 * init_params: host float32[SDPDEM_MLP_PARAMS] in the order W1 [4 x 64]
 * row-major (input-major), b1[64], W2 [64 x 64], b2, W3 [64 x 64], b3,
 * W4 [64 x 1], b4[1].  Rejects std <= 0, lr <= 0, betas outside [0, 1),
 * eps < 0, max_batch outside 1..256, a short or missing workspace. */
int sdpdem_mlp_create(const sdpdem_mlp_config* cfg, const float* init_params, void* d_workspace,
                      size_t workspace_bytes, void* hip_stream, sdpdem_mlp** out);

/* Answer viscosity queries in place of runs of Alg. 1 (Secs. 4.1, 4.3):
 * y[i] = network(x[i]) for i < n; x: device float32 [n][4], y: device
 * float32 [n].  Only enqueues. */
int sdpdem_mlp_predict(sdpdem_mlp* m, const float* d_x, float* d_y, int64_t n, void* hip_stream);

/* One training step towards viscosities measured by the batched runs of
 * Alg. 1 (the measurement of Sec. 4.1 on sheared boxes), on a batch
 * (device x [batch][4], targets t [batch]):
 * forward, loss, backward; with update != 0 also one Adam step.  The loss
 * and gradient of the step stay readable with sdpdem_mlp_read. */
int sdpdem_mlp_train_step(sdpdem_mlp* m, const float* d_x, const float* d_t, int32_t batch,
                          int32_t update, void* hip_stream);

/* State of the viscosity surrogate (Secs. 4.1, 4.3), synchronises.
 * Host copies (any pointer may be NULL): float32 master parameters, the
 * parameters as used (bfloat16 values widened to float32), the gradient of
 * the last train_step, its loss, and the number of Adam steps taken. */
int sdpdem_mlp_read(sdpdem_mlp* m, float* params, float* used_params, float* grad, float* loss,
                    int64_t* steps, void* hip_stream);

/* Release the surrogate's handle (the viscosity model of Secs. 4.1,
 * 4.3); the caller frees the workspace afterwards. */
void sdpdem_mlp_destroy(sdpdem_mlp* m);

#ifdef __cplusplus
}
#endif
#endif /* SDPDEM_MLP_H */
