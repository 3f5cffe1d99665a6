/*
 * rfps_mlp.h -- C ABI of the voxel-parameter network of librfps.so.
 *
 * The paper chooses the voxel resolution v (n_vox of eq. voxel_size) by
 * hand and reports that the best value depends on the cloud (Sec. 5.6.2).
 * This small network predicts, from 516 features of a cloud, the relative
 * run time and the pruning rate of RadiusFPS-G for each of 36 candidate
 * (n_vox, shell spacing) pairs, so that a cloud can be indexed with the
 * candidate it expects to be fastest.  The choice never changes the
 * sampled sequence (every partition of a cloud into voxels and tiles gives
 * the plain FPS result); the library's default rule is the fallback and
 * the yardstick of every choice.
 *
 * Network: 516 -> 64 (ReLU) -> 64 (ReLU) -> 72, weight matrices used in
 * bfloat16 (round to nearest even of an FP32 master copy), biases,
 * activations and accumulation in FP32; trained with Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8) on a weighted squared error.
 *
 * Parameters are packed in this order, each matrix row-major [out][in]:
 *   W1 [64][516], b1 [64], W2 [64][64], b2 [64], W3 [72][64], b3 [72]
 * (41,928 values).  Outputs: y[k] = predicted ln of the run time (index
 * build + sampling) of candidate k minus the mean of that log over the 36
 * candidates (only the ranking matters), y[36 + k] = its predicted pruning
 * rate (fraction of point visits saved).
 *
 * Features of a cloud of N points (float32): f[0] = (ln N - 11) / 2;
 * f[1..3] = ln(1 + E_a) / 2 with E_a the bounding-box extents; f[4 + c] =
 * ln(1 + 64 * count_c / N) for the cells c = (z * 8 + y) * 8 + x of a cubic 8^3
 * grid of edge (1 + 1e-4) * max(E) / 8 from the box minimum (FP64
 * coordinates, clamped to the grid).
 *
 * Memory and errors follow rfps.h: the caller owns the model state and the
 * workspace (device memory, 256-byte aligned), host-visible errors return
 * at once, every call is asynchronous on `stream` unless stated.
 */
#ifndef RFPS_MLP_H
#define RFPS_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "rfps.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RFPS_MLP_INPUTS 516
#define RFPS_MLP_OUTPUTS 72
#define RFPS_MLP_CANDIDATES 36
#define RFPS_MLP_PARAMS 41928

/* Candidate k (0..35): n_vox = {12,16,24,32,48,64,96,128,192}[k / 4], shell
 * spacing = {0 (one shell), 5, 10, 20}[k % 4].  Returns 0, or 1 for a bad k. */
int32_t rfps_mlp_candidate(int32_t k, int32_t *n_vox, float *shell_spacing);

/* Bytes of the model state: FP32 master parameters, Adam moments, the
 * bfloat16 copy and the step counter. */
size_t rfps_mlp_state_size(void);

/* Bytes of workspace for calls on up to `batch` rows (1..65536); 0 if out
 * of range.  rfps_mlp_features and rfps_mlp_choose need batch 1. */
size_t rfps_mlp_workspace_size(int32_t batch);

/* Copies RFPS_MLP_PARAMS packed FP32 parameters from host memory into the
 * state, clears the Adam moments and step, rounds the bfloat16 copy.
 * Synchronous. */
rfps_status rfps_mlp_load(void *state, size_t state_bytes, const float *params_host, void *stream);

/* Waits for the stream, then copies the FP32 master parameters to host memory. */
rfps_status rfps_mlp_save(const void *state, size_t state_bytes, float *params_host, void *stream);

/* Features of one cloud (xyz device float32 [n][3]) into feat (device
 * float32 [516]); a non-finite coordinate makes every feature NaN. */
rfps_status rfps_mlp_features(const float *xyz, int32_t n, void *ws, size_t ws_bytes, float *feat,
                              void *stream);

/* y (device [batch][72]) = network(x) for x device [batch][516]. */
rfps_status rfps_mlp_forward(const void *state, size_t state_bytes, const float *x, int32_t batch,
                             void *ws, size_t ws_bytes, float *y, void *stream);

/* Gradient of L = sum_{b,o} w[b][o] (y[b][o] - t[b][o])^2 / batch with
 * respect to the packed parameters (device grad [RFPS_MLP_PARAMS]; the
 * bfloat16 rounding passes gradients straight through) and L (device
 * float, may be NULL).  t, w: device [batch][72]; w NULL = all ones. */
rfps_status rfps_mlp_gradient(const void *state, size_t state_bytes, const float *x, const float *t,
                              const float *w, int32_t batch, void *ws, size_t ws_bytes, float *grad,
                              float *loss, void *stream);

/* One Adam step with learning rate lr on the loss above (loss: device
 * float of the loss before the step, may be NULL). */
rfps_status rfps_mlp_train_step(void *state, size_t state_bytes, const float *x, const float *t,
                                const float *w, int32_t batch, float lr, void *ws, size_t ws_bytes,
                                float *loss, void *stream);

/* Choice for one cloud: the candidate with the lowest predicted log time,
 * kept only if it beats the prediction for default_cand by more than
 * margin, else default_cand.  feat: device [516] (rfps_mlp_features);
 * choice: device int32; y: device [72] predictions or NULL. */
rfps_status rfps_mlp_choose(const void *state, size_t state_bytes, const float *feat,
                            int32_t default_cand, float margin, void *ws, size_t ws_bytes,
                            int32_t *choice, float *y, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RFPS_MLP_H */
