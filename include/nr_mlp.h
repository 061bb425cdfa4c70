/*
 * nr_mlp.h -- C ABI of the learned proposal: a 64 -> 256 -> 256 -> 1
 * multilayer perceptron (ReLU hidden layers, one logit) trained with the
 * mean binary cross-entropy and Adam, and the feature builder that turns a
 * coarse segment-sum grid into one 64-value input per region.
 *
 * The network ranks (chirp-mass cell, sub-band) regions of a coarse template
 * grid so that only the top-ranked regions are re-searched on a finer
 * chirp-mass grid; the exhaustive fine grid remains the fallback and the
 * judge.  The paper's semicoherent statistic (Sec. III.C) is what the
 * features are built from; the network itself is not in the paper.
 *
 * Precision: FP32 master parameters; the weight matrices and the output
 * vector are multiplied as bfloat16 (rounded to nearest even from the
 * masters after every update) with FP32 activations and FP32 accumulation;
 * weight gradients are FP32 matrix-core products over fixed chunks of the
 * batch whose partial results are added in FP64 in chunk order, so every
 * call is bitwise reproducible.
 *
 * Parameter vector (NR_MLP_PARAMS = 82,689 floats):
 *   W1[256][64], b1[256], W2[256][256], b2[256], w3[256], b3[1]
 * (W[out][in], row-major).
 *
 * Conventions: host pointers are read during the call only; device pointers
 * are caller-owned; work is enqueued on the stream given at creation; no
 * exception crosses the ABI; status codes are those of nufft_resample.h.
 */
#ifndef NR_MLP_H
#define NR_MLP_H

#include <stdint.h>

#include "nufft_resample.h"

#ifdef __cplusplus
extern "C" {
#endif

#define NR_MLP_IN 64
#define NR_MLP_HIDDEN 256
#define NR_MLP_PARAMS 82689

typedef struct nr_mlp_s* nr_mlp;

/* Network with device state for batches of up to max_batch rows (>= 1).
 * stream: hipStream_t (NULL: the null stream).  Parameters start at zero. */
nr_status nr_mlp_create(nr_mlp* out, int64_t max_batch, void* stream);

/* Copy NR_MLP_PARAMS host floats into the masters, reset the Adam moments
 * and the step count, and refresh the bfloat16 copies (synchronous). */
nr_status nr_mlp_set_params(nr_mlp m, const float* host_params);

/* Copy the masters to NR_MLP_PARAMS host floats (synchronous). */
nr_status nr_mlp_get_params(nr_mlp m, float* host_params);

/* Training state for checkpoint and resume: the masters, both Adam moment
 * vectors and the Adam step count.  get copies them to the host (synchronous):
 * state[3 * NR_MLP_PARAMS] = masters, first moments, second moments; *step =
 * updates taken.  set restores them (and refreshes the bfloat16 copies), so a
 * network resumed from a saved state continues training exactly as the
 * original would have.  step >= 0. */
nr_status nr_mlp_get_state(nr_mlp m, float* host_state, int64_t* step);
nr_status nr_mlp_set_state(nr_mlp m, const float* host_state, int64_t step);

/* logits[B] = network(x[B][64]) (device pointers, 1 <= B <= max_batch). */
nr_status nr_mlp_forward(nr_mlp m, const float* x, int64_t B, float* logits);

/* Mean binary cross-entropy of x against labels y[B] (0 or 1) and its
 * gradient with respect to the masters: grad[NR_MLP_PARAMS] (device, or
 * NULL), loss[1] (device, or NULL).  Parameters are not changed. */
nr_status nr_mlp_gradient(nr_mlp m, const float* x, const float* y, int64_t B, float* grad,
                          float* loss);

/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * gradient grad[NR_MLP_PARAMS] (device) and learning rate lr > 0. */
nr_status nr_mlp_adam_step(nr_mlp m, const float* grad, float lr);

/* Gradient of the batch followed by one Adam update; loss[1] (device, or
 * NULL) receives the loss before the update. */
nr_status nr_mlp_train_step(nr_mlp m, const float* x, const float* y, int64_t B, float lr,
                            float* loss);

/*
 * Region features from a coarse segment-sum grid (all device pointers):
 *   stat[(mc * n_sub + sb) * K + k]  summed |X|^2 of template (mc, sb), bin k;
 *   n_used[mc * n_sub + sb]          segments in that sum;
 *   norm                             1 / (L sigma^2): |X|^2 * norm is the power
 *                                    in units of its white-noise mean;
 *   features[(mc * n_sub + sb) * 64 + 8 i + c] = z of template (clamp(mc - 3 + i), sb)
 *                                    at bin clamp(k* - 3 + c), where k* is the
 *                                    lowest bin of template (mc, sb) with the
 *                                    largest power, and z = (S norm - N)/sqrt(N)
 *                                    (0 when N = 0).
 * n_mc >= 1, n_sub >= 1, 1 <= K <= 4096.
 */
nr_status nr_mlp_region_features(const float* stat, const int32_t* n_used, int32_t n_mc,
                                 int32_t n_sub, int32_t K, double norm, float* features,
                                 void* stream);

/* Message of the last failure on m (m == NULL: of the last failed create or
 * feature call on this thread). */
const char* nr_mlp_last_error(nr_mlp m);

/* Free the network (synchronises its stream).  NULL is a no-op. */
void nr_mlp_destroy(nr_mlp m);

#ifdef __cplusplus
}
#endif

#endif /* NR_MLP_H */
