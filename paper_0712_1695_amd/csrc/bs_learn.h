// bs_learn.h -- launch interface of the rule-selector kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bs_internal.h"

namespace bsk {

// Packed parameter blob (BF16): mu[16], inv_sigma[16], W1[16][64], b1[64],
// W2[64][64], b2[64], W3[64][4], b3[4].
constexpr int kMlpBlobLen = 5540;
// Trainable part (everything after mu, inv_sigma).
constexpr int kMlpGradLen = 5508;

hipError_t launch_label(const DevMesh &m, const int2 *pairs, int n, float hbar, const double *tri, int nq,
                        const float *rules, double tau, float *feats, int8_t *labels, float *errs, hipStream_t s);
hipError_t launch_mlp_grad_step(const float *feats, const int8_t *labels, const int *index, int n, __bf16 *wb,
                                const float *class_w, float *gpart, float *wpart, float *lpart, float *master,
                                float *mom1, float *mom2, float lr, float beta1, float beta2, float eps, int step,
                                float *grad_out, hipStream_t s);
hipError_t launch_sum_f(const float *a, int n, double *out, hipStream_t s);
hipError_t launch_mlp_logits(const float *feats, int n, const __bf16 *wb, float *logits, hipStream_t s);

} // namespace bsk
