// Learned bound on the k-NN search radius (predictor.hip).
#pragma once

#include "search.h"

namespace pdd {

constexpr int kPredParams = 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1;

int pred_set(Ctx* c, const float* host, int64_t n);
int pred_get(Ctx* c, float* host, int64_t n);
// network outputs of n bf16 feature rows (device buffers, stream-ordered)
int pred_forward(Ctx* c, const uint16_t* feat, int64_t n, float* out);
// gradient of the mean pinball loss over n <= 128 rows; loss (if not null) gets the loss
int pred_grad(Ctx* c, const uint16_t* feat, const float* target, int64_t n, float tau, float* grad, float* loss);
// `steps` Adam steps on minibatches of `batch` rows; loss (if not null) gets one value per step
int pred_train(Ctx* c, const uint16_t* feat, const float* target, int64_t n, int steps, int batch, float lr, float tau,
               uint64_t seed, float* loss);
// training rows of a grid: features and targets of every anchor cell (first `cap`), their count in *count
int pred_samples(Ctx* c, const GridView& g, int k, int K, uint16_t* feat, float* target, int64_t cap, int64_t* count);
// squared search radius per cell (indexed by level base + cell; 0 = none) for the anchors of g
int pred_radii(Ctx* c, const GridView& g, int K, const uint64_t** r2_out);

}  // namespace pdd
