// Learned cost model: a 12 -> 64 -> 64 -> 1 MLP that predicts an anchor's
// scatter-gather work (log1p of its algorithmic bytes) from cheap window and
// degree features.  Weights are stored in BF16 and used in every forward and
// backward pass; arithmetic accumulates in FP32; training keeps FP32 master
// weights and Adam moments.
#pragma once

#include "internal.h"

constexpr int kMlpF = 12;  // features
constexpr int kMlpH = 64;  // hidden width
constexpr int kMlpRaw = 8; // raw integer features stored per anchor
// flat parameter layout
constexpr int kOffW1 = 0;                        // [H][F]
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpF;   // [H]
constexpr int kOffW2 = kOffB1 + kMlpH;           // [H][H] (row = output unit)
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;   // [H]
constexpr int kOffW3 = kOffB2 + kMlpH;           // [H]
constexpr int kOffB3 = kOffW3 + kMlpH;           // [1]
constexpr int kMlpParams = kOffB3 + 1;           // 5057

// Raw features of an anchor e = (u -> v, t) (all counts):
//  0 |OUT(u) in [lo, t]|   1 |IN(v) in [lo, t]|   2 |IN(u) in [lo, t)|
//  3 |OUT(v) in [lo, t)|   4 out-degree of u      5 in-degree of u
//  6 out-degree of v       7 in-degree of v
// The network input adds log1p(r2 * r1), log1p(r2 * r3), log1p(delta hours)
// and log1p(L), after log1p of the eight raw counts; every input is then
// standardised with the training-set mean and standard deviation.

struct MlpModel {
  bool loaded = false;
  uint32_t train_samples = 0;
  float master[kMlpParams];   // FP32 master weights
  float mean[kMlpF], inv_std[kMlpF];
  // the length rule fitted on the same labels: predicted bytes = len_coef x
  // sender-window length (geometric mean of bytes / length); 0 if unknown
  float len_coef = 0.f;
  uint16_t *d_w16 = nullptr;  // device BF16 weights
  float *d_norm = nullptr;    // device mean[12], inv_std[12]
};

MlpModel &global_model();
hipError_t model_upload(MlpModel &m);

// Predict log-work for n anchors whose raw features are feat[i * 8 ...].
// Predict log-work for list items: pred[i] from feat[idx[i] * 8 ...] (idx
// may be NULL for the identity); the item count is *n_dev if n_dev is not
// NULL, else n_host.
// Batched stores (vgraph != NULL): each item's window and cycle length are
// its sub-graph's (item idx[i] is a CSC position, in_dst[idx[i]] its vertex).
struct SubParams;
hipError_t mlp_infer(const MlpModel &m, const uint32_t *feat, const uint32_t *idx, uint32_t n_host,
                     const uint32_t *n_dev, float delta_hours, float L, float *pred, hipStream_t s,
                     const uint32_t *in_dst = nullptr, const uint32_t *vgraph = nullptr,
                     const SubParams *sub = nullptr);

uint16_t f32_to_bf16(float f);
float bf16_to_f32(uint16_t h);
