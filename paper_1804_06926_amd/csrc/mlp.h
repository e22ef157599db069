// The kernel-selector network: shapes, parameter layout and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace tcx {

constexpr int MLP_IN = 6, MLP_H = 32, MLP_OUT = 3;
// float32 parameter vector: W1 [32][6], b1, W2 [32][32], b2, W3 [3][32], b3
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_OUT * MLP_H;
constexpr int MLP_NPARAM = MLP_OFF_B3 + MLP_OUT;   // 1379
constexpr int MLP_MAX_BATCH = 65536;
static_assert(sizeof(((Ctrl*)nullptr)->features[0]) == MLP_IN * sizeof(float), "feature row size");

// Compute copy: bfloat16 weights, float32 biases.
struct MlpCompute {
    uint16_t W1[MLP_H * MLP_IN];
    uint16_t W2[MLP_H * MLP_H];
    uint16_t W3[MLP_OUT * MLP_H];
    float b1[MLP_H];
    float b2[MLP_H];
    float b3[MLP_OUT];
};

// Per-sample activations and errors of a training batch (device arrays).
struct MlpActs {
    float* h1;    // [B][32]
    float* h2;    // [B][32]
    float* dh1;   // [B][32]
    float* dh2;   // [B][32]
    float* dz;    // [B][3]
    float* loss;  // [B]
};

void mlp_cast(const float* master, MlpCompute* cw, hipStream_t s);
void mlp_forward(const MlpCompute* cw, const float* X, int B, float* logits, hipStream_t s);
void mlp_gradient(const MlpCompute* cw, const float* X, const int32_t* y, const float* w, int B, const MlpActs& acts,
                  float* grad, float* loss, hipStream_t s);
void mlp_adam(float* master, const float* grad, float* m, float* v, float lr, int step, hipStream_t s);
void mlp_select(const MlpCompute* cw, Ctrl* ctrl, uint8_t* choice, hipStream_t s);
void bucket_features_launch(Ctrl* ctrl, hipStream_t s);

}  // namespace tcx
