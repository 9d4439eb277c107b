// The alpha predictor: a three-layer perceptron 65 -> 128 -> 128 -> 1 with
// exact-erf GELU, on bfloat16 matrix-core products with FP32 accumulation
// (16x16x16 MFMA tiles, one wavefront per 16 batch rows or per 16x16 output
// tile) and FP32 master weights updated by Adam.
//
// Inputs are the 65 spectral features of a data set (64 log-energies of
// the data per quarter-decade level of the kernel spectrum |k^|^2 / s_max,
// and log10(delta/||F||)); they are standardised with stored mean and
// deviation.  The output y is the standardised log10 alpha:
// log10 alpha = t_mu + t_sigma * y.
//
// Parameter vector (FP32, this order): W1[128][65], b1[128], W2[128][128],
// b2[128], w3[128], b3[1] -- 25089 values.  Normalisation vector:
// mu[65], sigma[65], t_mu, t_sigma -- 132 values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "control.hpp"

namespace fr3d {

constexpr int MLP_IN = 65;
constexpr int MLP_INP = 80;  // input width padded to whole 16-wide K steps
constexpr int MLP_H = 128;
constexpr int MLP_NP = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;
constexpr int MLP_NNORM = 2 * MLP_IN + 2;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H,
              OFF_B2 = OFF_W2 + MLP_H * MLP_H, OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H;

// Device workspace of one training step for batches of up to `cap` rows.
struct MlpWork {
  int cap;
  uint16_t* xb;   // [cap][80]  standardised inputs, bf16
  float* z1;      // [cap][128]
  uint16_t* h1b;  // [cap][128]
  float* z2;      // [cap][128]
  uint16_t* h2b;  // [cap][128]
  float* y;       // [cap] standardised prediction
  float* dz1;     // [cap][128] FP32 (bias gradients)
  uint16_t* dz1b; // [cap][128]
  float* dz2;     // [cap][128]
  uint16_t* dz2b; // [cap][128]
  float* dy;      // [cap]
  float* sq;      // [cap] squared errors
};

size_t mlp_work_bytes(int cap);
void mlp_work_carve(MlpWork* w, void* base, int cap);

// Forward pass for B rows of raw features X[B][65]: writes log10 alpha to
// out (may be null) and, with w non-null, the activations a training step
// needs.  With seed non-null (B = 1, w null) the prediction plus the
// calibration cal[0] + sum_k cal[1+k] X[k] (cal: 66 doubles on the device,
// or null for none), clipped to [seed->lo, seed->hi], becomes the first
// point of a seeded search.
hipError_t mlp_forward(const float* params, const float* norm, const float* X, int B, float* out, MlpWork* w,
                       Ctrl* seed, hipStream_t s, const double* cal = nullptr);

// Backward pass (after mlp_forward with the same w) for targets t[B]
// (log10 alpha), gradients of the mean squared error in standardised units
// into grad[25089], loss into *loss (device, may be null); then, if lr > 0,
// one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with bias corrections
// c1 = 1 - beta1^step, c2 = 1 - beta2^step.
hipError_t mlp_backward_adam(float* params, const float* norm, const float* t, int B, MlpWork* w, float* grad,
                             float* loss, float* m, float* v, double lr, double c1, double c2, hipStream_t s);

}  // namespace fr3d
