// Learned GENO gate: the small network that predicts the path function chi
// (Eq. (4)) of a cell and direction from its normalised 5-cell stencil.
//
// Parameters (6849 floats, flat, in this order): W1[64][40], b1[64],
// W2[64][64], b2[64], w3[64], b3.
//   a1 = W1 x + b1, h1 = gelu(a1), a2 = W2 h1 + b2, h2 = gelu(a2),
//   z = w3 . h2 + b3, p = 1 / (1 + exp(-z)).
// gelu(u) = u/2 (1 + tanh(sqrt(2/pi) (u + 0.044715 u^3))).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace mlp {

constexpr int NIN = 40;
constexpr int NH = 64;
constexpr int OW1 = 0;
constexpr int OB1 = OW1 + NH * NIN;   // 2560
constexpr int OW2 = OB1 + NH;         // 2624
constexpr int OB2 = OW2 + NH * NH;    // 6720
constexpr int OW3 = OB2 + NH;         // 6784
constexpr int OB3 = OW3 + NH;         // 6848
constexpr int NPARAM = OB3 + 1;       // 6849

constexpr float GC = 0.7978845608028654f;   // sqrt(2/pi)

__device__ __forceinline__ float gelu(float u) {
  const float t = tanhf(GC * (u + 0.044715f * u * u * u));
  return 0.5f * u * (1.0f + t);
}

__device__ __forceinline__ float gelu_d(float u) {
  const float t = tanhf(GC * (u + 0.044715f * u * u * u));
  return 0.5f * (1.0f + t) + 0.5f * u * (1.0f - t * t) * GC * (1.0f + 3.0f * 0.044715f * u * u);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// The same function for inference, where the result is rounded to bfloat16
// or summed in float32: u (1 + tanh z) / 2 = u / (1 + exp(-2 z)), with the
// hardware exponential and reciprocal (a few units in the last place of
// float32, far below bfloat16 resolution). Large |z| give u or 0 exactly.
__device__ __forceinline__ float gelu_fast(float u) {
  const float z = GC * (u + 0.044715f * u * u * u);
  return u * __builtin_amdgcn_rcpf(1.0f + __expf(-2.0f * z));
}

// stable softplus(z) - y z
__device__ __forceinline__ float bce(float z, float y) {
  return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))) - y * z;
}

}  // namespace mlp
