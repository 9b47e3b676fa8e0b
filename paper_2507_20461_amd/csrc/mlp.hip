// Training kernels of the learned GENO gate (float32): forward pass, loss,
// back-propagation and Adam, written out per sample and per parameter.
// Gradients are reduced over the samples in two deterministic passes (no
// atomics): per chunk of CH samples and parameter a float64 partial sum, then
// per parameter the sum of its partials in chunk order.
//
// Minibatch layout: X[n][40], y[n]; scratch per sample: a1[64], h1[64],
// a2[64], h2[64], da1[64], da2[64], dz, loss, then the partial sums
// [ceil(n / CH)][6849] (see geno_mlp_train_workspace_bytes).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>

#include "geno_gks.h"
#include "mlp_device.hpp"

namespace geno_err {
int fail(int code, const char* fmt, ...);
}

namespace {

using geno_err::fail;
using namespace mlp;

constexpr int TB = 128;   // threads per work-group of the per-sample kernels

constexpr int CH = 256;   // samples per partial sum of the gradient reduction

struct Scratch {
  float *a1, *h1, *a2, *h2, *da1, *da2, *dz, *ls;
  double* part;   // [nchunk][NPARAM]
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int nchunks(int n) { return (n + CH - 1) / CH; }

Scratch scratch_of(void* ws, int n) {
  char* b = (char*)ws;
  Scratch s;
  size_t off = 0;
  float** per_sample[6] = {&s.a1, &s.h1, &s.a2, &s.h2, &s.da1, &s.da2};
  for (float** f : per_sample) {
    *f = (float*)(b + off);
    off = align256(off + sizeof(float) * NH * (size_t)n);
  }
  s.dz = (float*)(b + off);
  off = align256(off + sizeof(float) * (size_t)n);
  s.ls = (float*)(b + off);
  off = align256(off + sizeof(float) * (size_t)n);
  s.part = (double*)(b + off);
  return s;
}

size_t scratch_bytes(int n) {
  return 6 * align256(sizeof(float) * NH * (size_t)n) + 2 * align256(sizeof(float) * (size_t)n) +
         align256(sizeof(double) * NPARAM * (size_t)nchunks(n));
}

// weights of both hidden layers in LDS (26.6 KB), the rest in registers
__device__ __forceinline__ void load_weights(const float* __restrict__ P, float* sW1, float* sW2,
                                             float* sv) {
  for (int q = threadIdx.x; q < NH * NIN; q += blockDim.x) sW1[q] = P[OW1 + q];
  for (int q = threadIdx.x; q < NH * NH; q += blockDim.x) sW2[q] = P[OW2 + q];
  for (int q = threadIdx.x; q < 3 * NH + 1; q += blockDim.x) {
    const int src = q < NH ? OB1 + q : (q < 2 * NH ? OB2 + q - NH : (q < 3 * NH ? OW3 + q - 2 * NH : OB3));
    sv[q] = P[src];
  }
  __syncthreads();
}

// Per sample: forward pass and the back-propagated pre-activation gradients.
// With y == nullptr only the probabilities are written (prob).
__global__ void __launch_bounds__(TB) k_mlp_sample(const float* __restrict__ P,
                                                   const float* __restrict__ X,
                                                   const float* __restrict__ y, int n,
                                                   Scratch s, float* __restrict__ prob) {
  __shared__ float sW1[NH * NIN], sW2[NH * NH], sv[3 * NH + 1];
  load_weights(P, sW1, sW2, sv);
  const float* b1 = sv;
  const float* b2 = sv + NH;
  const float* w3 = sv + 2 * NH;
  const float b3 = sv[3 * NH];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[NIN];
#pragma unroll
  for (int k = 0; k < NIN; ++k) x[k] = X[(size_t)i * NIN + k];
  float h1[NH];
#pragma unroll
  for (int o = 0; o < NH; ++o) {
    float a = b1[o];
#pragma unroll
    for (int k = 0; k < NIN; ++k) a += sW1[o * NIN + k] * x[k];
    h1[o] = gelu(a);
    if (y) {
      s.a1[(size_t)i * NH + o] = a;
      s.h1[(size_t)i * NH + o] = h1[o];
    }
  }
  float z = b3;
  float a2[NH];
#pragma unroll
  for (int o = 0; o < NH; ++o) {
    float a = b2[o];
#pragma unroll
    for (int k = 0; k < NH; ++k) a += sW2[o * NH + k] * h1[k];
    a2[o] = a;
    z += w3[o] * gelu(a);
  }
  if (!y) {
    prob[i] = sigmoid(z);
    return;
  }
  const float yi = y[i];
  const float dzi = (sigmoid(z) - yi) / (float)n;
  s.dz[i] = dzi;
  s.ls[i] = bce(z, yi);
  // da2 = dz w3 * gelu'(a2); reuse a2 for da2
#pragma unroll
  for (int o = 0; o < NH; ++o) {
    s.a2[(size_t)i * NH + o] = a2[o];
    s.h2[(size_t)i * NH + o] = gelu(a2[o]);
    a2[o] = dzi * w3[o] * gelu_d(a2[o]);
    s.da2[(size_t)i * NH + o] = a2[o];
  }
  // da1 = (W2^T da2) * gelu'(a1)
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    float d = 0.0f;
#pragma unroll
    for (int o = 0; o < NH; ++o) d += sW2[o * NH + k] * a2[o];
    s.da1[(size_t)i * NH + k] = d * gelu_d(s.a1[(size_t)i * NH + k]);
  }
}

// Partial sums of the gradient terms: thread (parameter p, chunk blockIdx.y)
// over the chunk's samples, in sample order.
__global__ void __launch_bounds__(256) k_mlp_partial(const float* __restrict__ X, Scratch s,
                                                     int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const int i0 = (int)blockIdx.y * CH, i1 = min(n, i0 + CH);
  double acc = 0.0;
  if (p < OB1) {
    const int o = p / NIN, k = p % NIN;
    for (int i = i0; i < i1; ++i)
      acc += (double)s.da1[(size_t)i * NH + o] * X[(size_t)i * NIN + k];
  } else if (p < OW2) {
    const int o = p - OB1;
    for (int i = i0; i < i1; ++i) acc += s.da1[(size_t)i * NH + o];
  } else if (p < OB2) {
    const int q = p - OW2, o = q / NH, k = q % NH;
    for (int i = i0; i < i1; ++i)
      acc += (double)s.da2[(size_t)i * NH + o] * s.h1[(size_t)i * NH + k];
  } else if (p < OW3) {
    const int o = p - OB2;
    for (int i = i0; i < i1; ++i) acc += s.da2[(size_t)i * NH + o];
  } else if (p < OB3) {
    const int k = p - OW3;
    for (int i = i0; i < i1; ++i) acc += (double)s.dz[i] * s.h2[(size_t)i * NH + k];
  } else {
    for (int i = i0; i < i1; ++i) acc += s.dz[i];
  }
  s.part[(size_t)blockIdx.y * NPARAM + p] = acc;
}

// One thread per parameter: its partial sums in chunk order.
__global__ void __launch_bounds__(256) k_mlp_sum(Scratch s, int nch, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  double acc = 0.0;
  for (int c = 0; c < nch; ++c) acc += s.part[(size_t)c * NPARAM + p];
  grad[p] = (float)acc;
}

// mean of the per-sample losses (one work-group, float64 accumulation)
__global__ void __launch_bounds__(256) k_mlp_loss(Scratch s, int n, float* __restrict__ loss) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += s.ls[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = (float)((red[0] + red[1] + red[2] + red[3]) / n);
}

__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ P,
                                                  const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  float lr, float b1, float b2, float eps, float c1,
                                                  float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

}  // namespace

extern "C" {

size_t geno_mlp_train_workspace_bytes(int n) { return n < 1 ? 0 : scratch_bytes(n); }

int geno_mlp_forward(const float* params, const float* X, int n, float* prob, void* stream) {
  if (!params || !X || !prob) return fail(GENO_EINVAL, "null pointer");
  if (n < 0) return fail(GENO_EINVAL, "n must be >= 0");
  if (n == 0) return GENO_OK;
  hipLaunchKernelGGL(k_mlp_sample, dim3((n + TB - 1) / TB), dim3(TB), 0, (hipStream_t)stream,
                     params, X, (const float*)nullptr, n, Scratch{}, prob);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GENO_OK : fail(GENO_EHIP, "k_mlp_sample: %s", hipGetErrorString(e));
}

int geno_mlp_grad(const float* params, const float* X, const float* y, int n, float* grad,
                  float* loss, void* ws, void* stream) {
  if (!params || !X || !y || !grad || !ws) return fail(GENO_EINVAL, "null pointer");
  if (n < 1) return fail(GENO_EINVAL, "n must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  const Scratch s = scratch_of(ws, n);
  hipLaunchKernelGGL(k_mlp_sample, dim3((n + TB - 1) / TB), dim3(TB), 0, st, params, X, y, n, s,
                     (float*)nullptr);
  const int nch = nchunks(n);
  hipLaunchKernelGGL(k_mlp_partial, dim3((NPARAM + 255) / 256, nch), dim3(256), 0, st, X, s, n);
  hipLaunchKernelGGL(k_mlp_sum, dim3((NPARAM + 255) / 256), dim3(256), 0, st, s, nch, grad);
  if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, s, n, loss);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GENO_OK : fail(GENO_EHIP, "mlp gradient: %s", hipGetErrorString(e));
}

int geno_mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr,
                  float beta1, float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v) return fail(GENO_EINVAL, "null pointer");
  if (t < 1) return fail(GENO_EINVAL, "t counts from 1");
  const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GENO_OK : fail(GENO_EHIP, "k_mlp_adam: %s", hipGetErrorString(e));
}

}  // extern "C"
