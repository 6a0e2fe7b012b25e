// The learned warm start of the entropy filter's search: a 16-64-64-1 tanh MLP in
// FP32 (inference, backward pass, Adam), written as plain HIP kernels.
//
//   x_s = (x - mean) / std;  h1 = tanh(W1 x_s + b1);  h2 = tanh(W2 h1 + b2);  y = w3.h2 + b3
//   loss = mean over the batch of (y - t)^2
// Flat parameters (5,313): W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3[1].
// Gradients are reduced over the batch in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace frmi {

constexpr int MLP_IN = 16, MLP_H = 64;
constexpr int MLP_OW1 = 0, MLP_OB1 = MLP_OW1 + MLP_H * MLP_IN, MLP_OW2 = MLP_OB1 + MLP_H,
              MLP_OB2 = MLP_OW2 + MLP_H * MLP_H, MLP_OW3 = MLP_OB2 + MLP_H, MLP_OB3 = MLP_OW3 + MLP_H,
              MLP_NP = MLP_OB3 + 1;

// Stage parameters and input scaling into LDS.
__device__ __forceinline__ void mlp_stage(const float* __restrict__ w, const float* __restrict__ scale, float* W,
                                          float* sc) {
  for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) W[i] = w[i];
  for (int i = threadIdx.x; i < 2 * MLP_IN; i += blockDim.x) sc[i] = scale[i];
  __syncthreads();
}

__device__ __forceinline__ float mlp_eval(const float* W, const float* sc, const float* x, float* h1, float* h2) {
  float xs[MLP_IN];
#pragma unroll
  for (int k = 0; k < MLP_IN; ++k) xs[k] = (x[k] - sc[k]) / sc[MLP_IN + k];
  for (int i = 0; i < MLP_H; ++i) {
    float a = W[MLP_OB1 + i];
#pragma unroll
    for (int k = 0; k < MLP_IN; ++k) a += W[MLP_OW1 + i * MLP_IN + k] * xs[k];
    h1[i] = tanhf(a);
  }
  float y = W[MLP_OB3];
  for (int j = 0; j < MLP_H; ++j) {
    float a = W[MLP_OB2 + j];
    for (int i = 0; i < MLP_H; ++i) a += W[MLP_OW2 + j * MLP_H + i] * h1[i];
    const float t = tanhf(a);
    if (h2) h2[j] = t;
    y += W[MLP_OW3 + j] * t;
  }
  return y;
}

// Inference for rows with flag != 0 (flag may be null: all rows).  With n_bits > 0
// the output is the predicted dyadic index k^ = 2^(n_bits y) instead of y.
__global__ void __launch_bounds__(256) mlp_forward(const float* __restrict__ w, const float* __restrict__ scale,
                                                   const float* __restrict__ x, const int32_t* __restrict__ flag,
                                                   int64_t n, int n_bits, float* __restrict__ y) {
  __shared__ float W[MLP_NP];
  __shared__ float sc[2 * MLP_IN];
  mlp_stage(w, scale, W, sc);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || (flag && flag[r] == 0)) return;
  float h1[MLP_H];
  const float out = mlp_eval(W, sc, x + r * MLP_IN, h1, nullptr);
  y[r] = n_bits > 0 ? exp2f((float)n_bits * out) : out;
}

// Per-sample forward and backward quantities of one batch (rows idx[0..B)).
// Scratch per sample s: xs[16] | h1[64] | h2[64] | d1[64] | d2[64] | dy
constexpr int MLP_SS = MLP_IN + 4 * MLP_H + 1;

__global__ void __launch_bounds__(256) mlp_fwd_bwd(const float* __restrict__ w, const float* __restrict__ scale,
                                                   const float* __restrict__ x, const float* __restrict__ t,
                                                   const int32_t* __restrict__ idx, int B,
                                                   float* __restrict__ scratch, float* __restrict__ sqerr) {
  __shared__ float W[MLP_NP];
  __shared__ float sc[2 * MLP_IN];
  mlp_stage(w, scale, W, sc);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const int64_t row = idx ? idx[s] : s;
  float* S = scratch + (int64_t)s * MLP_SS;
  float* xs = S;
  float* h1 = S + MLP_IN;
  float* h2 = h1 + MLP_H;
  float* d1 = h2 + MLP_H;
  float* d2 = d1 + MLP_H;
  float hh1[MLP_H], hh2[MLP_H];
  const float yv = mlp_eval(W, sc, x + row * MLP_IN, hh1, hh2);
#pragma unroll
  for (int k = 0; k < MLP_IN; ++k) xs[k] = (x[row * MLP_IN + k] - sc[k]) / sc[MLP_IN + k];
  const float r = yv - t[row];
  const float dy = 2.0f * r / (float)B;
  sqerr[s] = r * r;
  for (int j = 0; j < MLP_H; ++j) {
    h1[j] = hh1[j];
    h2[j] = hh2[j];
    d2[j] = dy * W[MLP_OW3 + j] * (1.0f - hh2[j] * hh2[j]);
  }
  for (int i = 0; i < MLP_H; ++i) {
    float a = 0;
    for (int j = 0; j < MLP_H; ++j) a += d2[j] * W[MLP_OW2 + j * MLP_H + i];
    d1[i] = a * (1.0f - hh1[i] * hh1[i]);
  }
  S[MLP_SS - 1] = dy;
}

// Gradient of every parameter: a fixed-order sum over the batch (thread per parameter).
__global__ void __launch_bounds__(256) mlp_grad_reduce(const float* __restrict__ scratch, int B,
                                                       const float* __restrict__ sqerr, float* __restrict__ grad,
                                                       float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == MLP_NP) {               // the loss
    float a = 0;
    for (int s = 0; s < B; ++s) a += sqerr[s];
    *loss = a / (float)B;
    return;
  }
  if (p > MLP_NP) return;
  float a = 0;
  for (int s = 0; s < B; ++s) {
    const float* S = scratch + (int64_t)s * MLP_SS;
    const float* xs = S;
    const float* h1 = S + MLP_IN;
    const float* h2 = h1 + MLP_H;
    const float* d1 = h2 + MLP_H;
    const float* d2 = d1 + MLP_H;
    const float dy = S[MLP_SS - 1];
    float g;
    if (p < MLP_OB1) g = d1[(p - MLP_OW1) / MLP_IN] * xs[(p - MLP_OW1) % MLP_IN];
    else if (p < MLP_OW2) g = d1[p - MLP_OB1];
    else if (p < MLP_OB2) g = d2[(p - MLP_OW2) / MLP_H] * h1[(p - MLP_OW2) % MLP_H];
    else if (p < MLP_OW3) g = d2[p - MLP_OB2];
    else if (p < MLP_OB3) g = dy * h2[p - MLP_OW3];
    else g = dy;
    a += g;
  }
  grad[p] = a;
}

// Adam (t is the 1-based step count).
__global__ void __launch_bounds__(256) mlp_adam(float* __restrict__ w, const float* __restrict__ g,
                                                float* __restrict__ m, float* __restrict__ v, int t, float lr,
                                                float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NP) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.0f - b1) * gi;
  const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)t));
  const float vh = vi / (1.0f - powf(b2, (float)t));
  w[p] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace frmi
