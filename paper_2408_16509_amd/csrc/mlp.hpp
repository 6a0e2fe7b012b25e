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
constexpr int MLP_FB_WAVES = 4;            // samples per block of mlp_fwd_bwd

// One wave per sample, lane j = hidden unit j: every dot product is the sequential sum the
// single-thread form takes (same terms, same order), so the values are those of
// mlp_eval.  The weights sit in LDS twice, W2 as stored (rows read by the backward pass:
// consecutive lanes, consecutive words) and transposed (W2^T and W1^T for the forward
// pass), so no access is a bank conflict.
__global__ void __launch_bounds__(64 * MLP_FB_WAVES) mlp_fwd_bwd(const float* __restrict__ w,
                                                                 const float* __restrict__ scale,
                                                                 const float* __restrict__ x,
                                                                 const float* __restrict__ t,
                                                                 const int32_t* __restrict__ idx, int B,
                                                                 float* __restrict__ scratch,
                                                                 float* __restrict__ sqerr) {
  __shared__ float W2[MLP_H * MLP_H], W2T[MLP_H * MLP_H], W1T[MLP_IN * MLP_H];
  __shared__ float BV[3 * MLP_H + 1];       // b1 | b2 | w3 | b3
  __shared__ float sc[2 * MLP_IN];
  __shared__ float H[MLP_FB_WAVES][3][MLP_H];   // per wave: h1 | h2 | d2
  for (int i = threadIdx.x; i < MLP_H * MLP_H; i += blockDim.x) {
    const float v = w[MLP_OW2 + i];
    W2[i] = v;
    W2T[(i % MLP_H) * MLP_H + i / MLP_H] = v;
  }
  for (int i = threadIdx.x; i < MLP_H * MLP_IN; i += blockDim.x) W1T[(i % MLP_IN) * MLP_H + i / MLP_IN] = w[MLP_OW1 + i];
  for (int i = threadIdx.x; i < MLP_H; i += blockDim.x) {
    BV[i] = w[MLP_OB1 + i];
    BV[MLP_H + i] = w[MLP_OB2 + i];
    BV[2 * MLP_H + i] = w[MLP_OW3 + i];
  }
  if (threadIdx.x == 0) BV[3 * MLP_H] = w[MLP_OB3];
  for (int i = threadIdx.x; i < 2 * MLP_IN; i += blockDim.x) sc[i] = scale[i];
  __syncthreads();
  // every wave passes the three barriers below; a wave past the batch computes nothing
  const int wv = threadIdx.x / 64, j = threadIdx.x % 64;
  const int s = blockIdx.x * MLP_FB_WAVES + wv;
  const bool valid = s < B;
  const int64_t row = valid ? (idx ? idx[s] : s) : 0;
  float xs[MLP_IN];
#pragma unroll
  for (int k = 0; k < MLP_IN; ++k) xs[k] = (x[row * MLP_IN + k] - sc[k]) / sc[MLP_IN + k];
  float a = BV[j];
#pragma unroll
  for (int k = 0; k < MLP_IN; ++k) a += W1T[k * MLP_H + j] * xs[k];
  const float h1 = tanhf(a);
  H[wv][0][j] = h1;
  __syncthreads();
  a = BV[MLP_H + j];
  for (int i = 0; i < MLP_H; ++i) a += W2T[i * MLP_H + j] * H[wv][0][i];
  const float h2 = tanhf(a);
  H[wv][1][j] = h2;
  __syncthreads();
  float y = BV[3 * MLP_H];
  for (int i = 0; i < MLP_H; ++i) y += BV[2 * MLP_H + i] * H[wv][1][i];
  const float r = y - (valid ? t[row] : 0.0f);
  const float dy = 2.0f * r / (float)B;
  const float d2 = dy * BV[2 * MLP_H + j] * (1.0f - h2 * h2);
  H[wv][2][j] = d2;
  __syncthreads();
  a = 0;
  for (int i = 0; i < MLP_H; ++i) a += H[wv][2][i] * W2[i * MLP_H + j];
  const float d1 = a * (1.0f - h1 * h1);
  if (!valid) return;
  float* S = scratch + (int64_t)s * MLP_SS;
  if (j < MLP_IN) S[j] = xs[j];
  S[MLP_IN + j] = h1;
  S[MLP_IN + MLP_H + j] = h2;
  S[MLP_IN + 2 * MLP_H + j] = d1;
  S[MLP_IN + 3 * MLP_H + j] = d2;
  if (j == 0) {
    S[MLP_SS - 1] = dy;
    sqerr[s] = r * r;
  }
}

// Gradient of every parameter: a fixed-order sum over the batch (thread per parameter,
// 64-thread blocks so the 84 blocks spread over as many CUs).  Each parameter's term is a
// product of two per-sample quantities (or one of them alone: biases, b3), so the thread
// takes their two offsets within a sample's scratch once and walks the batch with them.
constexpr int MLP_GR_NT = 64;
__global__ void __launch_bounds__(MLP_GR_NT) mlp_grad_reduce(const float* __restrict__ scratch, int B,
                                                             const float* __restrict__ sqerr, float* __restrict__ grad,
                                                             float* __restrict__ loss) {
  const int p = blockIdx.x * MLP_GR_NT + threadIdx.x;
  if (p == MLP_NP) {               // the loss
    float a = 0;
    for (int s = 0; s < B; ++s) a += sqerr[s];
    *loss = a / (float)B;
    return;
  }
  if (p > MLP_NP) return;
  constexpr int XS = 0, H1 = MLP_IN, H2 = H1 + MLP_H, D1 = H2 + MLP_H, D2 = D1 + MLP_H, DY = MLP_SS - 1;
  int oa, ob = -1;                 // term = S[oa] * S[ob] (S[oa] alone when ob < 0)
  if (p < MLP_OB1) { oa = D1 + (p - MLP_OW1) / MLP_IN; ob = XS + (p - MLP_OW1) % MLP_IN; }
  else if (p < MLP_OW2) oa = D1 + (p - MLP_OB1);
  else if (p < MLP_OB2) { oa = D2 + (p - MLP_OW2) / MLP_H; ob = H1 + (p - MLP_OW2) % MLP_H; }
  else if (p < MLP_OW3) oa = D2 + (p - MLP_OB2);
  else if (p < MLP_OB3) { oa = DY; ob = H2 + (p - MLP_OW3); }
  else oa = DY;
  float a = 0;
  if (ob >= 0) {
    const float* A = scratch + oa;
    const float* Bp = scratch + ob;
#pragma unroll 8
    for (int s = 0; s < B; ++s) a += A[(int64_t)s * MLP_SS] * Bp[(int64_t)s * MLP_SS];
  } else {
    const float* A = scratch + oa;
#pragma unroll 8
    for (int s = 0; s < B; ++s) a += A[(int64_t)s * MLP_SS];
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
