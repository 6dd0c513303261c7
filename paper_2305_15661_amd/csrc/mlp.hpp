// Warm-start network: y = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 on
// normalised inputs x = (mu - x_mean) / x_scale and outputs z = y_mean +
// y_scale * y, gelu(t) = t Phi(t) (erf form).  Training in FP32 with
// explicit forward and backward kernels (every reduction in a fixed order,
// so a training run is reproducible) and Adam; inference either in FP32 or
// with BF16 weights and activations on matrix cores (FP32 accumulation).
// Parameters are one flat FP32 array: per layer W [out][in] row-major, then b.
#pragma once
#include "mixed.hpp"

namespace ift {

IFT_DEV float gelu_f(float t) { return 0.5f * t * (1.f + erff(t * 0.70710678118654752f)); }
IFT_DEV float gelu_prime_f(float t) {
  return 0.5f * (1.f + erff(t * 0.70710678118654752f)) + t * 0.39894228040143268f * expf(-0.5f * t * t);
}

// A[n][o] = b[o] + sum_i W[o][i] H[n][i]; Hout[n][o] = gelu(A) (act) or A.
__global__ void k_mlp_fwd(const float* H, int in, const float* W, const float* b, int out, int N, float* A,
                          float* Hout, int act) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * out) return;
  const int n = (int)(t / out), o = (int)(t % out);
  float a = b[o];
  const float* h = H + (long long)n * in;
  const float* w = W + (long long)o * in;
  for (int i = 0; i < in; ++i) a += w[i] * h[i];
  if (A) A[t] = a;
  Hout[t] = act ? gelu_f(a) : a;
}

// dY = 2 (Y - T) / (N out); per-block partial sums of (Y - T)^2.
__global__ __launch_bounds__(256) void k_mlp_loss(const float* Y, const float* T, long long cnt, float scale, float* dY,
                                                  double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < cnt; i += (long long)gridDim.x * 256) {
    const float d = Y[i] - T[i];
    dY[i] = 2.f * d * scale;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mlp_loss_final(const double* part, int nb, double scale, double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  *loss = s * scale;
}

// dA = dH * gelu'(A), elementwise (hidden layers).
__global__ void k_mlp_act_bwd(const float* A, float* dH, long long cnt) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) dH[t] *= gelu_prime_f(A[t]);
}

// dW[o][i] = sum_n dA[n][o] H[n][i] (i = in: db[o] = sum_n dA[n][o]) in two
// fixed-order stages: block (x, c) sums the samples of chunk c into
// part[c][o][i]; k_mlp_wgrad_sum adds the chunks in order.
constexpr int MLP_WCHUNKS = 32;

__global__ void k_mlp_wgrad(const float* dA, const float* H, int in, int out, int N, float* part) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int cols = out * (in + 1);
  if (t >= cols) return;
  const int o = t / (in + 1), i = t % (in + 1);
  const int c = blockIdx.y;
  const int per = (N + MLP_WCHUNKS - 1) / MLP_WCHUNKS;
  const int n0 = c * per, n1 = min(N, n0 + per);
  float s = 0.f;
  if (i < in)
    for (int n = n0; n < n1; ++n) s += dA[(long long)n * out + o] * H[(long long)n * in + i];
  else
    for (int n = n0; n < n1; ++n) s += dA[(long long)n * out + o];
  part[(long long)c * cols + t] = s;
}

__global__ void k_mlp_wgrad_sum(const float* part, int in, int out, float* dW, float* db) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int cols = out * (in + 1);
  if (t >= cols) return;
  float s = 0.f;
  for (int c = 0; c < MLP_WCHUNKS; ++c) s += part[(long long)c * cols + t];
  const int o = t / (in + 1), i = t % (in + 1);
  if (i < in) dW[(long long)o * in + i] = s;
  else db[o] = s;
}

// dH[n][i] = sum_o dA[n][o] W[o][i].
__global__ void k_mlp_xgrad(const float* dA, const float* W, int in, int out, int N, float* dH) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * in) return;
  const int n = (int)(t / in), i = (int)(t % in);
  float s = 0.f;
  for (int o = 0; o < out; ++o) s += dA[(long long)n * out + o] * W[(long long)o * in + i];
  dH[t] = s;
}

// Adam: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(float* p, const float* g, float* m, float* v, int cnt, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// x = (mu - x_mean) / x_scale in FP32; optional target y = (z - y_mean) / y_scale.
__global__ void k_mlp_normalize(const double* mu, const double* z, int N, int in, int out, const double* xm,
                                const double* xs, const double* ym, const double* ys, float* X, float* T) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long long)N * in) {
    const int i = (int)(t % in);
    X[t] = float((mu[t] - xm[i]) / xs[i]);
  }
  if (z && t < (long long)N * out) {
    const int o = (int)(t % out);
    T[t] = float((z[t] - ym[o]) / ys[o]);
  }
}

__global__ void k_mlp_denormalize(const float* Y, int N, int out, const double* ym, const double* ys, double* z) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * out) return;
  const int o = (int)(t % out);
  z[t] = ym[o] + ys[o] * double(Y[t]);
}

// One layer on BF16 matrix cores: one wave per 16 x 16 tile of the output
// [N][out] (samples x units), k over the inputs in steps of 16 (zero past
// `in`); weights and activations rounded to BF16, FP32 accumulation.
// Lane l supplies A[l%16][4 (l/16) + t] = H[row][k], B[4 (l/16) + t][l%16]
// = W[col][k]; register v holds sample 4 (l/16) + v of unit l%16.
__global__ __launch_bounds__(64) void k_mlp_fwd_bf16(const float* H, int in, const float* W, const float* b, int out,
                                                      int N, float* Hout, int act) {
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * 16, c0 = blockIdx.y * 16;
  const int li = lane & 15, kq = lane >> 4;
  const int row = min(r0 + li, N - 1), col = min(c0 + li, out - 1);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < in; k0 += 16) {
    bf16x4 a, w;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + 4 * kq + t;
      const int kc = k < in ? k : in - 1;
      const float s = k < in ? 1.f : 0.f;
      a[t] = to_bf16(H[(long long)row * in + kc] * s);
      w[t] = to_bf16(W[(long long)col * in + kc] * s);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, w, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int n = r0 + 4 * kq + v, o = c0 + li;
    if (n < N && o < out) {
      const float x = acc[v] + b[o];
      Hout[(long long)n * out + o] = act ? gelu_f(x) : x;
    }
  }
}

}  // namespace ift
