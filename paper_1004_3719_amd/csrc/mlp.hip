// The learned format selector's network on the GPU: a 32 -> 64 -> 64 -> 6
// perceptron (ReLU hidden layers) predicting the log2 time of each storage
// format for one row block, with hand-written forward, backward and Adam
// kernels in FP32. Parameter layout: W1 (64x32 row-major), b1, W2 (64x64),
// b2, W3 (6x64), b3 -- 6,662 floats. Inputs are standardised with a per
// feature mean and scale stored with the parameters.
//
// Sizes are small (13 kFLOP per block), so every kernel keeps one sample (or
// one parameter) per thread; none of it is a dense contraction large enough
// for MFMA tiles to pay.
#include "host.h"
#include "mlp.h"

namespace ffx {

constexpr int NIN = 32, NH = 64, NOUT = 6;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NOUT * NH;
static_assert(OFF_B3 + NOUT == MLP_NPARAM, "parameter count");

// per-sample activations kept for the backward pass
constexpr int ACT = NIN + NH + NH + NH + NH + NOUT;  // x, z1, h1, z2, h2, out

__device__ inline void stage_params(const float* __restrict__ theta, float* sp) {
  for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) sp[i] = theta[i];
  __syncthreads();
}

// Forward pass of one sample; keeps activations when act != null.
__device__ inline void forward_one(const float* sp, const float* __restrict__ mean, const float* __restrict__ scale,
                                   const float* __restrict__ xin, float* out, float* act) {
  float x[NIN], h1[NH], h2[NH];
#pragma unroll
  for (int k = 0; k < NIN; ++k) x[k] = (xin[k] - mean[k]) * scale[k];
  for (int j = 0; j < NH; ++j) {
    float z = sp[OFF_B1 + j];
#pragma unroll
    for (int k = 0; k < NIN; ++k) z = fmaf(sp[OFF_W1 + j * NIN + k], x[k], z);
    h1[j] = fmaxf(z, 0.f);
    if (act) act[NIN + j] = z;
  }
  for (int j = 0; j < NH; ++j) {
    float z = sp[OFF_B2 + j];
    for (int k = 0; k < NH; ++k) z = fmaf(sp[OFF_W2 + j * NH + k], h1[k], z);
    h2[j] = fmaxf(z, 0.f);
    if (act) act[NIN + 2 * NH + j] = z;
  }
  for (int f = 0; f < NOUT; ++f) {
    float z = sp[OFF_B3 + f];
    for (int k = 0; k < NH; ++k) z = fmaf(sp[OFF_W3 + f * NH + k], h2[k], z);
    out[f] = z;
  }
  if (act) {
#pragma unroll
    for (int k = 0; k < NIN; ++k) act[k] = x[k];
    for (int j = 0; j < NH; ++j) act[NIN + NH + j] = h1[j];
    for (int j = 0; j < NH; ++j) act[NIN + 3 * NH + j] = h2[j];
    for (int f = 0; f < NOUT; ++f) act[NIN + 4 * NH + f] = out[f];
  }
}

__global__ __launch_bounds__(128) void k_mlp_predict(const float* __restrict__ theta, const float* __restrict__ mean,
                                                     const float* __restrict__ scale, const float* __restrict__ X,
                                                     int64_t n, float* __restrict__ out) {
  __shared__ float sp[MLP_NPARAM];
  stage_params(theta, sp);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float o[NOUT];
  forward_one(sp, mean, scale, X + i * NIN, o, nullptr);
  for (int f = 0; f < NOUT; ++f) out[i * NOUT + f] = o[f];
}

// forward with activations, then the per-sample output and hidden deltas:
// d[i] = (g_out[6], g_z2[64], g_z1[64]) with g_out = mask*(out - target)/n
constexpr int DEL = NOUT + NH + NH;
__global__ __launch_bounds__(128) void k_mlp_fwd_bwd(const float* __restrict__ theta, const float* __restrict__ mean,
                                                     const float* __restrict__ scale, const float* __restrict__ X,
                                                     const float* __restrict__ T, const float* __restrict__ M,
                                                     int64_t n, float* __restrict__ act, float* __restrict__ del,
                                                     float* __restrict__ sqerr) {
  __shared__ float sp[MLP_NPARAM];
  stage_params(theta, sp);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float o[NOUT];
  float* a = act + i * ACT;
  forward_one(sp, mean, scale, X + i * NIN, o, a);
  float go[NOUT], se = 0.f;
  for (int f = 0; f < NOUT; ++f) {
    float d = (o[f] - T[i * NOUT + f]) * M[i * NOUT + f];
    se += d * d;
    go[f] = d / (float)n;
  }
  sqerr[i] = se;
  float* dl = del + i * DEL;
  for (int f = 0; f < NOUT; ++f) dl[f] = go[f];
  float gz2[NH];
  for (int j = 0; j < NH; ++j) {
    float g = 0.f;
    for (int f = 0; f < NOUT; ++f) g = fmaf(go[f], sp[OFF_W3 + f * NH + j], g);
    gz2[j] = a[NIN + 2 * NH + j] > 0.f ? g : 0.f;
    dl[NOUT + j] = gz2[j];
  }
  for (int k = 0; k < NH; ++k) {
    float g = 0.f;
    for (int j = 0; j < NH; ++j) g = fmaf(gz2[j], sp[OFF_W2 + j * NH + k], g);
    dl[NOUT + NH + k] = a[NIN + k] > 0.f ? g : 0.f;
  }
}

// One thread per parameter: the sum over samples of delta x input.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ act, const float* __restrict__ del, int64_t n,
                                                  float* __restrict__ grad) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  int dcol, acol;  // delta column, activation column (-1: bias)
  if (p < OFF_B1) { dcol = NOUT + NH + p / NIN; acol = p % NIN; }
  else if (p < OFF_W2) { dcol = NOUT + NH + (p - OFF_B1); acol = -1; }
  else if (p < OFF_B2) { int q = p - OFF_W2; dcol = NOUT + q / NH; acol = NIN + NH + q % NH; }
  else if (p < OFF_W3) { dcol = NOUT + (p - OFF_B2); acol = -1; }
  else if (p < OFF_B3) { int q = p - OFF_W3; dcol = q / NH; acol = NIN + 3 * NH + q % NH; }
  else { dcol = p - OFF_B3; acol = -1; }
  float g = 0.f;
  for (int64_t i = 0; i < n; ++i) {
    float d = del[i * DEL + dcol];
    g = fmaf(d, acol < 0 ? 1.f : act[i * ACT + acol], g);
  }
  grad[p] = g;
}

__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  float gp = g[p];
  float mp = b1 * m[p] + (1.f - b1) * gp;
  float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  theta[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ void k_sum(const float* __restrict__ x, int64_t n, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t mlp_predict(const float* theta, const float* mean, const float* scale, const float* X, int64_t n, float* out,
                       hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_predict, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, theta, mean, scale, X, n,
                     out);
  return hipGetLastError();
}

hipError_t mlp_gradient(const float* theta, const float* mean, const float* scale, const float* X, const float* T,
                        const float* M, int64_t n, float* act, float* del, float* sqerr, float* grad, float* sse,
                        hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, theta, mean, scale, X, T, M,
                     n, act, del, sqerr);
  hipLaunchKernelGGL(k_mlp_grad, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, act, del, n, grad);
  if (sse) hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, sqerr, n, sse);
  return hipGetLastError();
}

hipError_t mlp_adam(float* theta, float* m, float* v, const float* g, float lr, int64_t t, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, theta, m, v, g, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

size_t mlp_act_floats() { return ACT; }
size_t mlp_del_floats() { return DEL; }

}  // namespace ffx
