// Learned per-source r_max: source features, a 7 -> 64 -> 64 -> 1 GELU MLP
// (FP32 training forward/backward, Adam, BF16 inference) and the mapping of
// its output to r_max. The eps guarantee of Algorithm 2 (Lemma 2) holds for
// any r_max, so a learned r_max changes cost only, never correctness.
//
// Parameter vector (FORA_MLP_PARAMS floats):
//   mu[7], sigma[7]        feature standardisation (not trained)
//   W1[64][7], b1[64], W2[64][64], b2[64], W3[64], b3
// y = W3 . gelu(W2 gelu(W1 x' + b1) + b2) + b3, x' = (x - mu) / sigma,
// gelu(z) = z * Phi(z) with the normal CDF written through erf.
#include "internal.h"
#include "scan.h"

namespace fora {

constexpr int kIn = 7, kH = 64;
constexpr int kMu = 0, kSig = 7, kW1 = 14, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH,
              kB2 = kW2 + kH * kH, kW3 = kB2 + kH, kB3 = kW3 + kH, kParams = kB3 + 1;
static_assert(kParams == FORA_MLP_PARAMS, "parameter layout");
constexpr int kTrainable = kParams - kW1;
constexpr int kActs = 2 * kH;  // saved pre-activations z1, z2 per sample

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// ---- features --------------------------------------------------------------
// One wavefront per source s. f0 = ln d(s); f1 = ln sum_{u in N(s)} d(u);
// f2 = residue mass on the next frontier after the first synchronous round at
// r_max* (each out-neighbour u holds (1-alpha)/d(s); it counts when that
// exceeds r_max* d(u); 0 if s itself is not pushed); f3 = ln n; f4 = ln m;
// f5 = alpha; f6 = eps.
__global__ __launch_bounds__(256) void k_features(const int32_t* __restrict__ srcs, int count,
                                                  const int2* __restrict__ info,
                                                  const int32_t* __restrict__ colidx, int n,
                                                  int64_t m, double alpha, double eps,
                                                  double rmax, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= count) return;  // uniform per wave
  const int s = srcs[w];
  if (s < 0 || s >= n) {  // not a node: NaN features (the predictor then falls back)
    if (lane < kIn) out[(size_t)w * kIn + lane] = __int_as_float(0x7fc00000);
    return;
  }
  const int2 si = info[s];
  const double share = (1.0 - alpha) / (double)si.y;
  const bool pushed = 1.0 > rmax * (double)si.y;
  double vol = 0.0, mass = 0.0;
  for (int k = lane; k < si.y; k += 64) {
    const int d = info[colidx[(int64_t)si.x + k]].y;
    vol += (double)d;
    if (pushed && share > rmax * (double)d) mass += share;
  }
  vol = wave_sum(vol);
  mass = wave_sum(mass);
  if (lane == 0) {
    float* f = out + (size_t)w * kIn;
    f[0] = (float)log((double)si.y);
    f[1] = (float)log(vol);
    f[2] = (float)mass;
    f[3] = (float)log((double)n);
    f[4] = (float)log((double)m);
    f[5] = (float)alpha;
    f[6] = (float)eps;
  }
}

hipError_t launch_features(const GraphDev& g, int count, const int32_t* srcs, double alpha,
                           double eps, double rmax, float* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int blocks = (count + 3) / 4;
  k_features<<<blocks, 256, 0, s>>>(srcs, count, g.info, g.colidx, g.n, g.m, alpha, eps, rmax,
                                    out);
  return hipGetLastError();
}

// ---- FP32 forward ----------------------------------------------------------
// One thread per sample; the parameters sit in LDS. Optionally saves z1, z2.
__global__ __launch_bounds__(256) void k_mlp_forward(int count, const float* __restrict__ x,
                                                     const float* __restrict__ params,
                                                     float* __restrict__ y,
                                                     float* __restrict__ acts) {
  __shared__ float p[kParams];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) p[i] = params[i];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float xs[kIn];
  for (int k = 0; k < kIn; ++k) xs[k] = (x[(size_t)i * kIn + k] - p[kMu + k]) / p[kSig + k];
  float h1[kH];
  for (int j = 0; j < kH; ++j) {
    float z = p[kB1 + j];
    for (int k = 0; k < kIn; ++k) z += p[kW1 + j * kIn + k] * xs[k];
    if (acts) acts[(size_t)i * kActs + j] = z;
    h1[j] = gelu(z);
  }
  float out = p[kB3];
  for (int j = 0; j < kH; ++j) {
    float z = p[kB2 + j];
    for (int k = 0; k < kH; ++k) z += p[kW2 + j * kH + k] * h1[k];
    if (acts) acts[(size_t)i * kActs + kH + j] = z;
    out += p[kW3 + j] * gelu(z);
  }
  y[i] = out;
}

// ---- backward ----------------------------------------------------------------
// Loss L = (1/N) sum_i (y_i - t_i)^2. Per sample: d3 = 2 (y - t) / N,
// d2_j = W3_j d3 gelu'(z2_j), d1_k = sum_j W2_jk d2_j gelu'(z1_k).
// Stores d1, d2, d3 and the layer inputs; the weight gradients are outer
// products summed over samples by k_mlp_grad (fixed order, no atomics).
constexpr int kDelta = 2 * kH + 1;
__global__ __launch_bounds__(256) void k_mlp_delta(int count, const float* __restrict__ params,
                                                   const float* __restrict__ acts,
                                                   const float* __restrict__ y,
                                                   const float* __restrict__ target,
                                                   float* __restrict__ delta,
                                                   float* __restrict__ loss_part) {
  __shared__ float p[kParams];
  __shared__ float s_tmp[4];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) p[i] = params[i];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float err2 = 0.0f;
  if (i < count) {
    const float e = y[i] - target[i];
    err2 = e * e;
    const float d3 = 2.0f * e / (float)count;
    const float* z = acts + (size_t)i * kActs;
    float* d = delta + (size_t)i * kDelta;
    float d2[kH];
    for (int j = 0; j < kH; ++j) {
      d2[j] = p[kW3 + j] * d3 * gelu_grad(z[kH + j]);
      d[kH + j] = d2[j];
    }
    for (int k = 0; k < kH; ++k) {
      float acc = 0.0f;
      for (int j = 0; j < kH; ++j) acc += p[kW2 + j * kH + k] * d2[j];
      d[k] = acc * gelu_grad(z[k]);
    }
    d[2 * kH] = d3;
  }
  const float s = block_sum(err2, s_tmp);
  if (threadIdx.x == 0) loss_part[blockIdx.x] = s;
}

// One thread per trainable parameter: sum over samples in sample order.
__global__ __launch_bounds__(256) void k_mlp_grad(int count, const float* __restrict__ x,
                                                  const float* __restrict__ params,
                                                  const float* __restrict__ acts,
                                                  const float* __restrict__ delta,
                                                  float* __restrict__ grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;  // trainable index
  if (q >= kTrainable) return;
  const int pidx = kW1 + q;
  float acc = 0.0f;
  if (pidx < kB1) {  // W1[j][k]: d1_j * x'_k
    const int j = (pidx - kW1) / kIn, k = (pidx - kW1) % kIn;
    const float mu = params[kMu + k], sg = params[kSig + k];
    for (int i = 0; i < count; ++i)
      acc += delta[(size_t)i * kDelta + j] * ((x[(size_t)i * kIn + k] - mu) / sg);
  } else if (pidx < kW2) {  // b1[j]
    const int j = pidx - kB1;
    for (int i = 0; i < count; ++i) acc += delta[(size_t)i * kDelta + j];
  } else if (pidx < kB2) {  // W2[j][k]: d2_j * gelu(z1_k)
    const int j = (pidx - kW2) / kH, k = (pidx - kW2) % kH;
    for (int i = 0; i < count; ++i)
      acc += delta[(size_t)i * kDelta + kH + j] * gelu(acts[(size_t)i * kActs + k]);
  } else if (pidx < kW3) {  // b2[j]
    const int j = pidx - kB2;
    for (int i = 0; i < count; ++i) acc += delta[(size_t)i * kDelta + kH + j];
  } else if (pidx < kB3) {  // W3[j]: d3 * gelu(z2_j)
    const int j = pidx - kW3;
    for (int i = 0; i < count; ++i)
      acc += delta[(size_t)i * kDelta + 2 * kH] * gelu(acts[(size_t)i * kActs + kH + j]);
  } else {  // b3
    for (int i = 0; i < count; ++i) acc += delta[(size_t)i * kDelta + 2 * kH];
  }
  grad[pidx] = acc;
}

__global__ void k_loss_sum(const float* part, int nparts, int count, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < nparts; ++i) s += part[i];
    loss[0] = s / (float)count;
  }
}

// Adam (Kingma & Ba), bias-corrected, on the trainable part only.
__global__ void k_adam(float* params, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, int step) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kTrainable) return;
  const int i = kW1 + q;
  const float g = grad[i];
  m[i] = b1 * m[i] + (1.0f - b1) * g;
  v[i] = b2 * v[i] + (1.0f - b2) * g * g;
  const float mh = m[i] / (1.0f - powf(b1, (float)step));
  const float vh = v[i] / (1.0f - powf(b2, (float)step));
  params[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ---- BF16 inference ----------------------------------------------------------
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void k_to_bf16(int count, const float* in, uint16_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = to_bf16(in[i]);
}

// Weights, standardised inputs and hidden activations rounded to BF16;
// products accumulated in FP32.
__global__ __launch_bounds__(256) void k_mlp_forward_bf16(int count, const float* __restrict__ x,
                                                          const uint16_t* __restrict__ pb,
                                                          float* __restrict__ y) {
  __shared__ float p[kParams];
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) p[i] = from_bf16(pb[i]);
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float xs[kIn];
  for (int k = 0; k < kIn; ++k)
    xs[k] = from_bf16(to_bf16((x[(size_t)i * kIn + k] - p[kMu + k]) / p[kSig + k]));
  float h1[kH];
  for (int j = 0; j < kH; ++j) {
    float z = p[kB1 + j];
    for (int k = 0; k < kIn; ++k) z += p[kW1 + j * kIn + k] * xs[k];
    h1[j] = from_bf16(to_bf16(gelu(z)));
  }
  float out = p[kB3];
  for (int j = 0; j < kH; ++j) {
    float z = p[kB2 + j];
    for (int k = 0; k < kH; ++k) z += p[kW2 + j * kH + k] * h1[k];
    out += p[kW3 + j] * from_bf16(to_bf16(gelu(z)));
  }
  y[i] = out;
}

// r_max = r_max* exp(y) if y is finite and within [lo, hi]; else r_max*.
__global__ void k_rmax_from_output(int count, const float* y, double rmax_star, double lo,
                                   double hi, double* out, int* fallbacks) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double v = (double)y[i];
  const bool ok = isfinite(v) && v >= lo && v <= hi;
  out[i] = ok ? rmax_star * exp(v) : rmax_star;
  if (!ok) atomicAdd(fallbacks, 1);
}

hipError_t launch_mlp_forward(int count, const float* x, const float* params, float* y,
                              float* acts, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_mlp_forward<<<(count + 255) / 256, 256, 0, s>>>(count, x, params, y, acts);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(int count, const float* x, const float* params, const float* acts,
                               const float* y, const float* target, float* grad, float* loss,
                               float* scratch, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int blocks = (count + 255) / 256;
  float* delta = scratch;
  float* part = scratch + (size_t)count * kDelta;
  k_mlp_delta<<<blocks, 256, 0, s>>>(count, params, acts, y, target, delta, part);
  k_mlp_grad<<<(kTrainable + 255) / 256, 256, 0, s>>>(count, x, params, acts, delta, grad);
  k_loss_sum<<<1, 64, 0, s>>>(part, blocks, count, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* params, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
  k_adam<<<(kTrainable + 255) / 256, 256, 0, s>>>(params, grad, m, v, lr, b1, b2, eps, step);
  return hipGetLastError();
}

hipError_t launch_to_bf16(int count, const float* in, uint16_t* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_to_bf16<<<(count + 255) / 256, 256, 0, s>>>(count, in, out);
  return hipGetLastError();
}

hipError_t launch_mlp_forward_bf16(int count, const float* x, const uint16_t* pb, float* y,
                                   hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_mlp_forward_bf16<<<(count + 255) / 256, 256, 0, s>>>(count, x, pb, y);
  return hipGetLastError();
}

hipError_t launch_rmax_from_output(int count, const float* y, double rmax_star, double lo,
                                   double hi, double* out, int* fallbacks, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_rmax_from_output<<<(count + 255) / 256, 256, 0, s>>>(count, y, rmax_star, lo, hi, out,
                                                        fallbacks);
  return hipGetLastError();
}

}  // namespace fora
