// Refinement classifier: a 64-64-64-1 MLP with GELU, trained in FP32 and
// evaluated in FP16 on the GPU.  Features are the last four rows of a leaf's
// 16 x 16 Chebyshev coefficient array; the logit says "refine".
//
// Parameters: one flat FP32 vector, W1 (64 x 64, [out][in]) at 0, b1 at 4096,
// W2 at 4160, b2 at 8256, w3 at 8320, b3 at 8384 (8385 values).
// GELU is the exact x Phi(x); the loss is the mean binary cross-entropy of
// the logits.  A work-group takes 32 samples: the two 64 x 64 weight
// matrices and the samples' activations live in LDS (rows padded to 65
// floats, so the 64 lanes of a wave reading one column hit distinct banks);
// thread (u, g) owns unit u for the samples g, g+4, ..., g+28.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>

#include "vfx_internal.h"

namespace vfx {

namespace {

constexpr int D = 64, S = 32, LDW = D + 1;
constexpr int OW1 = 0, OB1 = 4096, OW2 = 4160, OB2 = 8256, OW3 = 8320, OB3 = 8384;
constexpr int NPAR = 8385;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_prime(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

struct Tile {
  float W1[D * LDW], W2[D * LDW];
  float x[S * LDW], z1[S * LDW], a1[S * LDW], z2[S * LDW], a2[S * LDW];
  float logit[S];
};

// forward pass of samples s0..s0+ns-1 into the tile (weights already loaded)
__device__ void tile_forward(Tile& T, const float* __restrict__ th, const float* __restrict__ X, long s0, int ns) {
  const int t = threadIdx.x, u = t & 63, g = t >> 6;
  for (int s = g; s < S; s += 4)
    T.x[s * LDW + u] = s < ns ? X[(s0 + s) * D + u] : 0.0f;
  __syncthreads();
  const float b1 = th[OB1 + u], b2 = th[OB2 + u], w3 = th[OW3 + u];
  for (int s = g; s < S; s += 4) {
    float z = b1;
    for (int i = 0; i < D; ++i) z += T.W1[u * LDW + i] * T.x[s * LDW + i];
    T.z1[s * LDW + u] = z;
    T.a1[s * LDW + u] = gelu(z);
  }
  __syncthreads();
  for (int s = g; s < S; s += 4) {
    float z = b2;
    for (int i = 0; i < D; ++i) z += T.W2[u * LDW + i] * T.a1[s * LDW + i];
    T.z2[s * LDW + u] = z;
    const float a = gelu(z);
    T.a2[s * LDW + u] = a;
    // logit: sum over the 64 units (the lanes of this wave)
    float v = a * w3;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (u == 0) T.logit[s] = v + th[OB3];
  }
  __syncthreads();
}

__device__ void load_weights(Tile& T, const float* __restrict__ th) {
  for (int k = threadIdx.x; k < D * D; k += blockDim.x) {
    T.W1[(k >> 6) * LDW + (k & 63)] = th[OW1 + k];
    T.W2[(k >> 6) * LDW + (k & 63)] = th[OW2 + k];
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ th, const float* __restrict__ X, long B,
                                                     float* __restrict__ logits) {
  __shared__ Tile T;
  load_weights(T, th);
  for (long s0 = (long)blockIdx.x * S; s0 < B; s0 += (long)gridDim.x * S) {
    const int ns = (int)min((long)S, B - s0);
    tile_forward(T, th, X, s0, ns);
    if (threadIdx.x < ns) logits[s0 + threadIdx.x] = T.logit[threadIdx.x];
    __syncthreads();
  }
}

// per-tile partial gradient of the mean loss (1/B factor applied here); the
// partials of the tiles are added in tile order by k_mlp_reduce
__global__ void __launch_bounds__(256) k_mlp_grad_tiles(const float* __restrict__ th, const float* __restrict__ X,
                                                        const float* __restrict__ y, long B,
                                                        float* __restrict__ part) {
  __shared__ Tile T;
  __shared__ float ds[S];
  __shared__ float red[4 * D];
  load_weights(T, th);
  const long s0 = (long)blockIdx.x * S;
  const int ns = (int)min((long)S, B - s0);
  tile_forward(T, th, X, s0, ns);
  const int t = threadIdx.x, u = t & 63, g = t >> 6;
  float* P = part + (size_t)blockIdx.x * NPAR;
  if (t < S) ds[t] = t < ns ? (1.0f / (1.0f + expf(-T.logit[t])) - y[s0 + t]) / (float)B : 0.0f;
  __syncthreads();
  const float w3 = th[OW3 + u];
  // dz2 (in place of z2), dW3, db3
  float gw3 = 0.0f;
  for (int s = g; s < S; s += 4) {
    gw3 += ds[s] * T.a2[s * LDW + u];
    T.z2[s * LDW + u] = ds[s] * w3 * gelu_prime(T.z2[s * LDW + u]);
  }
  red[g * D + u] = gw3;
  __syncthreads();
  if (t < D) P[OW3 + t] = (red[t] + red[D + t]) + (red[2 * D + t] + red[3 * D + t]);
  if (t == 0) {
    float b = 0.0f;
    for (int s = 0; s < S; ++s) b += ds[s];
    P[OB3] = b;
  }
  // da1 = W2^T dz2, dz1 (in place of z1); thread (u = input unit i)
  for (int s = g; s < S; s += 4) {
    float a = 0.0f;
    for (int o = 0; o < D; ++o) a += T.W2[o * LDW + u] * T.z2[s * LDW + o];
    T.z1[s * LDW + u] = a * gelu_prime(T.z1[s * LDW + u]);
  }
  __syncthreads();
  // dW2[u][i] = sum_s dz2[s][u] a1[s][i]; dW1[u][i] = sum_s dz1[s][u] x[s][i]
  // thread (u, g) takes the columns i = 16 g .. 16 g + 15 over all samples
  for (int layer = 0; layer < 2; ++layer) {
    const float* dz = layer == 0 ? T.z2 : T.z1;
    const float* in = layer == 0 ? T.a1 : T.x;
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0f;
    float db = 0.0f;
    for (int s = 0; s < S; ++s) {
      const float d = dz[s * LDW + u];
      db += d;
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] += d * in[s * LDW + 16 * g + k];
    }
    const int OW = layer == 0 ? OW2 : OW1, OB = layer == 0 ? OB2 : OB1;
#pragma unroll
    for (int k = 0; k < 16; ++k) P[OW + u * D + 16 * g + k] = acc[k];
    if (g == 0) P[OB + u] = db;
  }
}

__global__ void k_mlp_reduce(int ntiles, const float* __restrict__ part, float* __restrict__ grad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NPAR) return;
  float a0 = 0.0f, a1 = 0.0f;
  int j = 0;
  for (; j + 1 < ntiles; j += 2) {
    a0 += part[(size_t)j * NPAR + k];
    a1 += part[(size_t)(j + 1) * NPAR + k];
  }
  if (j < ntiles) a0 += part[(size_t)j * NPAR + k];
  grad[k] = a0 + a1;
}

__global__ void k_mlp_adam(float* __restrict__ th, const float* __restrict__ grad, float* __restrict__ m,
                           float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NPAR) return;
  const float gk = grad[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  th[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void k_to_f16(long n, const float* __restrict__ a, __half* __restrict__ h) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    h[i] = __float2half(a[i]);
}

// FP16 inference: weights, inputs and activations stored as FP16, products
// accumulated in FP32
__global__ void __launch_bounds__(256) k_mlp_infer_f16(const __half* __restrict__ th, const __half* __restrict__ X,
                                                       long B, float* __restrict__ logits) {
  __shared__ __half W1[D * LDW], W2[D * LDW];
  __shared__ __half x[S * LDW], a1[S * LDW];
  for (int k = threadIdx.x; k < D * D; k += blockDim.x) {
    W1[(k >> 6) * LDW + (k & 63)] = th[OW1 + k];
    W2[(k >> 6) * LDW + (k & 63)] = th[OW2 + k];
  }
  __syncthreads();
  const int t = threadIdx.x, u = t & 63, g = t >> 6;
  const float b1 = __half2float(th[OB1 + u]), b2 = __half2float(th[OB2 + u]), w3 = __half2float(th[OW3 + u]);
  const float b3 = __half2float(th[OB3]);
  for (long s0 = (long)blockIdx.x * S; s0 < B; s0 += (long)gridDim.x * S) {
    const int ns = (int)min((long)S, B - s0);
    for (int s = g; s < S; s += 4) x[s * LDW + u] = s < ns ? X[(s0 + s) * D + u] : __float2half(0.0f);
    __syncthreads();
    for (int s = g; s < S; s += 4) {
      float z = b1;
      for (int i = 0; i < D; ++i) z += __half2float(W1[u * LDW + i]) * __half2float(x[s * LDW + i]);
      a1[s * LDW + u] = __float2half(gelu(z));
    }
    __syncthreads();
    for (int s = g; s < S; s += 4) {
      float z = b2;
      for (int i = 0; i < D; ++i) z += __half2float(W2[u * LDW + i]) * __half2float(a1[s * LDW + i]);
      float v = __half2float(__float2half(gelu(z))) * w3;
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (u == 0 && s < ns) logits[s0 + s] = v + b3;
    }
    __syncthreads();
  }
}

}  // namespace

int mlp_param_count() { return NPAR; }

int mlp_forward(const float* th, const float* X, long B, float* logits, hipStream_t s) {
  if (B <= 0) return VFX_OK;
  const int grid = (int)std::min<long>((B + S - 1) / S, 2048);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, s, th, X, B, logits);
  return hipGetLastError() == hipSuccess ? VFX_OK : VFX_EHIP;
}

long mlp_grad_work(long B) { return ((B + S - 1) / S) * (long)NPAR; }

int mlp_grad(const float* th, const float* X, const float* y, long B, float* grad, float* work, hipStream_t s) {
  if (B <= 0) return VFX_EINVAL;
  const int ntiles = (int)((B + S - 1) / S);
  hipLaunchKernelGGL(k_mlp_grad_tiles, dim3(ntiles), dim3(256), 0, s, th, X, y, B, work);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NPAR + 255) / 256), dim3(256), 0, s, ntiles, work, grad);
  return hipGetLastError() == hipSuccess ? VFX_OK : VFX_EHIP;
}

int mlp_adam(float* th, const float* grad, float* m, float* v, int step, float lr, float b1, float b2, float eps,
             hipStream_t s) {
  if (step < 1) return VFX_EINVAL;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, th, grad, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? VFX_OK : VFX_EHIP;
}

int mlp_to_f16(const float* a, uint16_t* h, long n, hipStream_t s) {
  if (n <= 0) return VFX_OK;
  const int grid = (int)std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_to_f16, dim3(grid), dim3(256), 0, s, n, a, (__half*)h);
  return hipGetLastError() == hipSuccess ? VFX_OK : VFX_EHIP;
}

int mlp_infer_f16(const uint16_t* th, const uint16_t* X, long B, float* logits, hipStream_t s) {
  if (B <= 0) return VFX_OK;
  const int grid = (int)std::min<long>((B + S - 1) / S, 2048);
  hipLaunchKernelGGL(k_mlp_infer_f16, dim3(grid), dim3(256), 0, s, (const __half*)th, (const __half*)X, B, logits);
  return hipGetLastError() == hipSuccess ? VFX_OK : VFX_EHIP;
}

}  // namespace vfx
