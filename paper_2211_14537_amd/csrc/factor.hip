// Plan stage on the GPU: the per-cut-leaf least-squares operators
// P_i = A_{X^I,G}^+ (Section 3.2: the least-squares fit on the interior
// stencil points; the paper factors each cut square by QR), for every cut
// leaf at once, one work-group per cut leaf, in FP64:
//   1. M = A[X^I, :] (N_I x N_G), column-major in a scratch buffer;
//   2. Householder QR of M, reflectors kept below the diagonal;
//   3. one-sided Jacobi SVD of B = R^T (N_G x r, r = min(N_I, N_G)) in LDS,
//      round-robin pairs, rotations accumulated in W (r x r);
//   4. pinv(R) = B diag(1/sigma^2) W^T, singular values below 1e-13 sigma_max
//      dropped (the minimum-norm solution when N_I < N_G);
//   5. P_i = pinv(R) Q^T, formed as Q [pinv(R)^T; 0] by applying the
//      reflectors in reverse order, written as P_i (N_G x N_I row-major).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "vfx_internal.h"

#define VFX_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#call) + ": " + hipGetErrorString(e_);                 \
      return VFX_EHIP;                                                         \
    }                                                                          \
  } while (0)

namespace vfx {

namespace {

constexpr int kG = 66;          // support points handled (stencil degree <= 10)
constexpr int LDB = kG + 1;     // LDS column stride
constexpr double kCut = 1e-13;  // relative singular-value cut-off
constexpr int kMaxSweeps = 40;

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the work-group (256 threads); red: 4 doubles of LDS
__device__ double block_sum(double v, double* red) {
  v = wsum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_factor(int nG, const int* __restrict__ pinv_ptr,
                                                const uint16_t* __restrict__ pinv_idx, const double* __restrict__ A,
                                                double* __restrict__ ws, double* __restrict__ Pout) {
  __shared__ double sB[kG * LDB];  // B = R^T, column i at sB[i * LDB]
  __shared__ double sW[kG * LDB];  // rotations, column i at sW[i * LDB]
  __shared__ double tau[kG], rdiag[kG], sig2[kG];
  __shared__ double red[4];
  __shared__ double s_off[4];
  const int c = blockIdx.x;
  const int off = pinv_ptr[c], m = pinv_ptr[c + 1] - off;
  if (m == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* M = ws + (size_t)off * nG;    // column j at M + j*m
  double* Z = Pout + (size_t)off * nG;  // column t at Z + t*m (= row t of P_i)
  const int r = min(m, nG);
  // 1. gather
  for (int e = tid; e < m * nG; e += blockDim.x) {
    const int i = e % m, j = e / m;
    M[(size_t)j * m + i] = A[(size_t)pinv_idx[off + i] * nG + j];
  }
  __syncthreads();
  // 2. Householder QR
  for (int j = 0; j < r; ++j) {
    double part = 0.0;
    for (int i = j + tid; i < m; i += blockDim.x) part += M[(size_t)j * m + i] * M[(size_t)j * m + i];
    const double nrm2 = block_sum(part, red);
    if (tid == 0) {
      const double x0 = M[(size_t)j * m + j];
      const double nrm = sqrt(nrm2);
      const double alpha = x0 >= 0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vn2 = nrm2 - x0 * x0 + v0 * v0;
      tau[j] = vn2 > 0 ? 2.0 / vn2 : 0.0;
      rdiag[j] = nrm2 > 0 ? alpha : 0.0;
      M[(size_t)j * m + j] = v0;
    }
    __syncthreads();
    const double tj = tau[j];
    for (int cc = j + 1 + w; cc < nG; cc += 4) {
      double d = 0.0;
      for (int i = j + lane; i < m; i += 64) d += M[(size_t)j * m + i] * M[(size_t)cc * m + i];
      d = wsum(d) * tj;
      for (int i = j + lane; i < m; i += 64) M[(size_t)cc * m + i] -= d * M[(size_t)j * m + i];
    }
    __syncthreads();
  }
  // 3. B = R^T (column i of B = row i of R), W = I
  for (int e = tid; e < kG * kG; e += blockDim.x) {
    const int i = e / kG, t = e % kG;
    double b = 0.0;
    if (i < r && t < nG) b = (t == i) ? rdiag[i] : (t > i ? M[(size_t)t * m + i] : 0.0);
    sB[i * LDB + t] = b;
    sW[i * LDB + t] = (i == t && i < r) ? 1.0 : 0.0;
  }
  __syncthreads();
  // one-sided Jacobi on the r columns of B (round-robin pairs)
  const int np = (r + 1) & ~1;  // players, even
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    double offmax = 0.0;
    for (int rd = 0; rd < np - 1; ++rd) {
      for (int k = w; k < np / 2; k += 4) {
        const int a = k == 0 ? 0 : 1 + (rd + k - 1) % (np - 1);
        const int b = 1 + (rd + np - 1 - k - 1) % (np - 1);
        if (a >= r || b >= r) continue;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int t = lane; t < nG; t += 64) {
          const double x = sB[a * LDB + t], y = sB[b * LDB + t];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wsum(al);
        be = wsum(be);
        ga = wsum(ga);
        if (ga == 0.0 || al == 0.0 || be == 0.0) continue;
        const double rel = fabs(ga) / sqrt(al * be);
        offmax = fmax(offmax, rel);
        if (rel < 1e-16) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int t = lane; t < nG; t += 64) {
          const double x = sB[a * LDB + t], y = sB[b * LDB + t];
          sB[a * LDB + t] = cs * x - sn * y;
          sB[b * LDB + t] = sn * x + cs * y;
        }
        for (int t = lane; t < r; t += 64) {
          const double x = sW[a * LDB + t], y = sW[b * LDB + t];
          sW[a * LDB + t] = cs * x - sn * y;
          sW[b * LDB + t] = sn * x + cs * y;
        }
      }
      __syncthreads();
    }
    if (lane == 0) s_off[w] = offmax;
    __syncthreads();
    const double om = fmax(fmax(s_off[0], s_off[1]), fmax(s_off[2], s_off[3]));
    __syncthreads();
    if (om < 1e-15) break;
  }
  // 4. squared singular values, cut-off
  for (int i = w; i < r; i += 4) {
    double s = 0.0;
    for (int t = lane; t < nG; t += 64) s += sB[i * LDB + t] * sB[i * LDB + t];
    s = wsum(s);
    if (lane == 0) sig2[i] = s;
  }
  __syncthreads();
  double smax = 0.0;
  for (int i = 0; i < r; ++i) smax = fmax(smax, sig2[i]);
  // X = pinv(R)^T (r x nG): X[k][t] = sum_i W[k][i] B[t][i] / sig2[i] -> Z rows k < r
  for (int e = tid; e < nG * m; e += blockDim.x) {
    const int k = e % m, t = e / m;
    double x = 0.0;
    if (k < r)
      for (int i = 0; i < r; ++i)
        if (sig2[i] > kCut * kCut * smax) x += sW[i * LDB + k] * sB[i * LDB + t] / sig2[i];
    Z[(size_t)t * m + k] = x;
  }
  __syncthreads();
  // 5. Z = H_0 ... H_{r-1} Z
  for (int j = r - 1; j >= 0; --j) {
    const double tj = tau[j];
    for (int t = w; t < nG; t += 4) {
      double d = 0.0;
      for (int i = j + lane; i < m; i += 64) d += M[(size_t)j * m + i] * Z[(size_t)t * m + i];
      d = wsum(d) * tj;
      for (int i = j + lane; i < m; i += 64) Z[(size_t)t * m + i] -= d * M[(size_t)j * m + i];
    }
    __syncthreads();
  }
}

}  // namespace

int factor_gpu(Plan* p, hipStream_t s, std::string& err) {
  const HostPlan& H = p->H;
  DevicePlan& D = p->D;
  const Tables& T = p->ctx->T;
  if (T.nG > kG) {
    err = "the GPU factorisation supports at most 66 support points (stencil degree <= 10)";
    return VFX_EINVAL;
  }
  if (H.ncut == 0) {
    D.factored = true;
    return VFX_OK;
  }
  const size_t nv = (size_t)H.pinv_ptr[H.ncut] * T.nG;
  if (!D.fac_ws) VFX_HIP(hipMalloc((void**)&D.fac_ws, sizeof(double) * nv));
  hipLaunchKernelGGL(k_factor, dim3(H.ncut), dim3(256), 0, s, T.nG, D.pinv_ptr, D.pinv_idx, p->ctx->D.A, D.fac_ws,
                     D.pinv_val);
  VFX_HIP(hipGetLastError());
  D.factored = true;
  return VFX_OK;
}

}  // namespace vfx
