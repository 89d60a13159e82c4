// Extension of a batch of right-hand sides (Section 3.2): the two matrix
// products of the least-squares extension as FP64 MFMA GEMMs, then the
// Chebyshev step (Section 4.1) and the evaluation at the target leaves for
// eight right-hand sides of a cut leaf per work-group.
//
//   A1, per cut leaf i:  F_G = P_i F_I        (nG x nrhs; P_i is nG x N_I and is
//                                              read once per 64 right-hand sides)
//   A2, all at once:     G = A_{Xbar,G} F_G   (Kbar^2 x (ncut nrhs); the universal
//                                              operator is shared by every column)
//
// Both are computed transposed, so that the right-hand sides (A1) and the
// (leaf, right-hand side) columns (A2) index the MFMA's A rows and every
// output tile stores 16 contiguous values per lane group:
// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16] and the
// outputs D[(l/16) + 4r][l%16], r = 0..3.
#include <hip/hip_runtime.h>

#include <string>

#include "vfx_internal.h"

namespace vfx {

namespace {

typedef double xb_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ xb_d4 xb_mfma(double a, double b, xb_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A1: work-group (cut leaf c, block of 64 right-hand sides); wave w takes the
// 16 right-hand sides 64 blockIdx.y + 16 w + (0..15) and all NRT row tiles of
// P_i.  A operand: F_I^T (right-hand side x interior index: the gathered
// samples), B operand: P_i^T (interior index x row).  fg[(c nrhs + r) nG + row].
template <int NRT>
__global__ void __launch_bounds__(256) k_ext_a1(int nG, int nX, const int* __restrict__ pinv_ptr,
                                                const uint16_t* __restrict__ pinv_idx,
                                                const double* __restrict__ pinv_val, const double* __restrict__ f_cut,
                                                long sfc, int nrhs, double* __restrict__ fg) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int off = pinv_ptr[c], ni = pinv_ptr[c + 1] - off;
  const int r_a = 64 * blockIdx.y + 16 * w + li;  // this lane's A row (right-hand side)
  const bool ok_a = r_a < nrhs;
  const double* fc = f_cut + (size_t)(ok_a ? r_a : 0) * sfc + (size_t)c * nX;
  const double* P = pinv_val + (size_t)off * nG;
  const uint16_t* ix = pinv_idx + off;
  xb_d4 acc[NRT];
#pragma unroll
  for (int t = 0; t < NRT; ++t) acc[t] = xb_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k = 0; k < ni; k += 4) {
    const int kq = k + lk;
    const bool ok = kq < ni;
    const double a = (ok && ok_a) ? fc[ix[kq]] : 0.0;
#pragma unroll
    for (int t = 0; t < NRT; ++t) {
      const int row = 16 * t + li;
      const double b = (ok && row < nG) ? P[(size_t)row * ni + kq] : 0.0;
      acc[t] = xb_mfma(a, b, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NRT; ++t) {
    const int row = 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rhs = 64 * blockIdx.y + 16 * w + lk + 4 * r;
      if (rhs < nrhs && row < nG) fg[((size_t)c * nrhs + rhs) * nG + row] = acc[t][r];
    }
  }
}

// A2: wave w of work-group b takes the 16 columns 64 b + 16 w + (0..15) of
// F_G and all NAT tiles of the Sbar grid.  A operand: F_G^T (column x
// stencil row), B operand: A_{Xbar,G}^T (stencil row x grid point; stored
// that way).  g[col Kb2 + a].
template <int NAT>
__global__ void __launch_bounds__(256) k_ext_a2(int nG, int Kb2, long cols, const double* __restrict__ fg,
                                                const double* __restrict__ AbarT, double* __restrict__ g) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const long col0 = 64L * blockIdx.x + 16 * w;
  const long col_a = col0 + li;
  const bool ok_a = col_a < cols;
  const double* fr = fg + (size_t)(ok_a ? col_a : 0) * nG;
  xb_d4 acc[NAT];
#pragma unroll
  for (int t = 0; t < NAT; ++t) acc[t] = xb_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (int k = 0; k < nG; k += 4) {
    const int kq = k + lk;
    const bool ok = kq < nG;
    const double a = (ok && ok_a) ? fr[kq] : 0.0;
#pragma unroll
    for (int t = 0; t < NAT; ++t) {
      const int ai = 16 * t + li;
      const double b = (ok && ai < Kb2) ? AbarT[(size_t)kq * Kb2 + ai] : 0.0;
      acc[t] = xb_mfma(a, b, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NAT; ++t) {
    const int ai = 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long col = col0 + lk + 4 * r;
      if (col < cols && ai < Kb2) g[(size_t)col * Kb2 + ai] = acc[t][r];
    }
  }
}

// The rest of the extension for RB right-hand sides of one cut leaf per
// work-group: the Sbar-grid values (given data, else A2's), the truncated
// Chebyshev coefficients c = C g C^T (total order < Kbar) and their values
// at the K x K nodes of every target leaf of the cut leaf.  The target
// geometry, C and the node positions are shared by the RB right-hand sides.
constexpr int kEvalRB = 8;
constexpr int kEvalMaxK = 16, kEvalMaxKb2 = 256;

__global__ void __launch_bounds__(256) k_ext_eval(int K, int Kb, int nX, const int* __restrict__ ext_ptr,
                                                  const int* __restrict__ ext_tgt, const double* __restrict__ ext_geo,
                                                  const double* __restrict__ t, const double* __restrict__ cbar,
                                                  const uint8_t* __restrict__ sbar_given,
                                                  const double* __restrict__ f_cut, long sfc,
                                                  const double* __restrict__ g_pre, double* __restrict__ fe, long sfe,
                                                  int nrhs) {
  __shared__ double s_cb[kEvalMaxKb2];
  __shared__ double s_g[kEvalRB * kEvalMaxKb2];
  __shared__ double s_tmp[kEvalRB * kEvalMaxKb2];  // C g, then the evaluation's partial products
  __shared__ double s_coef[kEvalRB * kEvalMaxKb2];
  __shared__ double s_Ex[kEvalMaxK * kEvalMaxK], s_Ey[kEvalMaxK * kEvalMaxK];
  __shared__ double s_t[kEvalMaxK];
  const int c = blockIdx.x, r0 = kEvalRB * blockIdx.y, nr = min(kEvalRB, nrhs - r0);
  const int tid = threadIdx.x, n = K * K, Kb2 = Kb * Kb;
  if (tid < Kb2) s_cb[tid] = cbar[tid];
  if (tid < K) s_t[tid] = t[tid];
  for (int e = tid; e < nr * Kb2; e += blockDim.x) {
    const int r = e / Kb2, a = e - r * Kb2;
    s_g[e] = sbar_given[(size_t)c * Kb2 + a] ? f_cut[(size_t)(r0 + r) * sfc + (size_t)c * nX + n + a]
                                             : g_pre[((size_t)c * nrhs + r0 + r) * Kb2 + a];
  }
  __syncthreads();
  for (int e = tid; e < nr * Kb2; e += blockDim.x) {  // tmp = C g
    const int r = e / Kb2, q = e - r * Kb2, m = q / Kb, j = q - m * Kb;
    const double* g = s_g + r * Kb2;
    double acc = 0.0;
    for (int i = 0; i < Kb; ++i) acc += s_cb[m * Kb + i] * g[i * Kb + j];
    s_tmp[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < nr * Kb2; e += blockDim.x) {  // coef = tmp C^T, total order < Kbar
    const int r = e / Kb2, q = e - r * Kb2, m = q / Kb, nn = q - m * Kb;
    const double* tm = s_tmp + r * Kb2;
    double acc = 0.0;
    if (m + nn < Kb)
      for (int j = 0; j < Kb; ++j) acc += tm[m * Kb + j] * s_cb[nn * Kb + j];
    s_coef[e] = acc;
  }
  const int e0 = ext_ptr[c], ne = ext_ptr[c + 1] - e0;
  for (int q = 0; q < ne; ++q) {
    const int j = ext_tgt[e0 + q];
    const double ox = ext_geo[3 * (e0 + q)], oy = ext_geo[3 * (e0 + q) + 1], sc = ext_geo[3 * (e0 + q) + 2];
    __syncthreads();  // coef complete; the previous target's reads of s_Ex, s_Ey, s_tmp done
    if (tid < 2 * K) {
      const int a = tid % K;
      const bool isy = tid >= K;
      const double xi = (isy ? oy : ox) + sc * s_t[a];
      double* dst = (isy ? s_Ey : s_Ex) + a * Kb;
      double t0 = 1.0, t1 = xi;
      dst[0] = 1.0;
      if (Kb > 1) dst[1] = xi;
      for (int m = 2; m < Kb; ++m) {
        const double t2 = 2.0 * xi * t1 - t0;
        dst[m] = t2;
        t0 = t1;
        t1 = t2;
      }
    }
    __syncthreads();
    const int kbk = Kb * K;
    for (int e = tid; e < nr * kbk; e += blockDim.x) {  // per right-hand side: coef Ey^T (Kb x K)
      const int r = e / kbk, q2 = e - r * kbk, m = q2 / K, b = q2 - m * K;
      const double* cf = s_coef + r * Kb2;
      double acc = 0.0;
      for (int nn = 0; nn < Kb - m; ++nn) acc += cf[m * Kb + nn] * s_Ey[b * Kb + nn];
      s_tmp[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < nr * n; e += blockDim.x) {  // Ex (coef Ey^T): the K x K values
      const int r = e / n, idx = e - r * n, a = idx / K, b = idx - a * K;
      const double* tr = s_tmp + r * kbk;
      double acc = 0.0;
      for (int m = 0; m < Kb; ++m) acc += s_Ex[a * Kb + m] * tr[m * K + b];
      fe[(size_t)(r0 + r) * sfe + (size_t)j * n + idx] = acc;
    }
  }
}

}  // namespace

int launch_ext_eval(const Plan* p, const double* f_cut, double* fe, int nrhs, hipStream_t s, std::string& err) {
  const HostPlan& H = p->H;
  const DevicePlan& D = p->D;
  const Tables& T = p->ctx->T;
  if (H.ncut == 0) return VFX_OK;
  if (T.K > kEvalMaxK || T.Kbar * T.Kbar > kEvalMaxKb2 || T.Kbar * T.K > kEvalMaxKb2) {
    err = "batched extension: grid larger than the evaluation kernel's buffers";
    return VFX_EINVAL;
  }
  const long sfc = (long)H.ncut * T.nX, sfe = (long)H.L * T.n;
  hipLaunchKernelGGL(k_ext_eval, dim3(H.ncut, (nrhs + kEvalRB - 1) / kEvalRB), dim3(256), 0, s, T.K, T.Kbar, T.nX,
                     D.ext_ptr, D.ext_tgt, D.ext_geo, p->ctx->D.t, p->ctx->D.cbar, D.sbar_given, f_cut, sfc,
                     D.ext_g, fe, sfe, nrhs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("batched extension: ") + hipGetErrorString(e);
    return VFX_EHIP;
  }
  return VFX_OK;
}

int launch_ext_gemm(const Plan* p, const double* f_cut, int nrhs, hipStream_t s, std::string& err) {
  const HostPlan& H = p->H;
  const DevicePlan& D = p->D;
  const Tables& T = p->ctx->T;
  if (H.ncut == 0) return VFX_OK;
  if (!D.ext_fg || !D.ext_g || nrhs < kExtGemmMinRhs || nrhs > D.cap) {
    err = "batched extension: buffers missing for this batch size";
    return VFX_EINVAL;
  }
  const int nG = T.nG, Kb2 = T.Kbar * T.Kbar;
  const long sfc = (long)H.ncut * T.nX;
  const int nrt = (nG + 15) / 16, nat = (Kb2 + 15) / 16;
  if (nrt > 9 || nat > 16) {
    err = "batched extension: stencil or Sbar grid larger than the kernels' tiles";
    return VFX_EINVAL;
  }
  const dim3 g1(H.ncut, (nrhs + 63) / 64);
#define VFX_A1(N)                                                                                                   \
  case N:                                                                                                           \
    hipLaunchKernelGGL(k_ext_a1<N>, g1, dim3(256), 0, s, nG, T.nX, D.pinv_ptr, D.pinv_idx, D.pinv_val, f_cut, sfc, \
                       nrhs, D.ext_fg);                                                                             \
    break;
  switch (nrt) {
    VFX_A1(1) VFX_A1(2) VFX_A1(3) VFX_A1(4) VFX_A1(5) VFX_A1(6) VFX_A1(7) VFX_A1(8) VFX_A1(9)
  }
#undef VFX_A1
  const long cols = (long)H.ncut * nrhs;
  const dim3 g2((unsigned)((cols + 63) / 64));
  const DeviceTables& DT = p->ctx->D;
#define VFX_A2(N)                                                                                        \
  case N:                                                                                                \
    hipLaunchKernelGGL(k_ext_a2<N>, g2, dim3(256), 0, s, nG, Kb2, cols, D.ext_fg, DT.AbarT, D.ext_g); \
    break;
  switch (nat) {
    VFX_A2(1) VFX_A2(2) VFX_A2(3) VFX_A2(4) VFX_A2(5) VFX_A2(6) VFX_A2(7) VFX_A2(8) VFX_A2(9) VFX_A2(10)
    VFX_A2(11) VFX_A2(12) VFX_A2(13) VFX_A2(14) VFX_A2(15) VFX_A2(16)
  }
#undef VFX_A2
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("batched extension: ") + hipGetErrorString(e);
    return VFX_EHIP;
  }
  return VFX_OK;
}

}  // namespace vfx
