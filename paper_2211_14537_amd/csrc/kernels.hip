// Device side of the extension + volume FMM path (gfx950, FP64).
//
// Execution order on one stream (every output element has one writer, so no
// atomics are needed and results are bitwise reproducible):
//   extension    f^e = f on regular leaves, 0 on leaves outside every
//                extension list, and per cut leaf: f_G = P_i f_{X^I}; values on the Kbar grid of
//                Sbar (given data where interior); total-order Chebyshev
//                expansion; evaluation on every leaf of its extension list
//                (Sections 3.2 and 4.1)
//   p2m, m2m     multipole expansions, leaves then upward
//   m2l          local expansions from list 2 (M2L) and list 4 (P2L)
//   l2l          locals downward
//   near         list 1 by the precomputed tables
//   far          L2P of the local expansion and M2P of list 3
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "vfx_internal.h"

namespace vfx {

#define VFX_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#call) + ": " + hipGetErrorString(e_);                 \
      return VFX_EHIP;                                                         \
    }                                                                          \
  } while (0)

constexpr int kMaxX = 648;   // |X| for K, Kbar <= 16, deg <= 15
constexpr int kMaxG = 136;
constexpr int kMaxK = 16;
constexpr int kMaxKb = 16;
constexpr double kInv2Pi = 0.15915494309189533576888376337251436;
constexpr double kLn2 = 0.69314718055994530941723212145817657;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double box_side(double root, int level) { return ldexp(root, -level); }

// -------------------------------------------------------------------------
// Extension of one cut leaf per work-group (256 threads): f_G = P_i f_I
// (A1), values on the Kbar x Kbar grid of Sbar (given data at interior
// nodes, A_{Xbar,G} f_G elsewhere; A2), the total-order Chebyshev
// coefficients (A3) and their values on the K x K nodes of every target
// leaf.  Every global load whose address is known early is issued at the
// start (two waves: indices/geometry, then the data they point to), so the
// work-group's critical path holds few memory round trips.
constexpr int kExtTgtMax = 16;  // targets whose geometry is staged in LDS

// f^e of the leaves no extension list writes, 16-byte pieces e0, e0 +
// step, ... below e1 (piece e: right-hand side e / half, element 2 (e mod
// half)): f on regular leaves (fe_src 1), zero elsewhere (fe_src 0); list
// targets (fe_src 2) are left to their cut leaf's work-group, so every
// element has one writer.
__device__ __forceinline__ void fe_init_range(long e0, long e1, long step, int n, long half,
                                              const int8_t* __restrict__ fe_src, const double* __restrict__ f_leaf,
                                              double* __restrict__ fe, long sfe) {
  // four pieces per round, so their loads are in flight together
  for (long e = e0; e < e1; e += 4 * step) {
    long off[4];
    int src[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const long ek = e + k * step;
      const long r = ek / half, i = 2 * (ek - r * half);
      off[k] = r * sfe + i;
      src[k] = ek < e1 ? fe_src[i / n] : 2;
    }
    double2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = src[k] == 1 ? *(const double2*)(f_leaf + off[k]) : make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (src[k] != 2) *(double2*)(fe + off[k]) = v[k];
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_extension(
    int K, int Kb, int nX, int nG, const int* __restrict__ pinv_ptr, const uint16_t* __restrict__ pinv_idx,
    const double* __restrict__ pinv_val, const uint8_t* __restrict__ sbar_given, const int* __restrict__ ext_ptr,
    const int* __restrict__ ext_tgt, const double* __restrict__ ext_geo, const double* __restrict__ t,
    const double* __restrict__ AbarT, const double* __restrict__ cbar, const double* __restrict__ f_cut,
    double* __restrict__ fe, int nrhs, long sfc, long sfe, int ext_blocks, int L,
    const int8_t* __restrict__ fe_src, const double* __restrict__ f_leaf) {
  const long half = (long)L * K * K / 2, pieces = half * nrhs;
  if ((int)blockIdx.x >= ext_blocks) {
    // the work-groups past the cut leaves initialise f^e of the other
    // leaves, grid-stride (they take the slots the cut leaves free)
    const long nb = (long)(gridDim.x - ext_blocks) * blockDim.x;
    fe_init_range((long)(blockIdx.x - ext_blocks) * blockDim.x + threadIdx.x, pieces, nb, K * K, half, fe_src,
                  f_leaf, fe, sfe);
    return;
  }
  // consecutive work-groups take the right-hand sides of one cut leaf, so
  // its operator P_i is read from HBM once and reused from L2
  const int rhs = blockIdx.x % nrhs;
  f_cut += rhs * sfc;
  fe += rhs * sfe;
  __shared__ double s_fI[kMaxX];
  __shared__ double s_fG[kMaxG];
  __shared__ double s_cb[kMaxKb * kMaxKb];
  __shared__ double s_g[kMaxKb * kMaxKb];
  __shared__ double s_tmp[kMaxKb * kMaxKb];
  __shared__ double s_coef[kMaxKb * kMaxKb];
  __shared__ double s_Ex[kMaxK * kMaxKb];
  __shared__ double s_Ey[kMaxK * kMaxKb];
  __shared__ double s_t[kMaxK];
  __shared__ double s_geo[3 * kExtTgtMax];
  __shared__ int s_tg[kExtTgtMax];
  __shared__ uint8_t s_given[kMaxKb * kMaxKb];
  const int c = blockIdx.x / nrhs;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: row indices in scalar registers
  const int n = K * K, Kb2 = Kb * Kb;
  const int off = pinv_ptr[c], ni = pinv_ptr[c + 1] - off;
  const int e0 = ext_ptr[c], ne = ext_ptr[c + 1] - e0;
  const double* fc = f_cut + (size_t)c * nX;
  // first load wave: indices, flags, small tables, target geometry
  int idx0 = tid < ni ? pinv_idx[off + tid] : 0;
  int idx1 = tid + 256 < ni ? pinv_idx[off + tid + 256] : 0;
  const bool given = tid < Kb2 && sbar_given[(size_t)c * Kb2 + tid];
  if (tid < Kb2) s_cb[tid] = cbar[tid];
  if (tid < K) s_t[tid] = t[tid];
  if (tid < ne && tid < kExtTgtMax) {
    s_tg[tid] = ext_tgt[e0 + tid];
    s_geo[3 * tid] = ext_geo[3 * (e0 + tid)];
    s_geo[3 * tid + 1] = ext_geo[3 * (e0 + tid) + 1];
    s_geo[3 * tid + 2] = ext_geo[3 * (e0 + tid) + 2];
  }
  // second load wave: interior samples and the given Sbar-grid values
  if (tid < ni) s_fI[tid] = fc[idx0];
  if (tid + 256 < ni) s_fI[tid + 256] = fc[idx1];
  for (int q = tid + 512; q < ni; q += blockDim.x) s_fI[q] = fc[pinv_idx[off + q]];
  if (tid < Kb2) {
    s_given[tid] = given;
    if (given) s_g[tid] = fc[n + tid];
  }
  __syncthreads();
  // A1: f_G = P_i f_I  (P_i: nG x ni row-major).  Wave w takes rows
  // 16w..16w+15 in four passes of 4, lane l the columns l, l + 64, l + 128,
  // l + 192 (then l + 256, ... for ni > 256): one pass reads four whole rows
  // (ni <= 256), every load of a wave 512 contiguous bytes, 16 loads in
  // flight at once.  The 4 row partials are combined across the lanes by a
  // recursive-halving reduce-scatter over lane bits 1..0 (lane l ends with
  // row l & 3) and four plain butterfly steps over bits 2..5.  Rows >= 64
  // (a stencil degree above 10) use wave sums.  Few live registers keep six
  // work-groups per CU resident, so the operators of all cut leaves stream
  // at once; P_i is read once per execute, so its loads are non-temporal
  // (they do not displace the data the later kernels reuse).
  const double* P = pinv_val + (size_t)off * nG;
#pragma unroll 1
  for (int pass = 0; pass < 4; ++pass) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int r0 = 16 * wave + 4 * pass;
#pragma unroll 1
    for (int q = lane; q < ni; q += 256) {
      double f[4], p[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) f[j] = q + 64 * j < ni ? s_fI[q + 64 * j] : 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = min(r0 + r, nG - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          p[r][j] = q + 64 * j < ni ? __builtin_nontemporal_load(P + row * ni + q + 64 * j) : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double m = (r0 + r < nG) ? 1.0 : 0.0;
        acc[r] += m * (p[r][0] * f[0] + p[r][1] * f[1] + p[r][2] * f[2] + p[r][3] * f[3]);
      }
    }
#pragma unroll
    for (int s = 2; s >= 1; s >>= 1) {
      const bool up = (lane & s) != 0;
#pragma unroll
      for (int j = 0; j < s; ++j) {
        const double send = up ? acc[j] : acc[j + s];
        const double keep = up ? acc[j + s] : acc[j];
        acc[j] = keep + __shfl_xor(send, s, 64);
      }
    }
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) acc[0] += __shfl_xor(acc[0], o, 64);
    if (lane < 4 && r0 + lane < nG) s_fG[r0 + lane] = acc[0];
  }
  for (int r = 64 + wave; r < nG; r += blockDim.x / 64) {
    double a = 0.0;
    const double* pr = P + (size_t)r * ni;
    for (int q = lane; q < ni; q += 64) a += pr[q] * s_fI[q];
    a = wave_sum(a);
    if (lane == 0) s_fG[r] = a;
  }
  __syncthreads();
  // A2: the Sbar grid values not given as data, A_{Xbar,G} f_G (universal
  // operator rows in batches of 16 independent loads)
  for (int a = tid; a < Kb2; a += blockDim.x) {
    if (s_given[a]) continue;
    double v0 = 0.0, v1 = 0.0;
    int r = 0;
    for (; r + 16 <= nG; r += 16) {
      double w[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) w[u] = AbarT[(size_t)(r + u) * Kb2 + a];
#pragma unroll
      for (int u = 0; u < 16; u += 2) {
        v0 += w[u] * s_fG[r + u];
        v1 += w[u + 1] * s_fG[r + u + 1];
      }
    }
    for (; r < nG; ++r) v0 += AbarT[(size_t)r * Kb2 + a] * s_fG[r];
    s_g[a] = v0 + v1;
  }
  __syncthreads();
  // A3: coefficients c = C g C^T, truncated to total order < Kbar
  for (int e = tid; e < Kb2; e += blockDim.x) {
    const int m = e / Kb, j = e % Kb;
    double acc = 0.0;
    for (int i = 0; i < Kb; ++i) acc += s_cb[m * Kb + i] * s_g[i * Kb + j];
    s_tmp[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < Kb2; e += blockDim.x) {
    const int m = e / Kb, nn = e % Kb;
    double acc = 0.0;
    if (m + nn < Kb)
      for (int j = 0; j < Kb; ++j) acc += s_tmp[m * Kb + j] * s_cb[nn * Kb + j];
    s_coef[e] = acc;
  }
  __syncthreads();
  // values at the K x K nodes of every target leaf (the cut leaf first)
  for (int q = 0; q < ne; ++q) {
    int j;
    double ox, oy, sc;
    if (q < kExtTgtMax) {
      j = s_tg[q];
      ox = s_geo[3 * q];
      oy = s_geo[3 * q + 1];
      sc = s_geo[3 * q + 2];
    } else {
      j = ext_tgt[e0 + q];
      ox = ext_geo[3 * (e0 + q)];
      oy = ext_geo[3 * (e0 + q) + 1];
      sc = ext_geo[3 * (e0 + q) + 2];
    }
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
    for (int idx = tid; idx < Kb * K; idx += blockDim.x) {
      const int m = idx / K, b = idx % K;
      double acc = 0.0;
      for (int nn = 0; nn < Kb - m; ++nn) acc += s_coef[m * Kb + nn] * s_Ey[b * Kb + nn];
      s_tmp[idx] = acc;
    }
    __syncthreads();
    for (int idx = tid; idx < n; idx += blockDim.x) {
      const int a = idx / K, b = idx % K;
      double acc = 0.0;
      for (int m = 0; m < Kb; ++m) acc += s_Ex[a * Kb + m] * s_tmp[m * K + b];
      fe[(size_t)j * n + idx] = acc;
    }
    __syncthreads();
  }
}

typedef double vfx_d4 __attribute__((ext_vector_type(4)));
typedef double vfx_d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Per-output rows of the lane-per-pair kernels' LDS staging: 65 (not 64)
// double2 apart, so the eight lanes of a segment that read the same entry
// of eight outputs fall in different banks.
constexpr int kSoStride = 65;

// Sum of s[q] over q in [q0, q1) in a fixed order with four
// interleaved partial sums (deterministic, and the LDS loads overlap).
__device__ __forceinline__ double2 seg_sum(const double2* s, int q0, int q1) {
  double r0 = 0.0, i0 = 0.0, r1 = 0.0, i1 = 0.0, r2 = 0.0, i2 = 0.0, r3 = 0.0, i3 = 0.0;
  int q = q0;
  for (; q + 3 < q1; q += 4) {
    const double2 v0 = s[q], v1 = s[q + 1], v2 = s[q + 2], v3 = s[q + 3];
    r0 += v0.x;
    i0 += v0.y;
    r1 += v1.x;
    i1 += v1.y;
    r2 += v2.x;
    i2 += v2.y;
    r3 += v3.x;
    i3 += v3.y;
  }
  for (; q < q1; ++q) {
    r0 += s[q].x;
    i0 += s[q].y;
  }
  return make_double2((r0 + r1) + (r2 + r3), (i0 + i1) + (i2 + i3));
}

// M2L with one lane per list-2 entry (target box, source box), for a group
// of consecutive target boxes with at most 64 entries and at most 8 boxes.
// Lane e holds s_k = (-t)^k a_k of its source (registers); the shared
// Pascal coefficients C(k+l-1,l) are wave-uniform operands.  For each output
// l the lane forms t^l sum_k C(k+l-1,l) s_k (minus a_0 t^l/l, plus the log
// term for l = 0); the per-target sums go through LDS in chunks of 8 outputs,
// in entry order (deterministic), together with the P2L contributions.
template <int PM>
__global__ void __launch_bounds__(64) k_m2l_pairs(int P, double root_size, const int* __restrict__ grp,
                                                  const int* __restrict__ box_level, const int* __restrict__ l2_ptr,
                                                  const int* __restrict__ l2_src, const int* __restrict__ l2_off,
                                                  const int* __restrict__ l2_tgt, const int* __restrict__ l4_ptr,
                                                  const int* __restrict__ l4_src, const int* __restrict__ l4_slot,
                                                  const int* __restrict__ leaf_box, int p2l_rows,
                                                  const double* __restrict__ pasT, const double* __restrict__ logd,
                                                  const double2* __restrict__ mpole, const double* __restrict__ p2l_y,
                                                  double2* __restrict__ local, long smp, long spl) {
  mpole += blockIdx.y * smp;  // right-hand side blockIdx.y
  local += blockIdx.y * smp;
  p2l_y += blockIdx.y * spl;
  __shared__ double2 s_o[8 * kSoStride];
  const int g = blockIdx.x;
  const int b0 = grp[g], b1 = grp[g + 1];
  const int e0 = l2_ptr[b0], e1 = l2_ptr[b1];
  const int lane = threadIdx.x;
  const int e = e0 + lane;
  const bool act = e < e1;
  const int o = act ? l2_off[e] : 0;
  const int src = act ? l2_src[e] : 0;
  const double dx = (o / 7) - 3, dy = (o % 7) - 3;
  const double dd = (dx * dx + dy * dy) > 0 ? dx * dx + dy * dy : 1.0;
  const double2 t = make_double2(dx / dd, -dy / dd);  // 1 / (dx + i dy)
  double2 s[PM];
  {
    double2 pw = make_double2(1.0, 0.0);
    const double2 mt = make_double2(-t.x, -t.y);
#pragma unroll
    for (int k = 0; k < PM; ++k) {
      const double2 a = (act && k < P) ? mpole[(size_t)src * P + k] : make_double2(0.0, 0.0);
      s[k] = cmul(pw, a);
      pw = cmul(pw, mt);
    }
  }
  const double a0 = s[0].x;
  const int tgt = act ? l2_tgt[e] : b0;
  const double logh = log(box_side(root_size, box_level[tgt]));
  const double lg0 = act ? a0 * (logd[o] + logh) : 0.0;
  double2 tl = make_double2(1.0, 0.0);
  const int nchunk = (P + 7) / 8;
  for (int c = 0; c < nchunk; ++c) {
    double2 outc[8];
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) {
      const int l = 8 * c + lc;
      double2 out = make_double2(0.0, 0.0);
      if (l < P) {
        const double* cr = pasT + (size_t)l * P;
        double ur = 0.0, ui = 0.0;
#pragma unroll
        for (int k = 1; k < PM; ++k) {
          if (k < P) {
            const double cf = cr[k];
            ur += cf * s[k].x;
            ui += cf * s[k].y;
          }
        }
        out = cmul(tl, make_double2(ur, ui));
        if (l == 0) {
          out.x += lg0;
        } else {
          out.x -= a0 * tl.x / l;
          out.y -= a0 * tl.y / l;
        }
        tl = cmul(tl, t);
      }
      outc[lc] = act ? out : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) s_o[lc * kSoStride + lane] = outc[lc];
    __syncthreads();
    const int lc = lane & 7, seg = lane >> 3;
    const int bb = b0 + seg, l = 8 * c + lc;
    if (bb < b1 && l < P) {
      const double2 sv = seg_sum(s_o + lc * kSoStride, l2_ptr[bb] - e0, l2_ptr[bb + 1] - e0);
      double re = sv.x, im = sv.y;
      const double h = box_side(root_size, box_level[bb]);
      const double h2 = h * h;
      for (int q = l4_ptr[bb]; q < l4_ptr[bb + 1]; ++q) {
        const double* y = p2l_y + (size_t)l4_slot[q] * p2l_rows + 2 * l;
        re += h2 * y[0];
        im += h2 * y[1];
        if (l == 0) re += log(h) * mpole[(size_t)leaf_box[l4_src[q]] * P].x;
      }
      local[(size_t)bb * P + l] = make_double2(re, im);
    }
  }
}

// -------------------------------------------------------------------------
// Lane-per-translation forms, instantiated for the exact expansion length P
// (compile-time loops, so the Pascal coefficients, read through wave-uniform
// pointers, become scalar operands of the FMAs and need no LDS traffic).

// M2L: one lane per list-2 entry (target, source), for a group of
// consecutive target boxes with at most 64 entries and at most 8 boxes.
// Lane e holds s_k = (-t)^k a_k of its source; for each output l it forms
// t^l sum_k C(k+l-1,l) s_k (minus a_0 t^l/l; plus a_0 (log|d/h| + log h) for
// l = 0).  Per-target sums go through LDS in chunks of 8 outputs, in entry
// order (deterministic), together with the P2L contributions.
template <int P>
__global__ void __launch_bounds__(64) k_m2l_lanes(double root_size, const int* __restrict__ grp,
                                                  const int* __restrict__ box_level, const int* __restrict__ l2_ptr,
                                                  const int* __restrict__ l2_src, const int* __restrict__ l2_off,
                                                  const int* __restrict__ l2_tgt, const int* __restrict__ l4_ptr,
                                                  const int* __restrict__ l4_src, const int* __restrict__ l4_slot,
                                                  const int* __restrict__ leaf_box, int p2l_rows,
                                                  const double* __restrict__ pasT, const double* __restrict__ logd,
                                                  const double2* __restrict__ mpole, const double* __restrict__ p2l_y,
                                                  double2* __restrict__ local, long smp, long spl) {
  mpole += blockIdx.y * smp;  // right-hand side blockIdx.y
  local += blockIdx.y * smp;
  p2l_y += blockIdx.y * spl;
  __shared__ double2 s_o[8 * kSoStride];
  const int g = blockIdx.x;
  const int b0 = grp[g], b1 = grp[g + 1];
  const int e0 = l2_ptr[b0], e1 = l2_ptr[b1];
  const int lane = threadIdx.x;
  const int e = e0 + lane;
  const bool act = e < e1;
  const int o = act ? l2_off[e] : 0;
  const int src = act ? l2_src[e] : 0;
  const double dx = (o / 7) - 3, dy = (o % 7) - 3;
  const double dd = dx * dx + dy * dy;
  const double2 t = make_double2(dx / dd, -dy / dd);  // 1 / (dx + i dy)
  double2 s[P];
  {
    double2 pw = make_double2(1.0, 0.0);
    const double2 mt = make_double2(-t.x, -t.y);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const double2 a = act ? mpole[(size_t)src * P + k] : make_double2(0.0, 0.0);
      s[k] = cmul(pw, a);
      pw = cmul(pw, mt);
    }
  }
  const double a0 = s[0].x;
  const int tgt = act ? l2_tgt[e] : b0;
  const double lg0 = act ? a0 * (logd[o] + log(box_side(root_size, box_level[tgt]))) : 0.0;
  double2 tl = make_double2(1.0, 0.0);
  constexpr int NC = (P + 7) / 8;
  // this lane's output role in every chunk: box bb = b0 + seg, outputs
  // l = 8c + lc; its list-2 range and the P2L contributions (h^2 times the
  // list-4 products, and log(h) a_0 of each list-4 leaf for l = 0) are
  // gathered once, here, so the chunk tails only sum LDS and store
  const int lc = lane & 7, seg = lane >> 3;
  const int bb = b0 + seg;
  const bool own = bb < b1;
  int r0 = 0, r1 = 0;
  double p2r[NC], p2i[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) p2r[c] = p2i[c] = 0.0;
  if (own) {
    r0 = l2_ptr[bb] - e0;
    r1 = l2_ptr[bb + 1] - e0;
    const double h = box_side(root_size, box_level[bb]);
    const double h2 = h * h;
    const int q0 = l4_ptr[bb], q1 = l4_ptr[bb + 1];
    double lgs = 0.0;
    for (int q = q0; q < q1; ++q) {
      const double* y = p2l_y + (size_t)l4_slot[q] * p2l_rows + 2 * lc;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (8 * c + lc < P) {
          p2r[c] += h2 * y[16 * c];
          p2i[c] += h2 * y[16 * c + 1];
        }
      if (lc == 0) lgs += mpole[(size_t)leaf_box[l4_src[q]] * P].x;
    }
    p2r[0] += log(h) * lgs;  // zero unless lc == 0 (output l = 0)
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    __syncthreads();
    // the eight outputs of the chunk accumulate side by side (k outer), so
    // their FMA chains interleave
    double ur[8], ui[8];
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) ur[lc] = ui[lc] = 0.0;
#pragma unroll
    for (int k = 1; k < P; ++k) {
#pragma unroll
      for (int lc = 0; lc < 8; ++lc) {
        const int l = 8 * c + lc;
        if (l < P) {
          const double cf = pasT[l * P + k];
          ur[lc] += cf * s[k].x;
          ui[lc] += cf * s[k].y;
        }
      }
    }
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) {
      const int l = 8 * c + lc;
      double2 out = make_double2(0.0, 0.0);
      if (l < P) {
        out = cmul(tl, make_double2(ur[lc], ui[lc]));
        if (l == 0) {
          out.x += lg0;
        } else {
          const double il = 1.0 / (double)l;  // compile-time constant
          out.x -= a0 * tl.x * il;
          out.y -= a0 * tl.y * il;
        }
        tl = cmul(tl, t);
      }
      s_o[lc * kSoStride + lane] = act ? out : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int l = 8 * c + lc;
    if (own && l < P) {
      const double2 sv = seg_sum(s_o + lc * kSoStride, r0, r1);
      local[(size_t)bb * P + l] = make_double2(sv.x + p2r[c], sv.y + p2i[c]);
    }
  }
}

// -------------------------------------------------------------------------
// Batched table GEMMs on the FP64 matrix cores (near field, P2L, P2M, M2P)
// for contraction lengths that are not a multiple of 32 (K = 4 and 12, whose
// K^2 is 16 and 144); the others run on k_tgemm below, which has a deeper
// pipeline.  Entries (pairs) are grouped by table configuration c; a work-group takes a
// tile of <= TE entries (64 or 16) of one configuration and a block of MTB
// row tiles (16 table rows each) and computes, for every entry e,
//   Y[e][row] = sum_k A_c[k][row] X[src(e)][k]
// (the table applied to the source leaf's K^2 values).
//   A: [c][k][row], R = 16*MT rows (rows fastest, MT a multiple of MTB);
//   X: [src][k] with row stride ldx, values k >= kx taken as zero (M2P reads
//   the 2P coefficients of a multipole); Y: [e][row].
// The K dimension is processed in blocks of 16 with both operands staged in
// double-buffered LDS: the global loads of block kb+1 are in flight while the
// waves run their MFMAs on block kb.  With TE = 64, wave w owns entries
// 16w..16w+15 and every row tile of the block; with TE = 16 the waves share
// the 16 entries and split the row tiles (w, w+4).  Row-tile counts are
// compile-time, so the MFMA sequence has no per-tile branches.  MFMA
// operands: A = entry data (16 entries x 4 k), B = table (4 k x 16 rows), so
// each output tile is (entries x rows) and the stores of a 16-lane group are
// 128 contiguous bytes.
// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16] and the
// outputs D[(l/16) + 4r][l%16], r = 0..3 (lane layout checked on gfx950).
// EPI = 1 (P2M): Y is the multipole array; rows < 2P of entry e (a leaf) are
// scaled by h^2 of that leaf and stored as its (p+1) complex coefficients.
template <int KD, int EPI, int TE, int MTB>
__global__ void __launch_bounds__(256) k_gemm(int nitems, int MT, const int* __restrict__ t_cfg,
                                              const int* __restrict__ t_first,
                                              const int* __restrict__ t_count, const int* __restrict__ src,
                                              const double* __restrict__ A, const double* __restrict__ X,
                                              double* __restrict__ Y, int P2, double root_size,
                                              const int* __restrict__ leaf_box, const int* __restrict__ box_level,
                                              long sx, long sy, int ldx, int kx) {
  static_assert(TE == 64 || MTB % 4 == 0, "TE = 16 splits the row tiles over the four waves");
  X += blockIdx.y * sx;  // right-hand side blockIdx.y
  Y += blockIdx.y * sy;
  constexpr int KB = 16;
  constexpr int LDA = TE;        // entries per LDS row (tile of TE = 64 or 16 entries)
  constexpr int LDB = 16 * MTB;  // table rows per LDS row
  constexpr int NACC = (TE == 64) ? MTB : MTB / 4;  // row tiles per wave
  constexpr int BE = MTB;        // table values staged per thread and K block
  __shared__ double sA[2][KB * LDA];
  __shared__ double sB[2][KB * LDB];
  const int nrb = MT / MTB;
  // XCD-aware, persistent order: work-groups are dispatched round-robin over
  // the 8 XCDs, so the work-groups of XCD x (blockIdx % 8 == x) walk one
  // contiguous range of work items; consecutive items share a configuration
  // and hence a table, which that XCD's L2 then serves to all of them.
  const int nb = gridDim.x, bb = blockIdx.x;
  const int x = bb & 7;
  const int q = nitems >> 3, rr = nitems & 7;
  const int xfirst = x * q + min(x, rr), xcount = q + (x < rr ? 1 : 0);
  const int xwgs = (nb - x + 7) >> 3;  // work-groups on this XCD
  for (int j = bb >> 3; j < xcount; j += xwgs) {
  const int item = xfirst + j;
  const int tile = item / nrb, rb = item - tile * nrb;
  const int c = t_cfg[tile], p0 = t_first[tile], np = t_count[tile];
  const int R = 16 * MT;
  const int row0 = 16 * MTB * rb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const double* Ac = A + (size_t)c * KD * R;
  // global -> register staging of one K block
  constexpr int AE = TE * KB / 256;                  // entry values per thread (4 or 1)
  const int aj = tid % TE, ak = (tid / TE) * AE;     // entry aj, k = ak..ak+AE-1
  // table block KB x LDB: thread tid stages the values tid, tid + 256, ...
  // (v = k * LDB + row), so consecutive lanes touch consecutive rows
  const bool a_ok = aj < np;
  const double* xsrc = X + (size_t)(a_ok ? src[p0 + aj] : 0) * ldx;
  double ra[AE], rbv[BE];
  auto gload = [&](int kb) {
    const int k0 = kb * KB;
#pragma unroll
    for (int e = 0; e < AE; ++e) ra[e] = (a_ok && k0 + ak + e < kx) ? xsrc[k0 + ak + e] : 0.0;
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int v = tid + 256 * e, bk = v / LDB, br = v - bk * LDB;
      rbv[e] = Ac[(size_t)(k0 + bk) * R + row0 + br];
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AE; ++e) sA[buf][(ak + e) * LDA + aj] = ra[e];
#pragma unroll
    for (int e = 0; e < BE; ++e) sB[buf][tid + 256 * e] = rbv[e];
  };
  // wave w: TE = 64 -> entries 16w..16w+15, every row tile;
  //         TE = 16 -> entries 0..15, row tiles w, w+4
  const int ebase = (TE == 64) ? 16 * w : 0;
  auto tile_of = [&](int r) { return (TE == 64) ? r : w + 4 * r; };
  vfx_d4 acc[NACC];
#pragma unroll
  for (int r = 0; r < NACC; ++r) acc[r] = vfx_d4{0, 0, 0, 0};
  constexpr int NKB = KD / KB;
  __syncthreads();  // the previous item is done with the LDS buffers
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kb = 0; kb < NKB; ++kb) {
    const int buf = kb & 1;
    if (kb + 1 < NKB) gload(kb + 1);
#pragma unroll
    for (int ks = 0; ks < KB / 4; ++ks) {
      const int k = 4 * ks + lk;
      const double a = sA[buf][k * LDA + ebase + li];
      double bv[NACC];
#pragma unroll
      for (int r = 0; r < NACC; ++r) bv[r] = sB[buf][k * LDB + 16 * tile_of(r) + li];
#pragma unroll
      for (int r = 0; r < NACC; ++r) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[r], acc[r], 0, 0, 0);
    }
    if (kb + 1 < NKB) lstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < NACC; ++r) {
    const int row = row0 + 16 * tile_of(r) + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ent = ebase + lk + 4 * e;
      if (ent >= np) continue;
      if (EPI == 0) {
        Y[(size_t)(p0 + ent) * R + row] = acc[r][e];
      } else if (row < P2) {
        const int leaf = src[p0 + ent];
        const int b = leaf_box[leaf];
        const double h = box_side(root_size, box_level[b]);
        Y[(size_t)b * P2 + row] = h * h * acc[r][e];
      }
    }
  }
  }  // work items
}

// -------------------------------------------------------------------------
// Table GEMMs with 64-entry tiles and K a multiple of 32 (near field dense
// operators, P2L, M2P, P2M for K = 8 and 16): the same products as k_gemm with a
// deeper pipeline.  A work item is a tile of <= 64 entries of one
// configuration and a block of MTB row tiles; wave w owns the entries
// 16w..16w+15.  The entry operands go straight from memory into a ring of
// three register blocks (contraction order permuted so that a lane reads 64
// contiguous bytes per block: MFMA step s of block kb pairs k = 32kb +
// 8(l/16) + s with lane l on both sides); the table block (32 k x 16 MTB
// rows), shared by the four waves, goes through a ring of two register
// blocks into double-buffered LDS.  Every global load is issued two
// compute phases before its data is needed.  LDS rows are 16 MTB + 2
// doubles apart, so the two lane groups of a half-wave (rows 8 apart) fall
// into opposite halves of the banks.  Persistent, XCD-aware item order as in
// k_gemm.
// calls f(integral_constant<int, I>) for I = I0 .. N-1 (ring indices in an
// unrolled pipeline stay compile-time constants)
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int KD, int MTB, int EPI>
__global__ void __launch_bounds__(256) k_tgemm(int nitems, int MT, const int* __restrict__ t_cfg,
                                               const int* __restrict__ t_first, const int* __restrict__ t_count,
                                               const int* __restrict__ src, const double* __restrict__ A,
                                               const double* __restrict__ X, double* __restrict__ Y, long sx,
                                               long sy, int ldx, int kx, int P2, double root_size,
                                               const int* __restrict__ leaf_box, const int* __restrict__ box_level) {
  static_assert(KD % 32 == 0, "contraction in blocks of 32");
  X += blockIdx.y * sx;  // right-hand side blockIdx.y
  Y += blockIdx.y * sy;
  constexpr int KB = 32, NKB = KD / KB;
  constexpr int NC = 16 * MTB, LDB = NC + 2;  // table columns per block, LDS row stride
  constexpr int BP = NC / 2;                  // 16-byte pieces per table row
  __shared__ __attribute__((aligned(16))) double sB[2 * KB * LDB];
  const int nrb = MT / MTB;
  const int nb = gridDim.x, bb = blockIdx.x;
  const int x = bb & 7;
  const int q = nitems >> 3, rr = nitems & 7;
  const int xfirst = x * q + min(x, rr), xcount = q + (x < rr ? 1 : 0);
  const int xwgs = (nb - x + 7) >> 3;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int R = 16 * MT;
  for (int j = bb >> 3; j < xcount; j += xwgs) {
    const int item = xfirst + j;
    const int tile = item / nrb, rb = item - tile * nrb;
    const int c = t_cfg[tile], p0 = t_first[tile], np = t_count[tile];
    const int row0 = NC * rb;
    const double* Ac = A + (size_t)c * KD * R + row0;
    // this lane's entry (an entry past the tile's end reads the first
    // entry's row; its results are not stored)
    const int ent = 16 * w + li;
    const double* xrow = X + (size_t)src[p0 + (ent < np ? ent : 0)] * ldx + 8 * lk;
    vfx_d2 ra[3][4], rbuf[2][MTB];
    auto ga = [&](auto kbc, auto slot) __attribute__((always_inline)) {
      constexpr int kb = decltype(kbc)::value, sl = decltype(slot)::value;
      static_for<0, 4>([&](auto ec) __attribute__((always_inline)) {
        constexpr int e = decltype(ec)::value;
        ra[sl][e] =
            (KB * kb + 8 * lk + 2 * e < kx) ? *(const vfx_d2*)(xrow + KB * kb + 2 * e) : vfx_d2{0.0, 0.0};
      });
    };
    auto gb = [&](auto kbc, auto slot) __attribute__((always_inline)) {
      constexpr int kb = decltype(kbc)::value, sl = decltype(slot)::value;
      static_for<0, MTB>([&](auto ec) __attribute__((always_inline)) {
        constexpr int e = decltype(ec)::value;
        const int qq = tid + 256 * e, row = qq / BP, col = 2 * (qq % BP);
        rbuf[sl][e] = *(const vfx_d2*)(Ac + (size_t)(KB * kb + row) * R + col);
      });
    };
    auto sb = [&](auto buf, auto slot) __attribute__((always_inline)) {
      constexpr int bf = decltype(buf)::value, sl = decltype(slot)::value;
      static_for<0, MTB>([&](auto ec) __attribute__((always_inline)) {
        constexpr int e = decltype(ec)::value;
        const int qq = tid + 256 * e, row = qq / BP, col = 2 * (qq % BP);
        *(vfx_d2*)(sB + (bf * KB + row) * LDB + col) = rbuf[sl][e];
      });
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    vfx_d4 acc[MTB];
#pragma unroll
    for (int r = 0; r < MTB; ++r) acc[r] = vfx_d4{0, 0, 0, 0};
    ga(I0{}, I0{});
    gb(I0{}, I0{});
    if constexpr (NKB > 1) {
      ga(I1{}, I1{});
      gb(I1{}, I1{});
    }
    __syncthreads();  // the previous item is done with sB
    sb(I0{}, I0{});
    __syncthreads();
    static_for<0, NKB>([&](auto kbc) __attribute__((always_inline)) {
      constexpr int kb = decltype(kbc)::value;
      if constexpr (kb + 2 < NKB) {
        ga(std::integral_constant<int, kb + 2>{}, std::integral_constant<int, (kb + 2) % 3>{});
        gb(std::integral_constant<int, kb + 2>{}, std::integral_constant<int, kb % 2>{});
      }
      const double* sbk = sB + ((kb % 2) * KB + 8 * lk) * LDB + li;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const double av = (s & 1) ? ra[kb % 3][s >> 1].y : ra[kb % 3][s >> 1].x;
        double bv[MTB];
#pragma unroll
        for (int r = 0; r < MTB; ++r) bv[r] = sbk[s * LDB + 16 * r];
#pragma unroll
        for (int r = 0; r < MTB; ++r) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[r], acc[r], 0, 0, 0);
      }
      if constexpr (kb + 1 < NKB) sb(std::integral_constant<int, (kb + 1) % 2>{}, std::integral_constant<int, (kb + 1) % 2>{});
      __syncthreads();
    });
    // outputs D[lk + 4e][16 r + li]: entry 16w + lk + 4e, row row0 + 16r + li
    // (EPI = 1: rows < 2P of a leaf, scaled by h^2, into its multipole)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int en = 16 * w + lk + 4 * e;
      if (en >= np) continue;
      if constexpr (EPI == 0) {
#pragma unroll
        for (int r = 0; r < MTB; ++r) Y[(size_t)(p0 + en) * R + row0 + 16 * r + li] = acc[r][e];
      } else {
        const int b = leaf_box[src[p0 + en]];
        const double h = box_side(root_size, box_level[b]);
#pragma unroll
        for (int r = 0; r < MTB; ++r) {
          const int row = row0 + 16 * r + li;
          if (row < P2) Y[(size_t)b * P2 + row] = h * h * acc[r][e];
        }
      }
    }
  }
}

// -------------------------------------------------------------------------
// Near field in low-rank form, for the configurations c whose operator
// factorises as Q_c W_c (rank R_c <= 64, padded to a multiple of 16).  A
// work item is a tile of <= 32 list-1 pairs of one configuration:
//   Z = X W_c^T  (pairs x R_c: the source leaf values times the row factor),
//   Y = Z Q_c^T  (pairs x n),
// both as FP64 MFMA tile products.  Wave w = pg + 2 hf works on the pair
// group pg (pairs 16pg..16pg+15): in phase 1 on the source nodes of half hf
// (the two partial Z of a pair group meet in LDS), in phase 2 on the target
// rows of half hf.  So a wave carries half of a 16-pair share of the work,
// and a few hundred tiles spread evenly over the SIMDs.  Phase 1 takes its A
// operands (the wave's own source rows) straight from memory into a ring of
// three register blocks, with the contraction order permuted so that a lane
// reads 16 contiguous bytes per block of 8 nodes; W_c, shared by the four
// waves, goes through a ring of two register blocks into double-buffered
// LDS (both halves' rows of a block at once), and Q_c the same way, 4 ranks
// per block.  Every global load is issued two compute phases before its
// data is needed.  With about 51 KB of LDS and <= 168 VGPRs three
// work-groups share a CU.  Persistent, XCD-aware item order as in k_gemm
// (items are configuration-major, so an XCD's L2 holds the factors of the
// few configurations it works on).
// LDS row strides: W rows 72 doubles (the lane groups of a half-wave read
// rows 2 apart: 2 x 72 x 8 bytes = 128 mod 256, opposite halves of the
// banks); Q rows 272 doubles (rows 1 apart: 272 x 8 = 128 mod 256).
constexpr int kLrKB = 8, kLrLDW = 72, kLrLDZ = kNearLrMax + 1, kLrQB = 4, kLrLDQ = 272;
constexpr int kLrTile = 32;

template <int KD, int MT1>
__device__ __forceinline__ void near_lr_item(const double* __restrict__ xrow, const double* __restrict__ Wc,
                                             const double* __restrict__ Qc, double* sbuf, double* sZ,
                                             double* __restrict__ Yp, int np) {
  constexpr int LM = kNearLrMax, HK = KD / 2, NKB = HK / kLrKB, R = 16 * MT1;
  constexpr int NQB = R / kLrQB, NRT2 = HK / 16;
  static_assert(2 * 2 * kLrKB * kLrLDW >= 2 * kLrQB * kLrLDQ && KD <= kLrLDQ, "staging buffer sizes");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pg = w & 1, hf = w >> 1;
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  // ---- phase 1: partial Z over the source nodes of half hf; MFMA step s of
  // block kb pairs node HK hf + 8kb + 2(l/16) + s with lane l on both sides
  vfx_d2 ra[3], rw[2][2];
  auto ga = [&](auto kbc, auto slc) __attribute__((always_inline)) {
    constexpr int kb = decltype(kbc)::value, sl = decltype(slc)::value;
    ra[sl] = *(const vfx_d2*)(xrow + kLrKB * kb);
  };
  // W block: rows 8kb..8kb+7 of both halves (LDS rows 0..7 half 0, 8..15
  // half 1), 16-byte pieces q = tid + 256 e
  auto gw = [&](auto kbc, auto slc) __attribute__((always_inline)) {
    constexpr int kb = decltype(kbc)::value, sl = decltype(slc)::value;
    static_for<0, 2>([&](auto ec) __attribute__((always_inline)) {
      constexpr int e = decltype(ec)::value;
      const int q = tid + 256 * e, r16 = q >> 5, col = 2 * (q & 31);
      const int row = (r16 >> 3) * HK + kLrKB * kb + (r16 & 7);
      rw[sl][e] = col < R ? *(const vfx_d2*)(Wc + (size_t)row * LM + col) : vfx_d2{0.0, 0.0};
    });
  };
  auto sw = [&](auto bufc, auto slc) __attribute__((always_inline)) {
    constexpr int bf = decltype(bufc)::value, sl = decltype(slc)::value;
    static_for<0, 2>([&](auto ec) __attribute__((always_inline)) {
      constexpr int e = decltype(ec)::value;
      const int q = tid + 256 * e, r16 = q >> 5, col = 2 * (q & 31);
      *(vfx_d2*)(sbuf + (bf * 2 * kLrKB + r16) * kLrLDW + col) = rw[sl][e];
    });
  };
  vfx_d4 acc[MT1];
#pragma unroll
  for (int r = 0; r < MT1; ++r) acc[r] = vfx_d4{0, 0, 0, 0};
  ga(I0{}, I0{});
  gw(I0{}, I0{});
  ga(I1{}, I1{});
  gw(I1{}, I1{});
  __syncthreads();  // the previous item is done with sbuf and sZ
  sw(I0{}, I0{});
  __syncthreads();
  static_for<0, NKB>([&](auto kbc) __attribute__((always_inline)) {
    constexpr int kb = decltype(kbc)::value;
    if constexpr (kb + 2 < NKB) {
      ga(std::integral_constant<int, kb + 2>{}, std::integral_constant<int, (kb + 2) % 3>{});
      gw(std::integral_constant<int, kb + 2>{}, std::integral_constant<int, kb % 2>{});
    }
    const double* sb = sbuf + ((kb % 2) * 2 * kLrKB + kLrKB * hf + 2 * lk) * kLrLDW + li;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double av = ra[kb % 3][s];
      double bv[MT1];
#pragma unroll
      for (int r = 0; r < MT1; ++r) bv[r] = sb[s * kLrLDW + 16 * r];
#pragma unroll
      for (int r = 0; r < MT1; ++r) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[r], acc[r], 0, 0, 0);
    }
    if constexpr (kb + 1 < NKB)
      sw(std::integral_constant<int, (kb + 1) % 2>{}, std::integral_constant<int, (kb + 1) % 2>{});
    __syncthreads();
  });
  // partial Z of half hf for the pair group's rows: D[lk + 4e][16 r + li]
  double* sZh = sZ + hf * kLrTile * kLrLDZ;
#pragma unroll
  for (int r = 0; r < MT1; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) sZh[(16 * pg + lk + 4 * e) * kLrLDZ + 16 * r + li] = acc[r][e];
  // ---- phase 2: rows HK hf.. of Y = Z Q^T, Z = the sum of the two partials;
  // Q block = 4 ranks x n rows, pieces v = tid + 256 e
  vfx_d2 rq[2][2];
  auto gq = [&](auto qbc, auto slc) __attribute__((always_inline)) {
    constexpr int qb = decltype(qbc)::value, sl = decltype(slc)::value;
    static_for<0, 2>([&](auto ec) __attribute__((always_inline)) {
      constexpr int e = decltype(ec)::value;
      const int v = tid + 256 * e, rank = v / (KD / 2), col = 2 * (v % (KD / 2));
      rq[sl][e] = *(const vfx_d2*)(Qc + (size_t)(kLrQB * qb + rank) * KD + col);
    });
  };
  auto sq = [&](auto bufc, auto slc) __attribute__((always_inline)) {
    constexpr int bf = decltype(bufc)::value, sl = decltype(slc)::value;
    static_for<0, 2>([&](auto ec) __attribute__((always_inline)) {
      constexpr int e = decltype(ec)::value;
      const int v = tid + 256 * e, rank = v / (KD / 2), col = 2 * (v % (KD / 2));
      *(vfx_d2*)(sbuf + (bf * kLrQB + rank) * kLrLDQ + col) = rq[sl][e];
    });
  };
  vfx_d4 acc2[NRT2];
#pragma unroll
  for (int r = 0; r < NRT2; ++r) acc2[r] = vfx_d4{0, 0, 0, 0};
  gq(I0{}, I0{});
  if constexpr (NQB > 1) gq(I1{}, I1{});
  __syncthreads();  // phase 1 is done with sbuf; both partial Z complete
  sq(I0{}, I0{});
  __syncthreads();
  const double* z0 = sZ + (16 * pg + li) * kLrLDZ + lk;
  const double* z1 = z0 + kLrTile * kLrLDZ;
  static_for<0, NQB>([&](auto qbc) __attribute__((always_inline)) {
    constexpr int qb = decltype(qbc)::value;
    if constexpr (qb + 2 < NQB) gq(std::integral_constant<int, qb + 2>{}, std::integral_constant<int, qb % 2>{});
    const double a = z0[kLrQB * qb] + z1[kLrQB * qb];
    const double* qrow = sbuf + ((qb % 2) * kLrQB + lk) * kLrLDQ + HK * hf + li;
#pragma unroll
    for (int r = 0; r < NRT2; ++r) acc2[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, qrow[16 * r], acc2[r], 0, 0, 0);
    if constexpr (qb + 1 < NQB)
      sq(std::integral_constant<int, (qb + 1) % 2>{}, std::integral_constant<int, (qb + 1) % 2>{});
    __syncthreads();
  });
#pragma unroll
  for (int r = 0; r < NRT2; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ent = 16 * pg + lk + 4 * e;
      if (ent < np) Yp[(size_t)ent * KD + HK * hf + 16 * r + li] = acc2[r][e];
    }
}

template <int KD>
__global__ void __launch_bounds__(256, 3) k_near_lr(int nitems, const int* __restrict__ t_cfg,
                                                    const int* __restrict__ t_first, const int* __restrict__ t_count,
                                                    const int* __restrict__ src, const int* __restrict__ lr_R,
                                                    const double* __restrict__ W, const double* __restrict__ Q,
                                                    const double* __restrict__ X, double* __restrict__ Y, long sx,
                                                    long sy) {
  X += blockIdx.y * sx;  // right-hand side blockIdx.y
  Y += blockIdx.y * sy;
  constexpr int LM = kNearLrMax;  // 64
  __shared__ __attribute__((aligned(16))) double sbuf[2 * 2 * kLrKB * kLrLDW];
  __shared__ double sZ[2 * kLrTile * kLrLDZ];
  const int nb = gridDim.x, bb = blockIdx.x;
  const int x = bb & 7;
  const int q = nitems >> 3, rr = nitems & 7;
  const int xfirst = x * q + min(x, rr), xcount = q + (x < rr ? 1 : 0);
  const int xwgs = (nb - x + 7) >> 3;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int j = bb >> 3; j < xcount; j += xwgs) {
    const int tile = xfirst + j;
    const int c = t_cfg[tile], p0 = t_first[tile], np = t_count[tile];
    const double* Wc = W + (size_t)c * KD * LM;
    const double* Qc = Q + (size_t)c * LM * KD;
    // this lane's A-operand pair (a pair past the tile's end reads the first
    // pair's row; its results are not stored) and its half of the nodes
    const int ent = 16 * (w & 1) + li;
    const double* xrow = X + (size_t)src[p0 + (ent < np ? ent : 0)] * KD + (KD / 2) * (w >> 1) + 2 * lk;
    double* Yp = Y + (size_t)p0 * KD;
    switch (lr_R[c] >> 4) {
      case 1: near_lr_item<KD, 1>(xrow, Wc, Qc, sbuf, sZ, Yp, np); break;
      case 2: near_lr_item<KD, 2>(xrow, Wc, Qc, sbuf, sZ, Yp, np); break;
      case 3: near_lr_item<KD, 3>(xrow, Wc, Qc, sbuf, sZ, Yp, np); break;
      default: near_lr_item<KD, 4>(xrow, Wc, Qc, sbuf, sZ, Yp, np); break;
    }
  }  // work items
}

// -------------------------------------------------------------------------
// Upward pass without the level-by-level chain.  The multipole of a non-leaf
// box B (level >= 2) about its own centre is the sum, over the leaves L below
// it, of the leaf multipoles shifted to B.  The shifted coefficients b_l
// depend only on a_k with k <= l, so they are exact (up to rounding) for any
// number of levels between L and B.  Scaled form (a_k h_L^-k, b_l h_B^-l):
//   b_0 = a_0,  b_l = w^l [ sum_{1<=k<=l} C(l-1,k-1) (r/w)^k a_k - a_0/l ],
// w = (c_L - c_B)/h_B, r = h_L/h_B.  One lane per (box, leaf) pair; a group
// of <= 8 boxes and <= 64 pairs per wave; per-box sums in pair order through
// LDS (deterministic).  Slices of a box with more than 64 pairs write
// partial sums, added in slice order by k_up_sum.
template <int PM, bool EXACT>
__global__ void __launch_bounds__(64) k_up(int Prt, double root_size, const int* __restrict__ grp, const int* __restrict__ up_box,
                                           const int* __restrict__ up_ptr, const int* __restrict__ up_src,
                                           const int* __restrict__ up_pos, const int* __restrict__ box_level,
                                           const double* __restrict__ box_cx, const double* __restrict__ box_cy,
                                           const double* __restrict__ pasT, double2* __restrict__ mpole,
                                           double2* __restrict__ part, long smp, long spart) {
  const int P = EXACT ? PM : Prt;
  mpole += blockIdx.y * smp;  // right-hand side blockIdx.y
  part += blockIdx.y * spart;
  __shared__ double2 s_o[8 * kSoStride];
  const int* gg = grp + 5 * blockIdx.x;
  const int u0 = gg[0], u1 = gg[1], e0 = gg[2], e1 = gg[3], slot = gg[4];
  const int lane = threadIdx.x;
  const int e = e0 + lane;
  const bool act = e < e1;
  const int src = act ? up_src[e] : up_box[u0];
  const int tgt = up_box[act ? up_pos[e] : u0];
  const int ls = box_level[src], lt = box_level[tgt];
  const double hb = box_side(root_size, lt);
  const double2 w = act ? make_double2((box_cx[src] - box_cx[tgt]) / hb, (box_cy[src] - box_cy[tgt]) / hb)
                        : make_double2(0.5, 0.5);
  const double r = act ? ldexp(1.0, lt - ls) : 1.0;
  const double ww = w.x * w.x + w.y * w.y;
  const double2 q = make_double2(r * w.x / ww, -r * w.y / ww);  // r / w
  const int NC = (P + 7) / 8;
  // work-group z computes the outputs l = 8c .. 8c+7 (chunk c = blockIdx.z,
  // a compile-time constant inside the matching branch); the scaled source
  // coefficients s_k = (r/w)^k a_k, k <= 8c+7, are formed on the fly (k
  // outer) rather than held, which keeps the kernel at a few dozen registers
  static_for<0, (PM + 7) / 8>([&](auto cc) __attribute__((always_inline)) {
    constexpr int c = decltype(cc)::value;
    constexpr int KH = (8 * c + 8 < PM) ? 8 * c + 8 : PM;  // k < KH
    if (c != (int)blockIdx.z || c >= NC) return;
    // w^(l-1) before output l: the same product sequence as a running power
    double2 wl = make_double2(1.0, 0.0);
#pragma unroll
    for (int i = 1; i < 8 * c; ++i) wl = cmul(wl, w);
    double2 pw = make_double2(1.0, 0.0);
    const double2 a0 = cmul(pw, act ? mpole[(size_t)src * P] : make_double2(0.0, 0.0));
    pw = cmul(pw, q);
    // the eight outputs of the chunk accumulate side by side (k outer)
    double ur[8], ui[8];
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) {
      const int l = 8 * c + lc;
      const double il = l > 0 ? 1.0 / (double)l : 0.0;  // compile-time constant
      ur[lc] = -a0.x * il;
      ui[lc] = -a0.y * il;
    }
#pragma unroll
    for (int k = 1; k < KH; ++k) {
      const double2 a = (act && k < P) ? mpole[(size_t)src * P + k] : make_double2(0.0, 0.0);
      const double2 sk = cmul(pw, a);
      pw = cmul(pw, q);
#pragma unroll
      for (int lc = 0; lc < 8; ++lc) {
        const int l = 8 * c + lc;
        if (k <= l && l < P) {
          const double cf = pasT[l * P + k];
          ur[lc] += cf * sk.x;
          ui[lc] += cf * sk.y;
        }
      }
    }
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) {
      const int l = 8 * c + lc;
      double2 out = make_double2(0.0, 0.0);
      if (l == 0) {
        out = a0;
      } else if (l < P) {
        wl = cmul(wl, w);
        out = cmul(wl, make_double2(ur[lc], ui[lc]));
      }
      s_o[lc * kSoStride + lane] = act ? out : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lc = lane & 7, seg = lane >> 3;
    const int uu = u0 + seg, l = 8 * c + lc;
    if (uu < u1 && l < P) {
      const int q0 = max(up_ptr[uu], e0), q1 = min(up_ptr[uu + 1], e1);
      const double2 sv = seg_sum(s_o + lc * kSoStride, q0 - e0, q1 - e0);
      const double re = sv.x, im = sv.y;
      if (slot < 0)
        mpole[(size_t)up_box[uu] * P + l] = make_double2(re, im);
      else
        part[(size_t)slot * P + l] = make_double2(re, im);
    }
  });
}

// Multipoles of the split boxes: the slices' partial sums added in a fixed
// order (eight running sums, slice j into sum j mod 8, then combined
// pairwise), eight loads in flight per round rather than one round trip per
// slice.
__global__ void __launch_bounds__(64) k_up_sum(int P, const int* __restrict__ split, const double2* __restrict__ part,
                                               double2* __restrict__ mpole, long spart, long smp) {
  part += blockIdx.y * spart;  // right-hand side blockIdx.y
  mpole += blockIdx.y * smp;
  const int* sp = split + 3 * blockIdx.x;
  const int l = threadIdx.x;
  if (l >= P) return;
  const int first = sp[1], ns = sp[2];
  double re[8], im[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) re[u] = im[u] = 0.0;
  for (int j = 0; j < ns; j += 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = j + u < ns ? part[(size_t)(first + j + u) * P + l] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      re[u] += v[u].x;
      im[u] += v[u].y;
    }
  }
  const double r = ((re[0] + re[1]) + (re[2] + re[3])) + ((re[4] + re[5]) + (re[6] + re[7]));
  const double i = ((im[0] + im[1]) + (im[2] + im[3])) + ((im[4] + im[5]) + (im[6] + im[7]));
  mpole[(size_t)sp[0] * P + l] = make_double2(r, i);
}

__device__ __forceinline__ double2 cpow(double2 z, int k) {
  double2 r = make_double2(1.0, 0.0);
  while (k) {
    if (k & 1) r = cmul(r, z);
    z = cmul(z, z);
    k >>= 1;
  }
  return r;
}

// -------------------------------------------------------------------------
// Downward pass without the level-by-level chain: the local expansion of a
// leaf b is its own (M2L + P2L) part plus the own parts of its ancestors A
// at levels >= 2 shifted directly to its centre (an exact polynomial shift,
// so equal up to rounding to the level-by-level pass).  Scaled form,
// w = (c_b - c_A)/h_A, r = h_b/h_A:
//   c_l += (r/w)^l sum_{k>=l} C(k,l) w^k b_k(A).
// One lane per (leaf, ancestor) pair; a group of <= 8 leaves and <= 64
// pairs per wave; per-leaf sums in pair order through LDS (deterministic).
template <int PM, bool EXACT>
__global__ void __launch_bounds__(64) k_down(int Prt, double root_size, const int* __restrict__ grp,
                                             const int* __restrict__ anc_ptr, const int* __restrict__ anc,
                                             const int* __restrict__ anc_leaf, const int* __restrict__ leaf_box,
                                             const int* __restrict__ box_level, const double* __restrict__ box_cx,
                                             const double* __restrict__ box_cy, const double* __restrict__ pasT,
                                             const double2* __restrict__ local, double2* __restrict__ locf, long smp,
                                             long slf) {
  const int P = EXACT ? PM : Prt;
  local += blockIdx.y * smp;  // right-hand side blockIdx.y
  locf += blockIdx.y * slf;
  __shared__ double2 s_o[8 * kSoStride];
  const int f0 = grp[blockIdx.x], f1 = grp[blockIdx.x + 1];
  const int e0 = anc_ptr[f0], e1 = anc_ptr[f1];
  const int lane = threadIdx.x;
  const int e = e0 + lane;
  const bool act = e < e1;
  const int A = act ? anc[e] : 0;
  const int b = leaf_box[act ? anc_leaf[e] : f0];
  const int la = box_level[A], lb = box_level[b];
  const double hA = box_side(root_size, la);
  const double2 w = act ? make_double2((box_cx[b] - box_cx[A]) / hA, (box_cy[b] - box_cy[A]) / hA)
                        : make_double2(0.5, 0.5);
  const double r = act ? ldexp(1.0, la - lb) : 1.0;
  const double ww = w.x * w.x + w.y * w.y;
  const double2 q = make_double2(r * w.x / ww, -r * w.y / ww);  // r / w
  const int NC = (P + 7) / 8;
  // work-group z computes the outputs l = 8c .. 8c+7 (chunk c = blockIdx.z);
  // the scaled ancestor coefficients s_k = w^k b_k, k >= 8c, are formed on
  // the fly (k outer) rather than held, which keeps the kernel at a few
  // dozen registers
  static_for<0, (PM + 7) / 8>([&](auto cc) __attribute__((always_inline)) {
    constexpr int c = decltype(cc)::value;
    if (c != (int)blockIdx.z || c >= NC) return;
    // q^l before output l: the same product sequence as a running power
    double2 ql = make_double2(1.0, 0.0);
#pragma unroll
    for (int i = 0; i < 8 * c; ++i) ql = cmul(ql, q);
    // w^k from k = 0, the same product sequence as a running power
    double2 pw = make_double2(1.0, 0.0);
#pragma unroll
    for (int k = 0; k < 8 * c; ++k) pw = cmul(pw, w);
    // the eight outputs of the chunk accumulate side by side (k outer)
    double ur[8], ui[8];
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) ur[lc] = ui[lc] = 0.0;
#pragma unroll
    for (int k = 8 * c; k < PM; ++k) {
      const double2 a = (act && k < P) ? local[(size_t)A * P + k] : make_double2(0.0, 0.0);
      const double2 sk = cmul(pw, a);
      pw = cmul(pw, w);
#pragma unroll
      for (int lc = 0; lc < 8; ++lc) {
        const int l = 8 * c + lc;
        if (k >= l && k < P) {
          const double cf = pasT[l * P + k];
          ur[lc] += cf * sk.x;
          ui[lc] += cf * sk.y;
        }
      }
    }
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) {
      const int l = 8 * c + lc;
      double2 out = make_double2(0.0, 0.0);
      if (l < P) {
        out = cmul(ql, make_double2(ur[lc], ui[lc]));
        ql = cmul(ql, q);
      }
      s_o[lc * kSoStride + lane] = act ? out : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lc = lane & 7, seg = lane >> 3;
    const int f = f0 + seg, l = 8 * c + lc;
    if (f < f1 && l < P) {
      const int bf = leaf_box[f];
      double2 v = make_double2(0.0, 0.0);
      if (box_level[bf] >= 2) {
        const double2 sv = seg_sum(s_o + lc * kSoStride, anc_ptr[f] - e0, anc_ptr[f + 1] - e0);
        const double2 own = local[(size_t)bf * P + l];
        v = make_double2(own.x + sv.x, own.y + sv.y);
      }
      locf[(size_t)f * P + l] = v;
    }
  });
}

// -------------------------------------------------------------------------
// Far field and the near-field reduction, one wave per leaf; lane l holds
// the nodes l + 64j, j < NPL (NPL = ceil(K^2/64)): L2P of the leaf's full
// local expansion by Horner in the scaled node position, the list-1 sums of
// the near-field products and the list-3 sums of the M2P products (in list
// order, deterministic), and the log terms: log(h) a_0 of each list-1 source
// and log(h/2) a_0 of each list-3 box.  Every per-leaf quantity (the local
// expansion, the list slots) comes in with one vector load, lane k holding
// item k, and is broadcast with readlane, so no step waits on a chain of
// scalar loads.  One wave per leaf keeps the whole grid resident at once.
// Each row of the per-pair and M2P products is read once, by its target's
// wave: those loads are non-temporal.  (The kernels that write the rows use
// plain stores, so that part of them is still in the last-level cache when
// this kernel runs; non-temporal stores there measured slower.)
typedef double vfx_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int PM, bool EXACT, int NPL, bool NTS>
__global__ void __launch_bounds__(64) k_far(int K, int Prt, double root_size, const int* __restrict__ leaf_box,
                                            const int* __restrict__ box_level, const double* __restrict__ t,
                                            const int* __restrict__ l3_ptr, const int* __restrict__ l3_src,
                                            const int* __restrict__ l3_slot, const double* __restrict__ Y3,
                                            const double2* __restrict__ locf, const double2* __restrict__ mpole,
                                            const int* __restrict__ l1_ptr, const int* __restrict__ l1_srcbox,
                                            const int* __restrict__ l1_slot, const double* __restrict__ Y,
                                            double* __restrict__ V, long slf,
                                            long smp, long sny, long sy3, long sv) {
  const int P = EXACT ? PM : Prt;  // <= 64
  locf += blockIdx.y * slf;        // right-hand side blockIdx.y
  mpole += blockIdx.y * smp;
  Y += blockIdx.y * sny;
  Y3 += blockIdx.y * sy3;
  V += blockIdx.y * sv;
  const int n = K * K;
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = leaf_box[leaf];
  const int lev = box_level[b];
  const double h = box_side(root_size, lev);
  // per-lane items: list-1 entry `lane` (at most one per configuration,
  // fewer than 64), list-3 entry `lane` (at most 20), local coefficient `lane`
  const int e0 = l1_ptr[leaf], n1 = l1_ptr[leaf + 1] - e0;
  const int f0 = l3_ptr[leaf], n3 = l3_ptr[leaf + 1] - f0;
  const int my_slot = (!NTS && lane < n1) ? l1_slot[e0 + lane] : 0;
  const double my_a0 = lane < n1 ? mpole[(size_t)l1_srcbox[e0 + lane] * P].x : 0.0;
  const int my_slot3 = lane < n3 ? l3_slot[f0 + lane] : 0;
  const double my_b0 = lane < n3 ? mpole[(size_t)l3_src[f0 + lane] * P].x : 0.0;
  const double2 my_c = (lev >= 2 && lane < P) ? locf[(size_t)leaf * P + lane] : double2{0.0, 0.0};
  // lane l holds nodes 4l .. 4l+3 when K^2 = 256 (rows of the per-pair
  // products are read with two 16-byte loads per lane), else l + 64j
  int node[NPL];
  double tx[NPL], ty[NPL], acc[NPL];
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int nd = NPL == 4 ? 4 * lane + j : lane + 64 * j;
    node[j] = nd < n ? nd : 0;
    tx[j] = 0.5 * t[node[j] / K];
    ty[j] = 0.5 * t[node[j] % K];
  }
  // near field (list 1) and M2P (list 3) sums, log terms
  {
    double yn[NPL], y3[NPL], lg = 0.0, lg3 = 0.0;
#pragma unroll
    for (int j = 0; j < NPL; ++j) yn[j] = y3[j] = 0.0;
    if (NTS) {
      // the target-stationary kernel left h^2 times the list-1 table sum in V
#pragma unroll
      for (int j = 0; j < NPL; ++j) yn[j] = V[(size_t)leaf * n + node[j]];
      for (int e = 0; e < n1; ++e) lg += readlane_d(my_a0, e);
    } else {
#pragma unroll 4
      for (int e = 0; e < n1; ++e) {
        const double* y = Y + (size_t)__builtin_amdgcn_readlane(my_slot, e) * n;
        if constexpr (NPL == 4) {
          const vfx_d2 u0 = __builtin_nontemporal_load((const vfx_d2*)(y + 4 * lane)),
                       u1 = __builtin_nontemporal_load((const vfx_d2*)(y + 4 * lane + 2));
          yn[0] += u0.x;
          yn[1] += u0.y;
          yn[2] += u1.x;
          yn[3] += u1.y;
        } else {
#pragma unroll
          for (int j = 0; j < NPL; ++j) yn[j] += y[node[j]];
        }
        lg += readlane_d(my_a0, e);
      }
    }
#pragma unroll 4
    for (int q = 0; q < n3; ++q) {
      const double* y = Y3 + (size_t)__builtin_amdgcn_readlane(my_slot3, q) * n;
      if constexpr (NPL == 4) {
        const vfx_d2 u0 = __builtin_nontemporal_load((const vfx_d2*)(y + 4 * lane)),
                     u1 = __builtin_nontemporal_load((const vfx_d2*)(y + 4 * lane + 2));
        y3[0] += u0.x;
        y3[1] += u0.y;
        y3[2] += u1.x;
        y3[3] += u1.y;
      } else {
#pragma unroll
        for (int j = 0; j < NPL; ++j) y3[j] += y[node[j]];
      }
      lg3 += readlane_d(my_b0, q);
    }
    const double lh = log(h);
    const double lt = lh * lg + (lh - kLn2) * lg3;
#pragma unroll
    for (int j = 0; j < NPL; ++j) acc[j] = (NTS ? yn[j] : h * h * yn[j]) + y3[j] + lt;
  }
  // L2P
  if (lev >= 2) {
    double ur[NPL], ui[NPL];
    {
      const double cx = readlane_d(my_c.x, P - 1), cy = readlane_d(my_c.y, P - 1);
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        ur[j] = cx;
        ui[j] = cy;
      }
    }
#pragma unroll
    for (int l = P - 2; l >= 0; --l) {
      const double cx = readlane_d(my_c.x, l), cy = readlane_d(my_c.y, l);
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const double r = ur[j] * tx[j] - ui[j] * ty[j] + cx;
        ui[j] = ur[j] * ty[j] + ui[j] * tx[j] + cy;
        ur[j] = r;
      }
    }
#pragma unroll
    for (int j = 0; j < NPL; ++j) acc[j] += ur[j];
  }
  if constexpr (NPL == 4) {
    *(double2*)(V + (size_t)leaf * n + 4 * lane) = make_double2(kInv2Pi * acc[0], kInv2Pi * acc[1]);
    *(double2*)(V + (size_t)leaf * n + 4 * lane + 2) = make_double2(kInv2Pi * acc[2], kInv2Pi * acc[3]);
  } else {
#pragma unroll
    for (int j = 0; j < NPL; ++j)
      if (lane + 64 * j < n) V[(size_t)leaf * n + lane + 64 * j] = kInv2Pi * acc[j];
  }
}

// -------------------------------------------------------------------------
// Values of leaf-grid data at arbitrary points (e.g. boundary nodes): the leaf
// holding a point is found by descending the tree from the root (children in
// Morton order, a point on a box edge goes to the upper/right child); the value
// is the tensor interpolant of the leaf's K x K first-kind Chebyshev samples,
// evaluated by the barycentric formula with weights (-1)^a sin((2a+1)pi/2K).
// Points outside the root box get NaN.  One thread per point.
__global__ void k_interp(int K, double root_cx, double root_cy, double root_size, const int* __restrict__ box_child0,
                         const int* __restrict__ box_leaf, const double* __restrict__ t,
                         const double* __restrict__ V, long npts, const double* __restrict__ px,
                         const double* __restrict__ py, double* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  const double x = px[i], y = py[i];
  double cx = root_cx, cy = root_cy, h = root_size;
  if (!(fabs(x - cx) <= 0.5 * h && fabs(y - cy) <= 0.5 * h)) {
    out[i] = __builtin_nan("");
    return;
  }
  int b = 0;
  while (box_leaf[b] < 0) {
    const int dx = x >= cx, dy = y >= cy;
    h *= 0.5;
    cx += (dx ? 0.5 : -0.5) * h;
    cy += (dy ? 0.5 : -0.5) * h;
    b = box_child0[b] + dx + 2 * dy;
  }
  const int leaf = box_leaf[b];
  const double xi = 2.0 * (x - cx) / h, eta = 2.0 * (y - cy) / h;
  double lx[kMaxK], ly[kMaxK];
  auto weights = [&](double s, double* l) {
    int hit = -1;
    double sum = 0.0;
    for (int a = 0; a < K; ++a) {
      const double d = s - t[a];
      if (d == 0.0) hit = a;
      const double wa = ((a & 1) ? -1.0 : 1.0) * sin((2 * a + 1) * M_PI / (2 * K));
      l[a] = wa / (d == 0.0 ? 1.0 : d);
      sum += l[a];
    }
    if (hit >= 0) {
      for (int a = 0; a < K; ++a) l[a] = (a == hit) ? 1.0 : 0.0;
    } else {
      const double inv = 1.0 / sum;
      for (int a = 0; a < K; ++a) l[a] *= inv;
    }
  };
  weights(xi, lx);
  weights(eta, ly);
  const double* v = V + (size_t)leaf * K * K;
  double acc = 0.0;
  for (int a = 0; a < K; ++a) {
    double g = 0.0;
    for (int c = 0; c < K; ++c) g += ly[c] * v[a * K + c];
    acc += lx[a] * g;
  }
  out[i] = acc;
}

int launch_interp(Plan* p, const double* V, long npts, const double* px, const double* py, double* out,
                  hipStream_t s, std::string& err) {
  Context* c = p->ctx;
  const Tables& T = c->T;
  if (!c->D.ready) {
    int rc = upload_tables(c, err);
    if (rc) return rc;
  }
  if (!p->D.ready) {
    int rc = upload_plan(p, err);
    if (rc) return rc;
  }
  if (npts <= 0) return VFX_OK;
  const long blocks = (npts + 255) / 256;
  hipLaunchKernelGGL(k_interp, dim3((unsigned)blocks), dim3(256), 0, s, T.K, T.root_cx, T.root_cy, T.root_size,
                     p->D.box_child0, p->D.box_leaf, c->D.t, V, npts, px, py, out);
  VFX_HIP(hipGetLastError());
  return VFX_OK;
}

// -------------------------------------------------------------------------
// Net charge A^e = integral of f^e over the tree (Section 6, exterior
// problem: the volume potential then grows like A^e log|x|, which the
// boundary solve must offset).  Each leaf contributes h^2 sum_j w_j f_j with
// w the tensor first-kind Chebyshev (Fejer) weights of the unit square.  Two
// passes with a fixed partition, so the sum order depends on the tree only:
// block b of right-hand side r sums the nodes of leaves [b L/G, (b+1) L/G)
// (each thread a strided share, then a fixed LDS tree) into part[r G + b];
// one block per right-hand side then sums its G partials the same way
// (thread t the partials t, t + 256, ... in order).  G is about L n / 2048
// (eight samples per thread, enough loads in flight without flooding the
// dispatcher with tiny blocks), at least 1 and at most min(L, 2048).
constexpr int kChargeBlocks = 2048;

__device__ __forceinline__ double block_sum_256(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  return red[0];
}

__global__ void __launch_bounds__(256) k_charge_part(int n, int L, int G, double root_size,
                                                     const int* __restrict__ leaf_box, const int* __restrict__ box_level,
                                                     const double* __restrict__ w2, const double* __restrict__ fe,
                                                     long sfe, double* __restrict__ part) {
  __shared__ double red[256];
  fe += blockIdx.y * sfe;
  const int b = blockIdx.x;
  const long l0 = (long)b * L / G, l1 = (long)(b + 1) * L / G;
  double acc = 0.0;
  for (long i = l0 * n + threadIdx.x; i < l1 * n; i += 256) {
    const int leaf = (int)(i / n), j = (int)(i - (long)leaf * n);
    const double h = box_side(root_size, box_level[leaf_box[leaf]]);
    acc += h * h * w2[j] * fe[i];
  }
  const double s = block_sum_256(acc, red);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * G + b] = s;
}

__global__ void __launch_bounds__(256) k_charge_sum(int G, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int q = threadIdx.x; q < G; q += 256) v += part[(size_t)blockIdx.x * G + q];
  const double s = block_sum_256(v, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

int launch_net_charge(Plan* p, const double* fe, int nrhs, double* out, hipStream_t s, std::string& err) {
  Context* c = p->ctx;
  const Tables& T = c->T;
  if (!c->D.ready) {
    int rc = upload_tables(c, err);
    if (rc) return rc;
  }
  if (!p->D.ready) {
    int rc = upload_plan(p, err);
    if (rc) return rc;
  }
  DevicePlan& D = p->D;
  const int L = p->H.L, n = T.n;
  const int G = std::min(L, (int)std::max(1L, std::min((long)kChargeBlocks, (long)L * n / 2048)));
  if (nrhs > D.chg_cap) {
    p->gen++;  // graphs that captured the old buffer are stale
    if (D.chg_part) {
      VFX_HIP(hipDeviceSynchronize());  // no earlier call of this plan in flight
      VFX_HIP(hipFree(D.chg_part));
      D.chg_part = nullptr;
      D.chg_cap = 0;
    }
    VFX_HIP(hipMalloc((void**)&D.chg_part, sizeof(double) * kChargeBlocks * (size_t)nrhs));
    D.chg_cap = nrhs;
  }
  if (G > 0)
    hipLaunchKernelGGL(k_charge_part, dim3(G, nrhs), dim3(256), 0, s, n, L, G, T.root_size, D.leaf_box,
                       D.box_level, c->D.w2, fe, (long)L * n, D.chg_part);
  VFX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_charge_sum, dim3(nrhs), dim3(256), 0, s, G, D.chg_part, out);
  VFX_HIP(hipGetLastError());
  return VFX_OK;
}

// -------------------------------------------------------------------------
// Net charge without allocation (for callers that cannot allocate: code
// under HIP graph capture, tight serving loops).  The block partials go to
// a file-scope device array instead of the plan's buffer: one copy per GPU
// for the life of the process, kNoallocMaxRhs right-hand sides of
// kChargeBlocks partials (1 MiB).  Host code never names the array in a
// launch or a copy: on each device it asks hipGetSymbolAddress for that
// device's copy once (with the device current) and passes the address it
// returns.  Every partial the sum reads is written by the same call first,
// so nothing needs clearing; two calls that overlap on one GPU race on it.
constexpr int kNoallocMaxRhs = 64;
static __device__ __align__(256) double scratch[kChargeBlocks * kNoallocMaxRhs];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(int dev, void** out, std::string& err) {
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device ordinal out of range";
    return VFX_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    VFX_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      err = "hipGetSymbolAddress returned a null address";
      return VFX_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return VFX_OK;
}

int noalloc_max_rhs() { return kNoallocMaxRhs; }

int launch_net_charge_noalloc(Plan* p, const double* fe, int nrhs, double* out, hipStream_t s, std::string& err) {
  Context* c = p->ctx;
  if (!c->D.ready || !p->D.ready) {
    err = "the plan's device data are not resident (run vfx_execute or vfx_net_charge on it once first)";
    return VFX_EINVAL;
  }
  if (nrhs > kNoallocMaxRhs) {
    err = "nrhs exceeds the allocation-free limit of " + std::to_string(kNoallocMaxRhs);
    return VFX_EINVAL;
  }
  int dev = -1;
  VFX_HIP(hipGetDevice(&dev));
  if (dev != c->D.device) {
    err = "the current device is not the one holding the plan's data";
    return VFX_EINVAL;
  }
  void* ptr = nullptr;
  int rc = scratch_address(dev, &ptr, err);
  if (rc) return rc;
  double* part = static_cast<double*>(ptr);
  const Tables& T = c->T;
  const DevicePlan& D = p->D;
  const int L = p->H.L, n = T.n;
  const int G = std::min(L, (int)std::max(1L, std::min((long)kChargeBlocks, (long)L * n / 2048)));
  if (G > 0)
    hipLaunchKernelGGL(k_charge_part, dim3(G, nrhs), dim3(256), 0, s, n, L, G, T.root_size, D.leaf_box,
                       D.box_level, c->D.w2, fe, (long)L * n, part);
  VFX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_charge_sum, dim3(nrhs), dim3(256), 0, s, G, part, out);
  VFX_HIP(hipGetLastError());
  return VFX_OK;
}

// -------------------------------------------------------------------------
template <typename T>
static int upload(T** dst, const T* src, size_t count, std::string& err) {
  *dst = nullptr;
  if (count == 0) return VFX_OK;
  VFX_HIP(hipMalloc((void**)dst, count * sizeof(T)));
  VFX_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return VFX_OK;
}

#define UP(dst, vec)                                                       \
  do {                                                                     \
    int rc_ = upload(&(dst), (vec).data(), (vec).size(), err);             \
    if (rc_) return rc_;                                                   \
  } while (0)

static std::vector<double2> as_complex(const std::vector<double>& src) {
  std::vector<double2> o(src.size() / 2);
  for (size_t i = 0; i < o.size(); ++i) o[i] = make_double2(src[2 * i], src[2 * i + 1]);
  return o;
}

int upload_tables(Context* c, std::string& err) {
  const Tables& T = c->T;
  DeviceTables& D = c->D;
  const int n = T.n, P = T.p + 1;
  UP(D.t, T.t);
  UP(D.tbar, T.tbar);
  UP(D.w2, T.w2);
  UP(D.AbarT, T.AbarT);
  UP(D.A, T.A);
  UP(D.cbar, T.cbar);
  UP(D.near, T.near);
  UP(D.lr_R, T.lr_R);
  UP(D.lr_W, T.lr_W);
  UP(D.lr_Q, T.lr_Q);
  UP(D.fx_W, T.fx_W);
  UP(D.fx_Wexp, T.fx_Wexp);
  if (T.ts_ok) {
    UP(D.cls_R, T.cls_R);
    UP(D.lr_Wp, T.lr_Wp);
    UP(D.cls_QT, T.cls_QT);
    UP(D.self_T, T.self_T);
  }
  UP(D.fx_Q, T.fx_Q);
  UP(D.fx_Qexp, T.fx_Qexp);
  UP(D.fx_A, T.fx_A);
  UP(D.fx_Aexp, T.fx_Aexp);
  UP(D.f8_W, T.f8_W);
  UP(D.f8_Wexp, T.f8_Wexp);
  UP(D.f8_Q, T.f8_Q);
  UP(D.f8_Qexp, T.f8_Qexp);
  UP(D.f8_A, T.f8_A);
  UP(D.f8_Aexp, T.f8_Aexp);
  UP(D.p2l_gemm, T.p2l_gemm);
  UP(D.m2p_gemm, T.m2p_gemm);
  UP(D.p2m_gemm, T.p2m_gemm);
  UP(D.pas_m2l, T.pas_m2l);
  UP(D.pas_m2l_t, T.pas_m2l_t);
  UP(D.pas_m2m_t, T.pas_m2m_t);
  UP(D.pas_l2l_t, T.pas_l2l_t);
  UP(D.pas_m2m, T.pas_m2m);
  UP(D.pas_l2l, T.pas_l2l);
  UP(D.m2l_logd, T.m2l_logd);
  std::vector<double2> v;
  // p2m [k][j] -> [j][k]
  v.assign((size_t)n * P, make_double2(0, 0));
  for (int k = 0; k < P; ++k)
    for (int j = 0; j < n; ++j)
      v[(size_t)j * P + k] = make_double2(T.p2m[2 * ((size_t)k * n + j)], T.p2m[2 * ((size_t)k * n + j) + 1]);
  UP(D.p2m, v);
  // l2p [i][l] -> [l][i]
  v.assign((size_t)n * P, make_double2(0, 0));
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < P; ++l)
      v[(size_t)l * n + i] = make_double2(T.l2p[2 * ((size_t)i * P + l)], T.l2p[2 * ((size_t)i * P + l) + 1]);
  UP(D.l2p, v);
  v = as_complex(T.m2l_tpow);
  UP(D.m2l_tpow, v);
  v = as_complex(T.m2l_tneg);
  UP(D.m2l_tneg, v);
  v = as_complex(T.m2m_in);
  UP(D.m2m_in, v);
  v = as_complex(T.m2m_out);
  UP(D.m2m_out, v);
  v = as_complex(T.l2l_in);
  UP(D.l2l_in, v);
  v = as_complex(T.l2l_out);
  UP(D.l2l_out, v);
  VFX_HIP(hipGetDevice(&D.device));
  D.ready = true;
  return VFX_OK;
}

void free_tables_device(Context* c) {
  DeviceTables& D = c->D;
  c->gen++;
  void* ptrs[] = {D.t,        D.tbar,     D.w2,       D.AbarT,   D.cbar,     D.near,    D.near_s2,   D.A,
                  D.p2m,      D.l2p,      D.m2m,      D.l2l,     D.m2l,      D.p2l,     D.p2l_area,
                  D.pas_m2l,  D.pas_m2m,  D.pas_l2l,  D.m2l_logd, D.p2l_gemm, D.m2p_gemm, D.m2l_tpow, D.m2l_tneg, D.p2m_gemm,
                  D.m2m_in,   D.m2m_out,  D.l2l_in,   D.l2l_out,  D.pas_m2l_t, D.pas_m2m_t, D.pas_l2l_t,
                  D.lr_R,     D.lr_W,     D.lr_Q,     D.fx_W,     D.fx_Q,     D.fx_A,     D.fx_Wexp,
                  D.fx_Qexp,  D.fx_Aexp,  D.f8_W,     D.f8_Q,     D.f8_A,     D.f8_Wexp,  D.f8_Qexp,  D.f8_Aexp,
                  D.cls_R,    D.lr_Wp,    D.cls_QT,   D.self_T};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  D = DeviceTables();
}

// Buffers that hold one copy per right-hand side (expansions, near-field
// partials, P2L partials, leaf local expansions, bf16 slices): reallocated
// for `nrhs` copies when a larger batch is requested.
int ensure_rhs_capacity(Plan* p, int nrhs, std::string& err) {
  const HostPlan& H = p->H;
  DevicePlan& D = p->D;
  const Tables& T = p->ctx->T;
  const size_t P = T.p + 1, R = (size_t)nrhs;
  if (D.cap > 0) (void)hipDeviceSynchronize();  // no execute of this plan in flight
  p->gen++;  // graphs that captured the old buffers are stale
  void* old[] = {D.mpole, D.local, D.near_y, D.p2l_y, D.up_part, D.locf, D.xs, D.m2p_y, D.xs_exp, D.near_z,
                 D.ext_fg, D.ext_g};
  for (void* q : old)
    if (q) (void)hipFree(q);
  D.mpole = D.local = D.up_part = D.locf = nullptr;
  D.near_y = D.p2l_y = D.m2p_y = D.near_z = nullptr;
  D.xs = nullptr;
  D.xs_exp = nullptr;
  D.ext_fg = D.ext_g = nullptr;
  D.cap = 0;
  VFX_HIP(hipMalloc((void**)&D.mpole, sizeof(double2) * (size_t)H.B * P * R));
  VFX_HIP(hipMalloc((void**)&D.local, sizeof(double2) * (size_t)H.B * P * R));
  VFX_HIP(hipMemset(D.local, 0, sizeof(double2) * (size_t)H.B * P * R));
  if (!H.np_src.empty() && !H.ts) VFX_HIP(hipMalloc((void**)&D.near_y, sizeof(double) * H.np_src.size() * T.n * R));
  if (!H.np_src.empty() && H.ts)
    VFX_HIP(hipMalloc((void**)&D.near_z, sizeof(double) * H.np_src.size() * kNearLrMax * R));
  if (!H.p4_src.empty()) VFX_HIP(hipMalloc((void**)&D.p2l_y, sizeof(double) * H.p4_src.size() * T.p2l_rows * R));
  if (!H.p3_src.empty()) VFX_HIP(hipMalloc((void**)&D.m2p_y, sizeof(double) * H.p3_src.size() * T.n * R));
  if (H.up_slots > 0) VFX_HIP(hipMalloc((void**)&D.up_part, sizeof(double2) * (size_t)H.up_slots * P * R));
  VFX_HIP(hipMalloc((void**)&D.locf, sizeof(double2) * (size_t)H.L * P * R));
  if (H.precision >= 1 && !H.ts) {  // bf16 slices (mode 1) or int8 slices (mode 2, 5/8 of the size)
    VFX_HIP(hipMalloc((void**)&D.xs, sizeof(uint16_t) * 4 * (size_t)H.L * T.n * R));
    VFX_HIP(hipMalloc((void**)&D.xs_exp, sizeof(int) * (size_t)H.L * R));
  }
  if (nrhs >= kExtGemmMinRhs && H.ncut > 0) {
    VFX_HIP(hipMalloc((void**)&D.ext_fg, sizeof(double) * (size_t)H.ncut * R * T.nG));
    VFX_HIP(hipMalloc((void**)&D.ext_g, sizeof(double) * (size_t)H.ncut * R * T.Kbar * T.Kbar));
  }
  D.cap = nrhs;
  return VFX_OK;
}

int upload_plan(Plan* p, std::string& err) {
  const HostPlan& H = p->H;
  DevicePlan& D = p->D;
  const Tables& T = p->ctx->T;
  const int P = T.p + 1;
  UP(D.box_level, H.box_level);
  UP(D.box_child0, H.box_child0);
  UP(D.box_leaf, H.box_leaf);
  UP(D.box_parent, H.box_parent);
  UP(D.box_cx, H.box_cx);
  UP(D.box_cy, H.box_cy);
  UP(D.leaf_box, H.leaf_box);
  UP(D.kind, H.kind);
  {
    // where each leaf's f^e comes from: 2 an extension list, 1 f (regular), 0 zero
    std::vector<int8_t> src(H.L, 0);
    for (int i = 0; i < H.L; ++i) src[i] = H.owner[i] >= 0 ? 2 : (H.kind[i] == 1 ? 1 : 0);
    UP(D.fe_src, src);
  }
  UP(D.l1_ptr, H.l1_ptr);
  UP(D.l1_src, H.l1_src);
  UP(D.l1_cfg, H.l1_cfg);
  UP(D.l1_srcbox, H.l1_srcbox);
  UP(D.l2_ptr, H.l2_ptr);
  UP(D.l2_src, H.l2_src);
  UP(D.l2_off, H.l2_off);
  UP(D.l2_tgt, H.l2_tgt);
  UP(D.m2l_grp, H.m2l_grp);
  UP(D.l3_ptr, H.l3_ptr);
  UP(D.l3_src, H.l3_src);
  UP(D.anc_ptr, H.anc_ptr);
  UP(D.anc, H.anc);
  UP(D.anc_leaf, H.anc_leaf);
  UP(D.dn_grp, H.dn_grp);

  UP(D.up_box, H.up_box);
  UP(D.up_ptr, H.up_ptr);
  UP(D.up_src, H.up_src);
  UP(D.up_pos, H.up_pos);
  UP(D.up_grp, H.up_grp);
  UP(D.up_split, H.up_split);
  UP(D.l4_ptr, H.l4_ptr);
  UP(D.l4_src, H.l4_src);
  UP(D.l4_cfg, H.l4_cfg);
  UP(D.np_src, H.np_src);
  UP(D.l1_slot, H.l1_slot);
  UP(D.nt_cfg, H.nt_cfg);
  UP(D.nt_first, H.nt_first);
  UP(D.nt_count, H.nt_count);
  UP(D.nl_cfg, H.nl_cfg);
  UP(D.nl_first, H.nl_first);
  UP(D.nl_count, H.nl_count);
  UP(D.mt_cfg, H.mt_cfg);
  UP(D.mt_first, H.mt_first);
  UP(D.mt_count, H.mt_count);
  UP(D.ml_cfg, H.ml_cfg);
  UP(D.ml_first, H.ml_first);
  UP(D.ml_count, H.ml_count);
  UP(D.ts_grp, H.ts_grp);
  UP(D.ts_tcls, H.ts_tcls);
  UP(D.ts_row, H.ts_row);
  UP(D.ts_code, H.ts_code);

  UP(D.p4_src, H.p4_src);
  UP(D.l4_slot, H.l4_slot);
  UP(D.t4_cfg, H.t4_cfg);
  UP(D.t4_first, H.t4_first);
  UP(D.t4_count, H.t4_count);
  UP(D.p3_src, H.p3_src);
  UP(D.l3_slot, H.l3_slot);
  UP(D.t3_cfg, H.t3_cfg);
  UP(D.t3_first, H.t3_first);
  UP(D.t3_count, H.t3_count);
  UP(D.t0_cfg, H.t0_cfg);
  UP(D.t0_first, H.t0_first);
  UP(D.t0_count, H.t0_count);
  UP(D.leaf_ids, H.leaf_ids);

  UP(D.cut_leaf, H.cut_leaf);
  UP(D.ext_ptr, H.ext_ptr);
  UP(D.ext_tgt, H.ext_tgt);
  UP(D.ext_geo, H.ext_geo);
  UP(D.pinv_ptr, H.pinv_ptr);
  UP(D.pinv_idx, H.pinv_idx);
  if (H.factored) {
    UP(D.pinv_val, H.pinv_val);
  } else if (H.ncut > 0) {
    VFX_HIP(hipMalloc((void**)&D.pinv_val, sizeof(double) * (size_t)H.pinv_ptr[H.ncut] * T.nG));
  }
  D.factored = H.factored;
  UP(D.sbar_given, H.sbar_given);
  D.cap = 0;
  {
    int rc = ensure_rhs_capacity(p, 1, err);
    if (rc) return rc;
  }
  VFX_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
  VFX_HIP(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
  VFX_HIP(hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming));
  VFX_HIP(hipEventCreateWithFlags(&p->p2l_ev, hipEventDisableTiming));
  VFX_HIP(hipEventCreateWithFlags(&p->up_ev, hipEventDisableTiming));
  D.ready = true;
  return VFX_OK;
}

void free_plan_device(Plan* p) {
  DevicePlan& D = p->D;
  if (D.ready) (void)hipDeviceSynchronize();  // no execute of this plan in flight
  p->gen++;
  void* ptrs[] = {D.box_level, D.box_child0, D.box_leaf, D.box_parent, D.box_cx,   D.box_cy,   D.leaf_box,
                  D.kind,      D.l1_ptr,     D.l1_src,   D.l1_cfg,     D.l2_ptr,   D.l2_src,   D.l2_off,
                  D.l3_ptr,    D.l3_src,     D.l4_ptr,   D.l4_src,     D.l4_cfg,   D.np_src,   D.l1_slot,
                  D.nt_cfg,    D.nt_first,   D.nt_count, D.near_y,     D.p4_src,   D.l4_slot,  D.t4_cfg,
                  D.t4_first,  D.t4_count,   D.p2l_y,    D.cut_leaf,   D.ext_ptr,  D.ext_tgt,  D.pinv_ptr,
                  D.pinv_idx,  D.pinv_val,   D.sbar_given, D.mpole,    D.local,    D.t0_cfg,   D.t0_first,
                  D.t0_count,  D.leaf_ids,   D.l2_tgt,   D.m2l_grp,  D.up_box,   D.up_ptr,   D.up_src,
                  D.up_pos,    D.up_split,   D.up_grp,   D.up_part,  D.anc_ptr,  D.anc,
                  D.nl_cfg,    D.nl_first,   D.nl_count, D.l1_srcbox,  D.ext_geo,
                  D.anc_leaf,  D.dn_grp,     D.locf,     D.mt_cfg,   D.mt_first, D.mt_count, D.ml_cfg, D.fac_ws,
                  D.ml_first,  D.ml_count,   D.xs,       D.p3_src,   D.l3_slot,  D.t3_cfg,   D.t3_first,
                  D.t3_count,  D.m2p_y,    D.xs_exp,   D.chg_part, D.near_z, D.ts_grp, D.ts_tcls,
                  D.ts_row,    D.ts_code,  D.fe_src};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  D = DevicePlan();
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  p->ev.clear();
  p->n_timed = 0;
  if (p->side) (void)hipStreamSynchronize(p->side);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  if (p->join_ev) (void)hipEventDestroy(p->join_ev);
  if (p->p2l_ev) (void)hipEventDestroy(p->p2l_ev);
  if (p->up_ev) (void)hipEventDestroy(p->up_ev);
  if (p->side) (void)hipStreamDestroy(p->side);
  p->fork_ev = p->join_ev = p->p2l_ev = p->up_ev = nullptr;
  p->side = nullptr;
}

// Grid of a persistent, XCD-aware kernel: at most max_wgs work-groups (0 =
// one per item), but never fewer than min(items, 8) - the kernels split
// their items into eight contiguous ranges walked by the work-groups of one
// XCD each (blockIdx % 8), so every range needs a work-group.
static int persistent_grid(int items, int max_wgs) {
  int grid = (max_wgs > 0 && items > max_wgs) ? max_wgs : items;
  return std::max(grid, std::min(items, 8));
}

template <int KD, int EPI, int TE, int MTB>
static void launch_gemm(int ntiles, int MT, const int* cfg, const int* first, const int* count, const int* src,
                        const double* A, const double* X, double* Y, int P2, double root, const int* leaf_box,
                        const int* box_level, hipStream_t s, int max_wgs, unsigned R, long sx, long sy,
                        int ldx = KD, int kx = KD) {
  const int items = ntiles * (MT / MTB);
  const int grid = persistent_grid(items, max_wgs);
  if constexpr (TE == 64 && KD % 32 == 0)
    hipLaunchKernelGGL((k_tgemm<KD, MTB, EPI>), dim3(grid, R), dim3(256), 0, s, items, MT, cfg, first, count, src, A,
                       X, Y, sx, sy, ldx, kx, P2, root, leaf_box, box_level);
  else
    hipLaunchKernelGGL((k_gemm<KD, EPI, TE, MTB>), dim3(grid, R), dim3(256), 0, s, items, MT, cfg, first, count,
                       src, A, X, Y, P2, root, leaf_box, box_level, sx, sy, ldx, kx);
}

// Dense near-field tables: MT = n/16 row tiles (1, 4, 9 or 16 for K = 4, 8,
// 12, 16), in blocks of MTB = 1, 4, 9, 4.
static void near_gemm(int n, int ntiles, const int* cfg, const int* first, const int* count, const int* src,
                      const double* A, const double* X, double* Y, hipStream_t s, int max_wgs, int mtb, unsigned R,
                      long sx, long sy) {
  if (ntiles <= 0) return;
  const int MT = n / 16;
#define VFX_NG(KDV, MTBV) \
  launch_gemm<KDV, 0, 64, MTBV>(ntiles, MT, cfg, first, count, src, A, X, Y, 0, 0, nullptr, nullptr, s, max_wgs, R, sx, sy)
  switch (n) {
    case 16: VFX_NG(16, 1); break;
    case 64: VFX_NG(64, 4); break;
    case 144: VFX_NG(144, 9); break;
    default:
      if (mtb == 8)
        VFX_NG(256, 8);
      else
        VFX_NG(256, 4);
      break;
  }
#undef VFX_NG
}

// P2L (EPI 0, TE 64) and P2M (EPI 1, TE 64) tables: rows padded to a
// multiple of 64, so MT is 4 or 8; P2L takes them in one row block, P2M
// (one tile per 64 leaves, few tiles) two row tiles per work item on the
// pipelined kernel, for more items in flight (one row tile per item rereads
// the leaf data four times, four per item leaves most CUs idle).
template <int EPI, int TE>
static void expansion_gemm(int n, int ntiles, int MT, const int* cfg, const int* first, const int* count,
                           const int* src, const double* A, const double* X, double* Y, hipStream_t s, unsigned R,
                           long sx, long sy, int P2 = 0, double root = 0, const int* leaf_box = nullptr,
                           const int* box_level = nullptr) {
  if (ntiles <= 0) return;
#define VFX_EXP_CASE(KDV)                                                                                       \
  do {                                                                                                          \
    if (EPI == 1 && KDV % 32 == 0)                                                                              \
      launch_gemm<KDV, EPI, TE, 2>(ntiles, MT, cfg, first, count, src, A, X, Y, P2, root, leaf_box, box_level, s, 0, \
                                   R, sx, sy);                                                                  \
    else if (MT == 4)                                                                                           \
      launch_gemm<KDV, EPI, TE, 4>(ntiles, MT, cfg, first, count, src, A, X, Y, P2, root, leaf_box, box_level, s, 0, \
                                   R, sx, sy);                                                                  \
    else                                                                                                        \
      launch_gemm<KDV, EPI, TE, 8>(ntiles, MT, cfg, first, count, src, A, X, Y, P2, root, leaf_box, box_level, s, 0, \
                                   R, sx, sy);                                                                  \
  } while (0)
  switch (n) {
    case 16: VFX_EXP_CASE(16); break;
    case 64: VFX_EXP_CASE(64); break;
    case 144: VFX_EXP_CASE(144); break;
    default: VFX_EXP_CASE(256); break;
  }
#undef VFX_EXP_CASE
}

// M2P tables: contraction over the 2P real coefficients of a multipole
// (padded to KD = 64 or 128), n = K^2 rows in blocks as for the dense near
// field.
static void m2p_gemm(int n, int kd, int P2, int ntiles, const int* cfg, const int* first, const int* count,
                     const int* src, const double* A, const double* X, double* Y, hipStream_t s, unsigned R, long sx,
                     long sy) {
  if (ntiles <= 0) return;
  const int MT = n / 16;
#define VFX_M2P(KDV, MTBV)                                                                                        \
  launch_gemm<KDV, 0, 64, MTBV>(ntiles, MT, cfg, first, count, src, A, X, Y, 0, 0, nullptr, nullptr, s, 0, R, sx, \
                                sy, P2, P2)
#define VFX_M2P_N(KDV)            \
  switch (n) {                    \
    case 16: VFX_M2P(KDV, 1); break;  \
    case 64: VFX_M2P(KDV, 4); break;  \
    case 144: VFX_M2P(KDV, 9); break; \
    default: VFX_M2P(KDV, 4); break;  \
  }
  if (kd == 64) {
    VFX_M2P_N(64)
  } else {
    VFX_M2P_N(128)
  }
#undef VFX_M2P_N
#undef VFX_M2P
}

int launch_execute(Plan* p, int nrhs, const double* f_leaf, const double* f_cut, double* fe, double* V,
                   hipStream_t s, std::string& err) {
  Context* c = p->ctx;
  const Tables& T = c->T;
  if (!c->D.ready) {
    int rc = upload_tables(c, err);
    if (rc) return rc;
  }
  if (!p->D.ready) {
    int rc = upload_plan(p, err);
    if (rc) return rc;
  }
  if (nrhs > p->D.cap) {
    int rc = ensure_rhs_capacity(p, nrhs, err);
    if (rc) return rc;
  }
  if (!p->D.factored) {
    err = "the plan defers its least-squares operators to the GPU: call vfx_plan_factor_gpu first";
    return VFX_EINVAL;
  }
  const HostPlan& H = p->H;
  const DeviceTables& DT = c->D;
  const DevicePlan& D = p->D;
  const int n = T.n, P = T.p + 1, L = H.L;
  // per-right-hand-side strides (elements) of the batched buffers
  const long sFL = (long)L * n, sFC = (long)H.ncut * T.nX, sMP = (long)H.B * P;
  const long sNY = (long)H.np_src.size() * n, sPL = (long)H.p4_src.size() * T.p2l_rows;
  const long sNZ = (long)H.np_src.size() * kNearLrMax;
  const long sM3 = (long)H.p3_src.size() * n;
  const long sUP = (long)H.up_slots * P, sLF = (long)L * P;
  const unsigned R = (unsigned)nrhs;
    constexpr int kMaxTimed = 4096;
  constexpr int NE = Plan::kEvents;
  const bool timed = p->timing && p->n_timed < kMaxTimed;
  const size_t ev0 = (size_t)p->n_timed * NE;
  if (timed && p->ev.size() < ev0 + NE) {
    for (int k = 0; k < NE; ++k) {
      hipEvent_t e;
      VFX_HIP(hipEventCreate(&e));
      p->ev.push_back(e);
    }
  }
  // events on the caller's stream: 0 start, 12 after f^e initialisation, 1
  // after the extension, 2 after P2M and the upward pass, 3 after M2L, 4
  // after the downward pass, 8 after the join, 9 end; on the side stream: 10
  // start, 5 after P2L, 6 after the first near-field kernel (low-rank pairs,
  // or the factor products of the target-stationary path), 7 after the
  // second (dense pairs, or the per-target-group kernel), 13 after the wait
  // for the upward pass, 11 after M2P
  auto mark = [&](int k, hipStream_t st) -> int {
    if (timed) {
      hipError_t e = hipEventRecord(p->ev[ev0 + k], st);
      if (e != hipSuccess) {
        err = std::string("hipEventRecord: ") + hipGetErrorString(e);
        return VFX_EHIP;
      }
    }
    return VFX_OK;
  };
#define MARK(k, st)          \
  do {                       \
    int rc_ = mark(k, st);   \
    if (rc_) return rc_;     \
  } while (0)
  MARK(0, s);
  MARK(12, s);
  {
    // the extension of every cut leaf, and in the same launch the f^e
    // initialisation of the other leaves
    const int ext_blocks = H.ncut * nrhs;
    const long pieces = (long)L * n / 2 * nrhs;
    const int copy_blocks = (int)std::min<long>((pieces + 255) / 256, 1024);
    // a batch of at least kExtGemmMinRhs right-hand sides: A1 and A2 as
    // MFMA GEMMs, then the Chebyshev step and the evaluation for eight
    // right-hand sides per work-group; the extension kernel only
    // initialises the leaves no extension list writes
    const bool gemm = nrhs >= kExtGemmMinRhs && H.ncut > 0;
    if (gemm) {
      int rc = launch_ext_gemm(p, f_cut, nrhs, s, err);
      if (!rc) rc = launch_ext_eval(p, f_cut, fe, nrhs, s, err);
      if (rc) return rc;
    }
    const int blocks1 = gemm ? 0 : ext_blocks;
    hipLaunchKernelGGL(k_extension, dim3(blocks1 + copy_blocks), dim3(256), 0, s, T.K, T.Kbar, T.nX, T.nG,
                       D.pinv_ptr, D.pinv_idx, D.pinv_val, D.sbar_given, D.ext_ptr, D.ext_tgt, D.ext_geo, DT.t,
                       DT.AbarT, DT.cbar, f_cut, fe, nrhs, sFC, sFL, blocks1, L, D.fe_src, f_leaf);
  }
  VFX_HIP(hipGetLastError());
  MARK(1, s);
  // fork: P2L and the near field on the side stream, concurrent with P2M,
  // the upward pass, M2L and the downward pass on the caller's stream.  The
  // near-field grids are bounded (about two work-groups per CU, looping over
  // the tiles).
  VFX_HIP(hipEventRecord(p->fork_ev, s));
  VFX_HIP(hipStreamWaitEvent(p->side, p->fork_ev, 0));
  // P2L first on the side stream (it needs only f^e; M2L on the caller's
  // stream waits for it), then the near field
  MARK(10, p->side);
  if (H.nlev > 2)
    expansion_gemm<0, 64>(n, (int)H.t4_cfg.size(), T.p2l_rows / 16, D.t4_cfg, D.t4_first, D.t4_count, D.p4_src,
                          DT.p2l_gemm, fe, D.p2l_y, p->side, R, sFL, sPL);
  VFX_HIP(hipGetLastError());
  VFX_HIP(hipEventRecord(p->p2l_ev, p->side));
  MARK(5, p->side);
  const long total = (long)L * n;
  if (H.ts) {
    // target-stationary near field: the factor products Z = (W_b P_g^T) f
    // of every non-self pair (table GEMM over the configuration-major
    // tiles), then the per-target-group kernel, which leaves h^2 times each
    // leaf's list-1 table sum in V
    if (!H.nl_cfg.empty())
      launch_gemm<256, 0, 64, 4>((int)H.nl_cfg.size(), 4, D.nl_cfg, D.nl_first, D.nl_count, D.np_src, DT.lr_Wp, fe,
                                 D.near_z, 0, 0, nullptr, nullptr, p->side, p->tune.near_wgs, R, sFL, sNZ);
    VFX_HIP(hipGetLastError());
    MARK(6, p->side);
    {
      int rc = launch_near_ts(p, fe, V, nrhs, p->tune.near_wgs, p->side, err);
      if (rc) return rc;
    }
  } else {
    if (!H.nl_cfg.empty()) {
      const int items = (int)H.nl_cfg.size();
      hipLaunchKernelGGL(k_near_lr<256>, dim3(persistent_grid(items, p->tune.near_wgs), R), dim3(256), 0, p->side, items,
                         D.nl_cfg, D.nl_first, D.nl_count, D.np_src, DT.lr_R, DT.lr_W, DT.lr_Q, fe, D.near_y, sFL,
                         sNY);
    }
    if (H.precision >= 1) {
      // pairs in mixed precision: fixed-point bf16 (mode 1) or int8 (mode 2)
      // slices of the leaf data, then their low-rank and self products (FP64
      // results, same buffer)
      int rc = H.precision == 2 ? launch_near_f8(p, fe, nrhs, p->tune.near_wgs, p->side, err)
                                : launch_near_fx(p, fe, nrhs, p->tune.near_wgs, p->side, err);
      if (rc) return rc;
    }
    VFX_HIP(hipGetLastError());
    MARK(6, p->side);
    near_gemm(n, (int)H.nt_cfg.size(), D.nt_cfg, D.nt_first, D.nt_count, D.np_src, DT.near, fe, D.near_y, p->side,
              p->tune.near_wgs, p->tune.dense_mtb, R, sFL, sNY);
  }
  VFX_HIP(hipGetLastError());
  MARK(7, p->side);
  // multipoles of the leaves
  expansion_gemm<1, 64>(n, (int)H.t0_first.size(), T.p2l_rows / 16, D.t0_cfg, D.t0_first, D.t0_count, D.leaf_ids,
                        DT.p2m_gemm, fe, (double*)D.mpole, s, R, sFL, 2 * sMP, 2 * P, T.root_size, D.leaf_box,
                        D.box_level);
  if (!H.up_grp.empty()) {
    const int ng = (int)H.up_grp.size() / 5;
#define VFX_UP(PMV, EX)                                                                                            \
  hipLaunchKernelGGL((k_up<PMV, EX>), dim3(ng, R, (P + 7) / 8), dim3(64), 0, s, P, T.root_size, D.up_grp, D.up_box, D.up_ptr,  \
                     D.up_src, D.up_pos, D.box_level, D.box_cx, D.box_cy, DT.pas_m2m_t, D.mpole, D.up_part, sMP,  \
                     sUP)
    if (P == 21)
      VFX_UP(21, true);
    else if (P == 25)
      VFX_UP(25, true);
    else if (P == 31)
      VFX_UP(31, true);
    else if (P == 41)
      VFX_UP(41, true);
    else if (P <= 32)
      VFX_UP(32, false);
    else
      VFX_UP(64, false);
#undef VFX_UP
    if (!H.up_split.empty())
      hipLaunchKernelGGL(k_up_sum, dim3((int)H.up_split.size() / 3, R), dim3(64), 0, s, P, D.up_split, D.up_part,
                         D.mpole, sUP, sMP);
  }
  VFX_HIP(hipGetLastError());
  MARK(2, s);
  // M2P for list 3 on the side stream, behind the near field, once the
  // upward pass is done; the side stream then joins the caller's
  VFX_HIP(hipEventRecord(p->up_ev, s));
  VFX_HIP(hipStreamWaitEvent(p->side, p->up_ev, 0));
  MARK(13, p->side);
  m2p_gemm(n, T.p2l_rows, 2 * P, (int)H.t3_cfg.size(), D.t3_cfg, D.t3_first, D.t3_count, D.p3_src, DT.m2p_gemm,
           (const double*)D.mpole, D.m2p_y, p->side, R, 2 * sMP, sM3);
  VFX_HIP(hipGetLastError());
  MARK(11, p->side);
  VFX_HIP(hipEventRecord(p->join_ev, p->side));
  if (H.nlev > 2) {
    VFX_HIP(hipStreamWaitEvent(s, p->p2l_ev, 0));  // list-4 products from the side stream
    const int ng = (int)H.m2l_grp.size() - 1;
    if (ng > 0) {
#define VFX_M2L(PMV)                                                                                             \
  hipLaunchKernelGGL(k_m2l_pairs<PMV>, dim3(ng, R), dim3(64), 0, s, P, T.root_size, D.m2l_grp, D.box_level,      \
                     D.l2_ptr, D.l2_src, D.l2_off, D.l2_tgt, D.l4_ptr, D.l4_src, D.l4_slot, D.leaf_box, T.p2l_rows, \
                     DT.pas_m2l_t, DT.m2l_logd, D.mpole, D.p2l_y, D.local, sMP, sPL)
#define VFX_M2LL(PV)                                                                                             \
  hipLaunchKernelGGL(k_m2l_lanes<PV>, dim3(ng, R), dim3(64), 0, s, T.root_size, D.m2l_grp, D.box_level,          \
                     D.l2_ptr, D.l2_src, D.l2_off, D.l2_tgt, D.l4_ptr, D.l4_src, D.l4_slot, D.leaf_box, T.p2l_rows, \
                     DT.pas_m2l_t, DT.m2l_logd, D.mpole, D.p2l_y, D.local, sMP, sPL)
      if (P == 21)
        VFX_M2LL(21);
      else if (P == 25)
        VFX_M2LL(25);
      else if (P == 31)
        VFX_M2LL(31);
      else if (P == 41)
        VFX_M2LL(41);
      else if (P <= 32)
        VFX_M2L(32);
      else
        VFX_M2L(64);
#undef VFX_M2L
#undef VFX_M2LL
    }
  }
  VFX_HIP(hipGetLastError());
  MARK(3, s);
  // full local expansions of the leaves (downward pass)
  {
    const int ng = (int)H.dn_grp.size() - 1;
#define VFX_DOWN(PMV, EX)                                                                                          \
  hipLaunchKernelGGL((k_down<PMV, EX>), dim3(ng, R, (P + 7) / 8), dim3(64), 0, s, P, T.root_size, D.dn_grp, D.anc_ptr, D.anc,   \
                     D.anc_leaf, D.leaf_box, D.box_level, D.box_cx, D.box_cy, DT.pas_l2l_t, D.local, D.locf, sMP,  \
                     sLF)
    if (P == 21)
      VFX_DOWN(21, true);
    else if (P == 25)
      VFX_DOWN(25, true);
    else if (P == 31)
      VFX_DOWN(31, true);
    else if (P == 41)
      VFX_DOWN(41, true);
    else if (P <= 32)
      VFX_DOWN(32, false);
    else
      VFX_DOWN(64, false);
#undef VFX_DOWN
  }
  VFX_HIP(hipGetLastError());
  MARK(4, s);
  VFX_HIP(hipStreamWaitEvent(s, p->join_ev, 0));  // join
  MARK(8, s);
#define VFX_FAR(PMV, EX, NPLV, TSV)                                                                            \
  hipLaunchKernelGGL((k_far<PMV, EX, NPLV, TSV>), dim3(L, R), dim3(64), 0, s, T.K, P, T.root_size, D.leaf_box,      \
                     D.box_level, DT.t, D.l3_ptr, D.l3_src, D.l3_slot, D.m2p_y, D.locf, D.mpole, D.l1_ptr,         \
                     D.l1_srcbox, D.l1_slot, D.near_y, V, sLF, sMP, sNY, sM3, sFL)
#define VFX_FAR_N(PMV, EX)      \
  if (npl == 4 && H.ts)         \
    VFX_FAR(PMV, EX, 4, true);  \
  else if (npl == 4)            \
    VFX_FAR(PMV, EX, 4, false); \
  else if (npl == 3)            \
    VFX_FAR(PMV, EX, 3, false); \
  else                          \
    VFX_FAR(PMV, EX, 1, false);
  const int npl = (n + 63) / 64;  // 1, 3 or 4 for K = 4, 8, 12, 16
  if (P == 21) {
    VFX_FAR_N(21, true)
  } else if (P == 25) {
    VFX_FAR_N(25, true)
  } else if (P == 31) {
    VFX_FAR_N(31, true)
  } else if (P == 41) {
    VFX_FAR_N(41, true)
  } else {
    VFX_FAR_N(64, false)
  }
#undef VFX_FAR_N
#undef VFX_FAR
  VFX_HIP(hipGetLastError());
  MARK(9, s);
  if (timed) p->n_timed++;
  return VFX_OK;
}

}  // namespace vfx
