// Device side of the extension + volume FMM path (gfx950, FP64).
//
// Execution order on one stream (every output element has one writer, so no
// atomics are needed and results are bitwise reproducible):
//   fe_init      f^e = f on regular leaves, 0 elsewhere
//   extension    per cut leaf: f_G = P_i f_{X^I}; values on the Kbar grid of
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

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double box_side(double root, int level) { return ldexp(root, -level); }

// -------------------------------------------------------------------------
__global__ void k_fe_init(int n, int L, const int8_t* __restrict__ kind, const double* __restrict__ f_leaf,
                          double* __restrict__ fe) {
  const long total = (long)L * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int leaf = (int)(e / n);
    fe[e] = (kind[leaf] == 1) ? f_leaf[e] : 0.0;
  }
}

// -------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_extension(
    int K, int Kb, int nX, int nG, double root_size, const int* __restrict__ cut_leaf,
    const int* __restrict__ pinv_ptr, const uint16_t* __restrict__ pinv_idx, const double* __restrict__ pinv_val,
    const uint8_t* __restrict__ sbar_given, const int* __restrict__ ext_ptr, const int* __restrict__ ext_tgt,
    const double* __restrict__ t, const double* __restrict__ AbarT, const double* __restrict__ cbar,
    const int* __restrict__ leaf_box, const double* __restrict__ box_cx, const double* __restrict__ box_cy,
    const int* __restrict__ box_level, const double* __restrict__ f_cut, double* __restrict__ fe) {
  __shared__ double s_fI[kMaxX];
  __shared__ double s_fG[kMaxG];
  __shared__ double s_g[kMaxKb * kMaxKb];
  __shared__ double s_tmp[kMaxKb * kMaxKb];
  __shared__ double s_coef[kMaxKb * kMaxKb];
  __shared__ double s_Ex[kMaxK * kMaxKb];
  __shared__ double s_Ey[kMaxK * kMaxKb];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = K * K, Kb2 = Kb * Kb;
  const int off = pinv_ptr[c], ni = pinv_ptr[c + 1] - off;
  const double* fc = f_cut + (size_t)c * nX;
  for (int q = tid; q < ni; q += blockDim.x) s_fI[q] = fc[pinv_idx[off + q]];
  __syncthreads();
  // f_G = P_i f_I  (P_i: nG x ni row-major)
  const double* P = pinv_val + (size_t)off * nG;
  for (int r = wave; r < nG; r += blockDim.x / 64) {
    double acc = 0.0;
    const double* pr = P + (size_t)r * ni;
    for (int q = lane; q < ni; q += 64) acc += pr[q] * s_fI[q];
    acc = wave_sum(acc);
    if (lane == 0) s_fG[r] = acc;
  }
  __syncthreads();
  // values on the Kbar x Kbar grid of Sbar
  for (int a = tid; a < Kb2; a += blockDim.x) {
    double v;
    if (sbar_given[(size_t)c * Kb2 + a]) {
      v = fc[n + a];
    } else {
      v = 0.0;
      for (int r = 0; r < nG; ++r) v += AbarT[(size_t)r * Kb2 + a] * s_fG[r];
    }
    s_g[a] = v;
  }
  __syncthreads();
  // coefficients c = C g C^T, truncated to total order < Kbar
  for (int e = tid; e < Kb2; e += blockDim.x) {
    const int m = e / Kb, j = e % Kb;
    double acc = 0.0;
    for (int i = 0; i < Kb; ++i) acc += cbar[m * Kb + i] * s_g[i * Kb + j];
    s_tmp[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < Kb2; e += blockDim.x) {
    const int m = e / Kb, nn = e % Kb;
    double acc = 0.0;
    if (m + nn < Kb)
      for (int j = 0; j < Kb; ++j) acc += s_tmp[m * Kb + j] * cbar[nn * Kb + j];
    s_coef[e] = acc;
  }
  __syncthreads();
  const int bS = leaf_box[cut_leaf[c]];
  const double cxS = box_cx[bS], cyS = box_cy[bS];
  const double hS = box_side(root_size, box_level[bS]);
  for (int e = ext_ptr[c]; e < ext_ptr[c + 1]; ++e) {
    const int j = ext_tgt[e];
    const int bj = leaf_box[j];
    const double cxj = box_cx[bj], cyj = box_cy[bj];
    const double hj = box_side(root_size, box_level[bj]);
    if (tid < 2 * K) {
      const int a = tid % K;
      const bool isy = tid >= K;
      const double X = (isy ? cyj : cxj) + 0.5 * hj * t[a];
      const double xi = (X - (isy ? cyS : cxS)) / (1.5 * hS);
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

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Upward pass for the non-leaf boxes of one level, in the scaled-Pascal form
//   b_l = sum_q w_q^l [ sum_{1<=k<=l} C(l-1,k-1) (2 w_q)^-k a_{q,k} - a_{q,0}/l ],
//   b_0 = sum_q a_{q,0}   (w_q: child centre offset / parent side)
// One wave per box, lane l = output coefficient; the lane's Pascal row is
// held in registers.
template <int PM>
__global__ void __launch_bounds__(64) k_m2m(int P, int first, const int* __restrict__ box_child0,
                                            const double* __restrict__ pas, const double2* __restrict__ sin,
                                            const double2* __restrict__ sout, double2* __restrict__ mpole) {
  __shared__ double2 s_s[4][PM];
  const int b = first + blockIdx.x;
  const int c0 = box_child0[b];
  if (c0 < 0) return;
  const int l = threadIdx.x;
  double prow[PM];
#pragma unroll
  for (int k = 0; k < PM; ++k) prow[k] = (k < P && l < P) ? pas[(size_t)k * P + l] : 0.0;
  for (int q = 0; q < 4; ++q) {
    double2 v = make_double2(0.0, 0.0);
    if (l < P) {
      const double2 a = mpole[(size_t)(c0 + q) * P + l];
      v = (l == 0) ? a : cmul(sin[q * P + l], a);
    }
    if (l < PM) s_s[q][l] = v;
  }
  __syncthreads();
  if (l >= P) return;
  double re = 0.0, im = 0.0;
  for (int q = 0; q < 4; ++q) {
    if (l == 0) {
      re += s_s[q][0].x;
      im += s_s[q][0].y;
      continue;
    }
    double ur = 0.0, ui = 0.0;
#pragma unroll
    for (int k = 1; k < PM; ++k) {
      ur += prow[k] * s_s[q][k].x;
      ui += prow[k] * s_s[q][k].y;
    }
    ur -= s_s[q][0].x / l;
    ui -= s_s[q][0].y / l;
    const double2 w = sout[q * P + l];
    re += w.x * ur - w.y * ui;
    im += w.x * ui + w.y * ur;
  }
  mpole[(size_t)b * P + l] = make_double2(re, im);
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
                                                  double2* __restrict__ local) {
  __shared__ double2 s_o[8 * 64];
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
    for (int lc = 0; lc < 8; ++lc) s_o[lc * 64 + lane] = outc[lc];
    __syncthreads();
    const int lc = lane & 7, seg = lane >> 3;
    const int bb = b0 + seg, l = 8 * c + lc;
    if (bb < b1 && l < P) {
      double re = 0.0, im = 0.0;
      for (int q = l2_ptr[bb]; q < l2_ptr[bb + 1]; ++q) {
        const double2 v = s_o[lc * 64 + (q - e0)];
        re += v.x;
        im += v.y;
      }
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
                                                  double2* __restrict__ local) {
  __shared__ double2 s_o[8 * 64];
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
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    __syncthreads();
#pragma unroll
    for (int lc = 0; lc < 8; ++lc) {
      const int l = 8 * c + lc;
      double2 out = make_double2(0.0, 0.0);
      if (l < P) {
        double ur = 0.0, ui = 0.0;
#pragma unroll
        for (int k = 1; k < P; ++k) {
          const double cf = pasT[l * P + k];
          ur += cf * s[k].x;
          ui += cf * s[k].y;
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
      s_o[lc * 64 + lane] = act ? out : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lc = lane & 7, seg = lane >> 3;
    const int bb = b0 + seg, l = 8 * c + lc;
    if (bb < b1 && l < P) {
      double re = 0.0, im = 0.0;
      for (int q = l2_ptr[bb]; q < l2_ptr[bb + 1]; ++q) {
        const double2 v = s_o[lc * 64 + (q - e0)];
        re += v.x;
        im += v.y;
      }
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

// Downward pass into the boxes of one level:
//   c_l += (2w)^-l sum_{k>=l} C(k,l) w^k b_k(parent)
template <int PM>
__global__ void __launch_bounds__(64) k_l2l(int P, int first, const int* __restrict__ box_parent,
                                            const int* __restrict__ box_child0, const double* __restrict__ pas,
                                            const double2* __restrict__ sin, const double2* __restrict__ sout,
                                            double2* __restrict__ local) {
  __shared__ double2 s_s[PM];
  const int b = first + blockIdx.x;
  const int l = threadIdx.x;
  const int par = box_parent[b];
  const int q = b - box_child0[par];
  double prow[PM];
#pragma unroll
  for (int k = 0; k < PM; ++k) prow[k] = (k < P && l < P) ? pas[(size_t)k * P + l] : 0.0;
  double2 v = make_double2(0.0, 0.0);
  if (l < P) v = cmul(sin[q * P + l], local[(size_t)par * P + l]);
  if (l < PM) s_s[l] = v;
  __syncthreads();
  if (l >= P) return;
  double ur = 0.0, ui = 0.0;
#pragma unroll
  for (int k = 0; k < PM; ++k) {
    ur += prow[k] * s_s[k].x;
    ui += prow[k] * s_s[k].y;
  }
  const double2 g = cmul(sout[q * P + l], make_double2(ur, ui));
  double2 o = local[(size_t)b * P + l];
  o.x += g.x;
  o.y += g.y;
  local[(size_t)b * P + l] = o;
}

// -------------------------------------------------------------------------
// Batched table GEMMs on the FP64 matrix cores (near field, P2L, P2M).
// Entries (pairs) are grouped by table configuration c; a work-group takes a
// tile of <= TE entries (64 or 16) of one configuration and a block of <= 128
// table rows
// and computes, for every entry e, Y[e][row] = sum_k A_c[k][row] X[src(e)][k]
// (the table applied to the source leaf's K^2 values).
//   A: [c][k][row], R = 16*MT rows (rows fastest); X: [src][k]; Y: [e][row].
// The K dimension is processed in blocks of 16 with both operands staged in
// double-buffered LDS: the global loads of block kb+1 are in flight while the
// waves run their MFMAs on block kb.  With TE = 64, wave w owns entries
// 16w..16w+15 and every row tile of the block; with TE = 16 the waves share
// the 16 entries and split the row tiles.  MFMA operands: A = entry data (16 entries x 4
// k), B = table (4 k x 16 rows), so each output tile is (entries x rows) and
// the stores of a 16-lane group are 128 contiguous bytes.
// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16] and the
// outputs D[(l/16) + 4r][l%16], r = 0..3 (lane layout checked on gfx950).
// EPI = 1 (P2M): Y is the multipole array; rows < 2P of entry e (a leaf) are
// scaled by h^2 of that leaf and stored as its (p+1) complex coefficients.
template <int KD, int EPI, int TE>
__global__ void __launch_bounds__(256) k_gemm(int nitems, int MT, const int* __restrict__ t_cfg,
                                              const int* __restrict__ t_first,
                                              const int* __restrict__ t_count, const int* __restrict__ src,
                                              const double* __restrict__ A, const double* __restrict__ X,
                                              double* __restrict__ Y, int P2, double root_size,
                                              const int* __restrict__ leaf_box, const int* __restrict__ box_level) {
  constexpr int KB = 16;
  constexpr int LDA = TE;   // entries per LDS row (tile of TE = 64 or 16 entries)
  constexpr int LDB = 128;  // table rows per LDS row
  constexpr int NACC = (TE == 64) ? 8 : 2;  // row tiles per wave
  __shared__ double sA[2][KB * LDA];
  __shared__ double sB[2][KB * LDB];
  const int nrb = (MT + 7) / 8;  // row blocks of 8 tiles
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
  const int mtb = min(8, MT - 8 * rb);
  const int row0 = 128 * rb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const double* Ac = A + (size_t)c * KD * R;
  // global -> register staging of one K block
  constexpr int AE = TE * KB / 256;                  // entry values per thread (4 or 1)
  const int aj = tid % TE, ak = (tid / TE) * AE;     // entry aj, k = ak..ak+AE-1
  const int bk = tid >> 4, br = (tid & 15) * 8;      // table: k = bk, rows br..br+7
  const bool a_ok = aj < np;
  const double* xsrc = X + (size_t)(a_ok ? src[p0 + aj] : 0) * KD;
  double ra[AE], rb8[8];
  auto gload = [&](int kb) {
    const int k0 = kb * KB;
#pragma unroll
    for (int e = 0; e < AE; ++e) ra[e] = a_ok ? xsrc[k0 + ak + e] : 0.0;
    const bool b_ok = br < 16 * mtb;
    const double* ar = Ac + (size_t)(k0 + bk) * R + row0 + br;
#pragma unroll
    for (int e = 0; e < 8; ++e) rb8[e] = b_ok ? ar[e] : 0.0;
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AE; ++e) sA[buf][(ak + e) * LDA + aj] = ra[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) sB[buf][bk * LDB + br + e] = rb8[e];
  };
  // wave w: TE = 64 -> entries 16w..16w+15, row tiles 0..mtb-1;
  //         TE = 16 -> entries 0..15, row tiles w and w+4
  const int ebase = (TE == 64) ? 16 * w : 0;
  auto tile_of = [&](int r) { return (TE == 64) ? r : w + 4 * r; };
  vfx_d4 acc[NACC];
#pragma unroll
  for (int r = 0; r < NACC; ++r) acc[r] = vfx_d4{0, 0, 0, 0};
  constexpr int NKB = KD / KB;
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
#pragma unroll
      for (int r = 0; r < NACC; ++r) {
        const int rt = tile_of(r);
        if (rt < mtb)
          acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sB[buf][k * LDB + 16 * rt + li], acc[r], 0, 0, 0);
      }
    }
    if (kb + 1 < NKB) lstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < NACC; ++r) {
    const int rt = tile_of(r);
    if (rt >= mtb) continue;
    const int row = row0 + 16 * rt + li;
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

// With Y given, the near field is also finished here: the per-pair partials
// of the leaf's list-1 entries are summed in list order (deterministic) and
// the log(h) a_0 term added; V is then written, else it is accumulated.
__global__ void __launch_bounds__(256) k_far(int K, int P, double root_size, const int* __restrict__ leaf_box,
                                             const int* __restrict__ box_level, const double* __restrict__ box_cx,
                                             const double* __restrict__ box_cy, const double* __restrict__ t,
                                             const int* __restrict__ l3_ptr, const int* __restrict__ l3_src,
                                             const double2* __restrict__ l2p, const double2* __restrict__ local,
                                             const double2* __restrict__ mpole, const int* __restrict__ l1_ptr,
                                             const int* __restrict__ l1_src, const int* __restrict__ l1_slot,
                                             const double* __restrict__ Y, double* __restrict__ V) {
  __shared__ double2 s_a[64];
  const int n = K * K;
  const int leaf = blockIdx.x;
  const int i = threadIdx.x;
  const int b = leaf_box[leaf];
  const int lev = box_level[b];
  const double h = box_side(root_size, lev);
  double acc = 0.0;
  if (Y != nullptr && i < n) {
    double yn = 0.0, lg = 0.0;
    for (int e = l1_ptr[leaf]; e < l1_ptr[leaf + 1]; ++e) {
      yn += Y[(size_t)l1_slot[e] * n + i];
      lg += mpole[(size_t)leaf_box[l1_src[e]] * P].x;
    }
    acc = h * h * yn + log(h) * lg;
  }
  if (lev >= 2) {
    if (i < P) s_a[i] = local[(size_t)b * P + i];
    __syncthreads();
    if (i < n)
      for (int l = 0; l < P; ++l) {
        const double2 z = l2p[(size_t)l * n + i];
        acc += z.x * s_a[l].x - z.y * s_a[l].y;
      }
  }
  const double xi = box_cx[b] + 0.5 * h * t[(i < n ? i : 0) / K];
  const double yi = box_cy[b] + 0.5 * h * t[(i < n ? i : 0) % K];
  for (int e = l3_ptr[leaf]; e < l3_ptr[leaf + 1]; ++e) {
    const int w = l3_src[e];
    __syncthreads();
    if (i < P) s_a[i] = mpole[(size_t)w * P + i];
    __syncthreads();
    if (i < n) {
      const double hw = box_side(root_size, box_level[w]);
      const double zx = xi - box_cx[w], zy = yi - box_cy[w];
      const double r2 = zx * zx + zy * zy;
      // zeta = hw / z
      const double zr = hw * zx / r2, zi = -hw * zy / r2;
      double sr = 0.0, si = 0.0;  // Horner: sum_{k>=1} a_k zeta^k
      for (int k = P - 1; k >= 1; --k) {
        const double ar = sr + s_a[k].x, ai = si + s_a[k].y;
        sr = ar * zr - ai * zi;
        si = ar * zi + ai * zr;
      }
      acc += s_a[0].x * 0.5 * log(r2) + sr;
    }
  }
  if (i < n) {
    if (Y != nullptr)
      V[(size_t)leaf * n + i] = kInv2Pi * acc;
    else
      V[(size_t)leaf * n + i] += kInv2Pi * acc;
  }
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
  UP(D.cbar, T.cbar);
  UP(D.near, T.near);
  UP(D.p2l_gemm, T.p2l_gemm);
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
  void* ptrs[] = {D.t,        D.tbar,     D.w2,       D.AbarT,   D.cbar,     D.near,    D.near_s2,
                  D.p2m,      D.l2p,      D.m2m,      D.l2l,     D.m2l,      D.p2l,     D.p2l_area,
                  D.pas_m2l,  D.pas_m2m,  D.pas_l2l,  D.m2l_logd, D.p2l_gemm, D.m2l_tpow, D.m2l_tneg, D.p2m_gemm,
                  D.m2m_in,   D.m2m_out,  D.l2l_in,   D.l2l_out,  D.pas_m2l_t, D.pas_m2m_t, D.pas_l2l_t};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  D = DeviceTables();
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
  UP(D.l1_ptr, H.l1_ptr);
  UP(D.l1_src, H.l1_src);
  UP(D.l1_cfg, H.l1_cfg);
  UP(D.l2_ptr, H.l2_ptr);
  UP(D.l2_src, H.l2_src);
  UP(D.l2_off, H.l2_off);
  UP(D.l2_tgt, H.l2_tgt);
  UP(D.m2l_grp, H.m2l_grp);
  UP(D.l3_ptr, H.l3_ptr);
  UP(D.l3_src, H.l3_src);
  UP(D.l4_ptr, H.l4_ptr);
  UP(D.l4_src, H.l4_src);
  UP(D.l4_cfg, H.l4_cfg);
  UP(D.np_src, H.np_src);
  UP(D.l1_slot, H.l1_slot);
  UP(D.nt_cfg, H.nt_cfg);
  UP(D.nt_first, H.nt_first);
  UP(D.nt_count, H.nt_count);
  UP(D.p4_src, H.p4_src);
  UP(D.l4_slot, H.l4_slot);
  UP(D.t4_cfg, H.t4_cfg);
  UP(D.t4_first, H.t4_first);
  UP(D.t4_count, H.t4_count);
  UP(D.t0_cfg, H.t0_cfg);
  UP(D.t0_first, H.t0_first);
  UP(D.t0_count, H.t0_count);
  UP(D.leaf_ids, H.leaf_ids);
  if (!H.np_src.empty()) VFX_HIP(hipMalloc((void**)&D.near_y, sizeof(double) * H.np_src.size() * T.n));
  if (!H.p4_src.empty()) VFX_HIP(hipMalloc((void**)&D.p2l_y, sizeof(double) * H.p4_src.size() * T.p2l_rows));
  UP(D.cut_leaf, H.cut_leaf);
  UP(D.ext_ptr, H.ext_ptr);
  UP(D.ext_tgt, H.ext_tgt);
  UP(D.pinv_ptr, H.pinv_ptr);
  UP(D.pinv_idx, H.pinv_idx);
  UP(D.pinv_val, H.pinv_val);
  UP(D.sbar_given, H.sbar_given);
  VFX_HIP(hipMalloc((void**)&D.mpole, sizeof(double2) * (size_t)H.B * P));
  VFX_HIP(hipMalloc((void**)&D.local, sizeof(double2) * (size_t)H.B * P));
  VFX_HIP(hipMemset(D.local, 0, sizeof(double2) * (size_t)H.B * P));
  VFX_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
  VFX_HIP(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
  VFX_HIP(hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming));
  D.ready = true;
  return VFX_OK;
}

void free_plan_device(Plan* p) {
  DevicePlan& D = p->D;
  void* ptrs[] = {D.box_level, D.box_child0, D.box_leaf, D.box_parent, D.box_cx,   D.box_cy,   D.leaf_box,
                  D.kind,      D.l1_ptr,     D.l1_src,   D.l1_cfg,     D.l2_ptr,   D.l2_src,   D.l2_off,
                  D.l3_ptr,    D.l3_src,     D.l4_ptr,   D.l4_src,     D.l4_cfg,   D.np_src,   D.l1_slot,
                  D.nt_cfg,    D.nt_first,   D.nt_count, D.near_y,     D.p4_src,   D.l4_slot,  D.t4_cfg,
                  D.t4_first,  D.t4_count,   D.p2l_y,    D.cut_leaf,   D.ext_ptr,  D.ext_tgt,  D.pinv_ptr,
                  D.pinv_idx,  D.pinv_val,   D.sbar_given, D.mpole,    D.local,    D.t0_cfg,   D.t0_first,
                  D.t0_count,  D.leaf_ids,   D.l2_tgt,   D.m2l_grp};
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
  if (p->side) (void)hipStreamDestroy(p->side);
  p->fork_ev = p->join_ev = nullptr;
  p->side = nullptr;
}

template <int KD, int EPI, int TE>
static void launch_gemm(int items, int MT, const int* cfg, const int* first, const int* count, const int* src,
                        const double* A, const double* X, double* Y, int P2, double root, const int* leaf_box,
                        const int* box_level, hipStream_t s, int max_wgs) {
  const int grid = (max_wgs > 0 && items > max_wgs) ? max_wgs : items;
  hipLaunchKernelGGL((k_gemm<KD, EPI, TE>), dim3(grid), dim3(256), 0, s, items, MT, cfg, first, count, src, A, X, Y,
                     P2, root, leaf_box, box_level);
}

// ntiles tiles of <= TE entries; each is split into ceil(MT/8) row blocks;
// max_wgs > 0 bounds the grid (the work-groups then loop over the items)
template <int EPI, int TE>
static void gemm(int n, int ntiles, int MT, const int* cfg, const int* first, const int* count, const int* src,
                 const double* A, const double* X, double* Y, hipStream_t s, int max_wgs = 0, int P2 = 0,
                 double root = 0, const int* leaf_box = nullptr, const int* box_level = nullptr) {
  if (ntiles <= 0) return;
  const int items = ntiles * ((MT + 7) / 8);
#define VFX_GEMM_CASE(KDV)                                                                                   \
  launch_gemm<KDV, EPI, TE>(items, MT, cfg, first, count, src, A, X, Y, P2, root, leaf_box, box_level, s, \
                            max_wgs)
  switch (n) {
    case 16: VFX_GEMM_CASE(16); break;
    case 64: VFX_GEMM_CASE(64); break;
    case 144: VFX_GEMM_CASE(144); break;
    default: VFX_GEMM_CASE(256); break;
  }
#undef VFX_GEMM_CASE
}

constexpr int kNearWgs = 512;

int launch_execute(Plan* p, const double* f_leaf, const double* f_cut, double* fe, double* V, hipStream_t s,
                   std::string& err) {
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
  const HostPlan& H = p->H;
  const DeviceTables& DT = c->D;
  const DevicePlan& D = p->D;
  const int n = T.n, P = T.p + 1, L = H.L;
  const bool big = P > 32;
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
  // events on the caller's stream: 0 start, 1 after the extension, 2 after
  // P2M+M2M, 3 after M2L+P2L, 4 after L2L, 7 after the join, 8 end; on the
  // side stream: 5 and 6 around the near-field GEMM
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
  {
    const long total = (long)L * n;
    int blocks = (int)std::min<long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fe_init, dim3(blocks), dim3(256), 0, s, n, L, D.kind, f_leaf, fe);
  }
  if (H.ncut > 0)
    hipLaunchKernelGGL(k_extension, dim3(H.ncut), dim3(256), 0, s, T.K, T.Kbar, T.nX, T.nG, T.root_size,
                       D.cut_leaf, D.pinv_ptr, D.pinv_idx, D.pinv_val, D.sbar_given, D.ext_ptr, D.ext_tgt,
                       DT.t, DT.AbarT, DT.cbar, D.leaf_box, D.box_cx, D.box_cy, D.box_level, f_cut, fe);
  VFX_HIP(hipGetLastError());
  MARK(1, s);
  // multipoles of the leaves (start of the critical chain)
  gemm<1, 16>(n, (int)H.t0_first.size(), T.p2l_rows / 16, D.t0_cfg, D.t0_first, D.t0_count, D.leaf_ids, DT.p2m_gemm,
              fe, (double*)D.mpole, s, 0, 2 * P, T.root_size, D.leaf_box, D.box_level);
  // fork: near field on the side stream, concurrent with the upward pass,
  // M2L/P2L and the downward pass on the caller's stream.  Its grid is
  // bounded (about two work-groups per CU, looping over the tiles) so the
  // latency-bound tree kernels keep CU slots.
  VFX_HIP(hipEventRecord(p->fork_ev, s));
  VFX_HIP(hipStreamWaitEvent(p->side, p->fork_ev, 0));
  MARK(5, p->side);
  gemm<0, 64>(n, (int)H.nt_cfg.size(), n / 16, D.nt_cfg, D.nt_first, D.nt_count, D.np_src, DT.near, fe, D.near_y,
              p->side, kNearWgs);
  VFX_HIP(hipGetLastError());
  MARK(6, p->side);
  VFX_HIP(hipEventRecord(p->join_ev, p->side));
  for (int l = H.nlev - 2; l >= 2; --l) {
    const int first = H.level_start[l], cnt = H.level_start[l + 1] - first;
    if (cnt <= 0) continue;
    if (big)
      hipLaunchKernelGGL(k_m2m<64>, dim3(cnt), dim3(64), 0, s, P, first, D.box_child0, DT.pas_m2m, DT.m2m_in,
                         DT.m2m_out, D.mpole);
    else
      hipLaunchKernelGGL(k_m2m<32>, dim3(cnt), dim3(64), 0, s, P, first, D.box_child0, DT.pas_m2m, DT.m2m_in,
                         DT.m2m_out, D.mpole);
  }
  VFX_HIP(hipGetLastError());
  MARK(2, s);
  if (H.nlev > 2) {
    gemm<0, 64>(n, (int)H.t4_cfg.size(), T.p2l_rows / 16, D.t4_cfg, D.t4_first, D.t4_count, D.p4_src, DT.p2l_gemm,
            fe, D.p2l_y, s);
    const int ng = (int)H.m2l_grp.size() - 1;
    if (ng > 0) {
#define VFX_M2L(PMV)                                                                                             \
  hipLaunchKernelGGL(k_m2l_pairs<PMV>, dim3(ng), dim3(64), 0, s, P, T.root_size, D.m2l_grp, D.box_level, D.l2_ptr, \
                     D.l2_src, D.l2_off, D.l2_tgt, D.l4_ptr, D.l4_src, D.l4_slot, D.leaf_box, T.p2l_rows,         \
                     DT.pas_m2l_t, DT.m2l_logd, D.mpole, D.p2l_y, D.local)
#define VFX_M2LL(PV)                                                                                             \
  hipLaunchKernelGGL(k_m2l_lanes<PV>, dim3(ng), dim3(64), 0, s, T.root_size, D.m2l_grp, D.box_level, D.l2_ptr,     \
                     D.l2_src, D.l2_off, D.l2_tgt, D.l4_ptr, D.l4_src, D.l4_slot, D.leaf_box, T.p2l_rows,         \
                     DT.pas_m2l_t, DT.m2l_logd, D.mpole, D.p2l_y, D.local)
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
  for (int l = 3; l < H.nlev; ++l) {
    const int first = H.level_start[l], cnt = H.level_start[l + 1] - first;
    if (cnt <= 0) continue;
    if (big)
      hipLaunchKernelGGL(k_l2l<64>, dim3(cnt), dim3(64), 0, s, P, first, D.box_parent, D.box_child0, DT.pas_l2l,
                         DT.l2l_in, DT.l2l_out, D.local);
    else
      hipLaunchKernelGGL(k_l2l<32>, dim3(cnt), dim3(64), 0, s, P, first, D.box_parent, D.box_child0, DT.pas_l2l,
                         DT.l2l_in, DT.l2l_out, D.local);
  }
  VFX_HIP(hipGetLastError());
  MARK(4, s);
  VFX_HIP(hipStreamWaitEvent(s, p->join_ev, 0));  // join
  MARK(7, s);
  hipLaunchKernelGGL(k_far, dim3(L), dim3(n < 64 ? 64 : n), 0, s, T.K, P, T.root_size, D.leaf_box, D.box_level,
                     D.box_cx, D.box_cy, DT.t, D.l3_ptr, D.l3_src, DT.l2p, D.local, D.mpole, D.l1_ptr, D.l1_src,
                     D.l1_slot, D.near_y, V);
  VFX_HIP(hipGetLastError());
  MARK(8, s);
  if (timed) p->n_timed++;
  return VFX_OK;
}

}  // namespace vfx
