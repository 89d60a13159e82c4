// Mixed-precision near field (K = 16): the list-1 table products on the bf16
// matrix cores with results that stay accurate to about 2^-32 of the
// operands' row maxima (the tables of Section 4, in the low-rank form Q W
// for the 32 neighbour configurations and dense for the self operator).
//
// Every operand row v (along the contraction) is cut into four fixed-point
// slices: with e the exponent of max |v| (max |v| < 2^e),
//     v = 2^e sum_{s<4} q_s 2^(-8(s+1))  (+ a residual below 2^(e-33)),
// q_0 an integer of magnitude <= 256, q_1..q_3 of magnitude <= 128, all
// exact in bf16.  A product of two rows is then
//     2^(e_a + e_b - 16) sum_{d<4} 2^(-8d) sum_{i+j=d} <q_i(a), q_j(b)>
// (the pairs with i + j >= 4 are below the residual and are dropped).  Per
// 32 contraction indices (one v_mfma_f32_16x16x32_bf16) the slice pairs of
// one d add up to at most 3 * 2^20 in magnitude, so over four such blocks
// every partial sum is an integer below 2^24 and the FP32 accumulation is
// exact; every four blocks the d-sums are widened to FP64, scaled by
// 2^(-8d) (exact) and added to FP64 accumulators (exact as well: 49 bits).
// The results are FP64, stored as the FP64 path's per-pair products.
//
// v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)+j], B[8(l/16)+j][l%16]
// (j = 0..7) and the outputs D[4(l/16)+r][l%16], r = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "vfx_internal.h"

namespace vfx {

namespace {

typedef short fx_s8 __attribute__((ext_vector_type(8)));
typedef float fx_f4 __attribute__((ext_vector_type(4)));
typedef double fx_d4 __attribute__((ext_vector_type(4)));

constexpr int kFxN = 256;               // K^2
constexpr int kFxBuf = 4 * 64 * 32;    // one staging buffer: 4 slices x 64 rows x 32 contraction values
constexpr int kFxLDZ = kNearLrMax + 4;  // LDS row stride of the FP64 factor products Z

__device__ __forceinline__ uint16_t fx_bf16_of_int(double q) {
  return (uint16_t)(__float_as_uint((float)q) >> 16);  // |q| <= 256: exact
}

// leaf data -> four fixed-point slices per node and one exponent per leaf
// (one work-group of 256 threads per leaf and right-hand side)
__global__ void __launch_bounds__(256) k_split4(int L, const double* __restrict__ x, uint16_t* __restrict__ xs,
                                                int* __restrict__ xe) {
  __shared__ double red[256];
  const long total = (long)L * kFxN;
  x += blockIdx.y * total;  // right-hand side blockIdx.y
  xs += blockIdx.y * 4 * total;
  xe += blockIdx.y * L;
  const int leaf = blockIdx.x, t = threadIdx.x;
  const double v = x[(size_t)leaf * kFxN + t];
  red[t] = fabs(v);
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  int e = 0;
  if (red[0] > 0.0) frexp(red[0], &e);
  double r = ldexp(v, -e);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    r *= 256.0;
    const double q = rint(r);
    xs[(size_t)s * total + (size_t)leaf * kFxN + t] = fx_bf16_of_int(q);
    r -= q;
  }
  if (t == 0) xe[leaf] = e;
}

__device__ __forceinline__ fx_f4 fx_mfma(fx_s8 a, fx_s8 b, fx_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// t[d] += the slice products of one 32-index block with i + j = d
__device__ __forceinline__ void fx_block(const fx_s8 a[4], const fx_s8 b[4], fx_f4 t[4]) {
  t[0] = fx_mfma(a[0], b[0], t[0]);
  t[1] = fx_mfma(a[0], b[1], t[1]);
  t[1] = fx_mfma(a[1], b[0], t[1]);
  t[2] = fx_mfma(a[0], b[2], t[2]);
  t[2] = fx_mfma(a[1], b[1], t[2]);
  t[2] = fx_mfma(a[2], b[0], t[2]);
  t[3] = fx_mfma(a[0], b[3], t[3]);
  t[3] = fx_mfma(a[1], b[2], t[3]);
  t[3] = fx_mfma(a[2], b[1], t[3]);
  t[3] = fx_mfma(a[3], b[0], t[3]);
}
__device__ __forceinline__ void fx_zero(fx_f4 t[4]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) t[d] = fx_f4{0.0f, 0.0f, 0.0f, 0.0f};
}
// the integer-scaled sum of the d-sums of output r
__device__ __forceinline__ double fx_value(const fx_f4 t[4], int r) {
  return (double)t[0][r] + 0x1p-8 * (double)t[1][r] + 0x1p-16 * (double)t[2][r] + 0x1p-24 * (double)t[3][r];
}

// B staging: 64 rows x 32 contraction values x 4 slices, 1024 pieces of 16
// bytes, four per thread; consecutive threads take consecutive pieces of a
// row.  In LDS a row is 64 bytes and its piece p sits at slot p ^ fx_sw(row):
// the 16 lanes of a fragment read (rows 16 r + li, piece lk) and the 16
// lanes of a store (four rows, four pieces each) then fall in distinct banks,
// as do the eight-lane halves of either.
struct FxStage {
  fx_s8 v[4];
};
__device__ __forceinline__ int fx_sw(int row) { return ((row >> 1) ^ (row >> 3)) & 3; }

__device__ __forceinline__ void fx_gload(FxStage& st, const uint16_t* __restrict__ base, size_t slice, int ld,
                                         int row0, int c0, int nrows) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = t >> 2, part = t & 3;  // slice j
    st.v[j] = row < nrows ? *(const fx_s8*)(base + (size_t)j * slice + (size_t)(row0 + row) * ld + c0 + 8 * part)
                          : fx_s8{0, 0, 0, 0, 0, 0, 0, 0};
  }
}
__device__ __forceinline__ void fx_lstore(const FxStage& st, uint16_t* sb) {
  const int t = threadIdx.x, row = t >> 2, part = t & 3;
#pragma unroll
  for (int j = 0; j < 4; ++j) *(fx_s8*)(sb + j * 2048 + row * 32 + 8 * (part ^ fx_sw(row))) = st.v[j];
}
// B fragments (four slices) of row tile r from a staged block
__device__ __forceinline__ void fx_bfrag(const uint16_t* sb, int r, fx_s8 b[4]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4, row = 16 * r + li;
#pragma unroll
  for (int s = 0; s < 4; ++s) b[s] = *(const fx_s8*)(sb + s * 2048 + row * 32 + 8 * (lk ^ fx_sw(row)));
}

// Phase 1: acc[r] (r < MT1) = the integer-scaled products of this lane's pair
// row of the leaf slices with B rows row0 + 16 r .. (B: [s][row][256], slice
// stride wslice) over the 256 nodes in 8 blocks of 32.  The A fragments of
// block kb + 4 are loaded once block kb is multiplied (a ring of four register
// blocks: they come from the leaf data in HBM); the B rows of block kb + 2
// are loaded into registers (from the L2-resident tables) once block kb + 1
// is stored to the other LDS buffer.
template <int MT1>
__device__ __forceinline__ void fx_phase1(const uint16_t* __restrict__ xrow, long xs_slice,
                                          const uint16_t* __restrict__ wbase, size_t wslice, int row0,
                                          uint16_t* sbuf, fx_d4 acc[4]) {
  constexpr int NKB = kFxN / 32;
  fx_f4 t[MT1][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = fx_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < MT1; ++r) fx_zero(t[r]);
  fx_s8 a[4][4];
  FxStage st;
  auto ga = [&](fx_s8* av, int kb) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < 4; ++s) av[s] = *(const fx_s8*)(xrow + (size_t)s * xs_slice + 32 * kb);
  };
#pragma unroll
  for (int k = 0; k < 4; ++k) ga(a[k], k);
  fx_gload(st, wbase, wslice, kFxN, row0, 0, 16 * MT1);
  __syncthreads();  // the previous user of sbuf is done
  fx_lstore(st, sbuf);
  fx_gload(st, wbase, wslice, kFxN, row0, 32, 16 * MT1);
  __syncthreads();
#pragma unroll 1
  for (int k0 = 0; k0 < NKB; k0 += 4) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kb = k0 + s4;
      const uint16_t* sb = sbuf + (s4 & 1) * kFxBuf;
#pragma unroll
      for (int r = 0; r < MT1; ++r) {
        fx_s8 b[4];
        fx_bfrag(sb, r, b);
        fx_block(a[s4], b, t[r]);
      }
      if (kb + 4 < NKB) ga(a[s4], kb + 4);
      if (kb + 1 < NKB) fx_lstore(st, sbuf + ((s4 + 1) & 1) * kFxBuf);
      if (kb + 2 < NKB) fx_gload(st, wbase, wslice, kFxN, row0, 32 * (kb + 2), 16 * MT1);
      if (s4 == 3) {  // four blocks done: widen
#pragma unroll
        for (int r = 0; r < MT1; ++r) {
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[r][e] += fx_value(t[r], e);
          fx_zero(t[r]);
        }
      }
      __syncthreads();
    }
  }
}

// One work item: a tile of <= 64 pairs of one configuration (wave w owns
// pairs 16w..16w+15).  LR: Z = X W^T (R_c ranks) in FP64, kept in LDS, cut
// into slices per pair, then Y = Z Q^T; dense (self operator): Y = X A^T for
// one block of 64 target rows (four row blocks per tile).  Results (FP64,
// exponents applied) go to the per-pair products Y.  Persistent, XCD-aware
// item order (items are configuration-major; an XCD's L2 holds the slices
// of the few configurations it works on).
template <bool LR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_near_fx(int nitems, int nrb, const int* __restrict__ t_cfg,
                                                 const int* __restrict__ t_first, const int* __restrict__ t_count,
                                                 const int* __restrict__ src, const int* __restrict__ lr_R,
                                                 const uint16_t* __restrict__ Wb, const int* __restrict__ Wexp,
                                                 const uint16_t* __restrict__ Qb, const int* __restrict__ Qexp,
                                                 const uint16_t* __restrict__ xs, const int* __restrict__ xe,
                                                 long xs_slice, int L, double* __restrict__ Y, long sy) {
  xs += blockIdx.y * 4 * xs_slice;  // right-hand side blockIdx.y
  xe += blockIdx.y * L;
  Y += blockIdx.y * sy;
  constexpr int n = kFxN, LM = kNearLrMax;
  __shared__ __attribute__((aligned(16))) uint16_t sbuf[2 * kFxBuf];
  __shared__ double sZ[LR ? 64 * kFxLDZ : 1];
  __shared__ int s_ez[64];
  const int nb = gridDim.x, bb = blockIdx.x;
  const int x = bb & 7;
  const int q = nitems >> 3, rr = nitems & 7;
  const int xfirst = x * q + min(x, rr), xcount = q + (x < rr ? 1 : 0);
  const int xwgs = (nb - x + 7) >> 3;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int j = bb >> 3; j < xcount; j += xwgs) {
    const int item = xfirst + j;
    const int tile = item / nrb, rb = item - tile * nrb;
    const int c = t_cfg[tile], p0 = t_first[tile], np = t_count[tile];
    const int ent = 16 * w + li;  // this lane's A-operand pair
    const int leaf = src[p0 + (ent < np ? ent : 0)];
    const uint16_t* xrow = xs + (size_t)leaf * n + 8 * lk;
    const int my_ex = xe[leaf];
    // exponents of the output rows this lane holds: pairs 16w + 4lk + e
    int ex_out[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) ex_out[e] = __shfl(my_ex, 4 * lk + e, 16);
    const int MT1 = LR ? lr_R[c] / 16 : 4;
    const size_t wslice = LR ? (size_t)LM * n : (size_t)n * n;
    const uint16_t* wbase = LR ? Wb + (size_t)c * 4 * wslice : Wb;
    const int* wexp = LR ? Wexp + (size_t)c * LM : Wexp;
    const int row0 = LR ? 0 : 64 * rb;
    fx_d4 acc[4];
    switch (MT1) {
      case 1: fx_phase1<1>(xrow, xs_slice, wbase, wslice, row0, sbuf, acc); break;
      case 2: fx_phase1<2>(xrow, xs_slice, wbase, wslice, row0, sbuf, acc); break;
      case 3: fx_phase1<3>(xrow, xs_slice, wbase, wslice, row0, sbuf, acc); break;
      default: fx_phase1<4>(xrow, xs_slice, wbase, wslice, row0, sbuf, acc); break;
    }
    if (!LR) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 64 * rb + 16 * r + li;
        const int ei = wexp[i];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int pe = 16 * w + 4 * lk + e;
          if (pe < np) Y[(size_t)(p0 + pe) * n + i] = ldexp(acc[r][e], ex_out[e] + ei - 16);
        }
      }
      continue;
    }
    // Z (FP64) of this wave's pairs to LDS (ranks >= R zero) and the
    // exponent of every pair's row of Z: the maximum over the row is taken
    // over r and over the 16 lanes li that hold it
    int ez_out[4];
    {
      double m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * r + li;
        const int ea = r < MT1 ? wexp[a] : 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double z = r < MT1 ? ldexp(acc[r][e], ex_out[e] + ea - 16) : 0.0;
          sZ[(16 * w + 4 * lk + e) * kFxLDZ + a] = z;
          m[e] = fmax(m[e], fabs(z));
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) m[e] = fmax(m[e], __shfl_xor(m[e], o, 16));
        int ee = 0;
        if (m[e] > 0.0) frexp(m[e], &ee);
        ez_out[e] = ee;
        if (li == 0) s_ez[16 * w + 4 * lk + e] = ee;
      }
    }
    // phase 2: Y = Z Q^T over the target rows in four chunks of 64; stage g
    // holds Q rows 64 (g / nkb) .. + 63, ranks 32 (g % nkb) .. + 31 (4 slices),
    // loaded two stages ahead into registers and stored one stage ahead into
    // the other LDS buffer
    const uint16_t* qbase = Qb + (size_t)c * 4 * LM * n;
    const int* qexp = Qexp + (size_t)c * n;
    const int nkb = (16 * MT1 + 31) / 32, nst = 4 * nkb;
    auto qload = [&](FxStage& stg, int g) __attribute__((always_inline)) {
      const int ch = g / nkb;
      fx_gload(stg, qbase, (size_t)LM * n, LM, 64 * ch, 32 * (g - ch * nkb), 64);
    };
    FxStage st[2];
    qload(st[0], 0);
    qload(st[1], 1);
    fx_lstore(st[0], sbuf);  // the last phase-1 barrier freed sbuf
    qload(st[0], 2);
    __syncthreads();         // Z, its exponents and stage 0 are in LDS
    // A fragments of Z for both 32-rank blocks: this lane's pair 16w + li,
    // ranks 32 kb + 8 lk + t, four slices
    const int myez = s_ez[16 * w + li];
    fx_s8 za[2][4];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const double* zr = sZ + (16 * w + li) * kFxLDZ + 32 * kb + 8 * lk;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        double r = ldexp(zr[t], -myez);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          r *= 256.0;
          const double qv = rint(r);
          za[kb][s][t] = (short)fx_bf16_of_int(qv);
          r -= qv;
        }
      }
    }
    fx_f4 t2[4][4];  // a chunk's contraction (<= 64 ranks) is at most two blocks: exact in FP32
#pragma unroll 1
    for (int g0 = 0; g0 < nst; g0 += 2) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int g = g0 + h;
        const int ch = g / nkb, kb = g - ch * nkb;
        if (kb == 0)
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) fx_zero(t2[r4]);
        const uint16_t* sb = sbuf + h * kFxBuf;
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          fx_s8 b[4];
          fx_bfrag(sb, r4, b);
          if (h == 1 && nkb == 2)
            fx_block(za[1], b, t2[r4]);
          else
            fx_block(za[0], b, t2[r4]);
        }
        if (g + 1 < nst) fx_lstore(st[(h + 1) & 1], sbuf + ((h + 1) & 1) * kFxBuf);
        if (g + 3 < nst) qload(st[(h + 1) & 1], g + 3);
        if (kb == nkb - 1) {
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const int i = 64 * ch + 16 * r4 + li;
            const int ei = qexp[i];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int pe = 16 * w + 4 * lk + e;
              if (pe < np) Y[(size_t)(p0 + pe) * n + i] = ldexp(fx_value(t2[r4], e), ez_out[e] + ei - 16);
            }
          }
        }
        __syncthreads();
      }
    }
  }
}

int persistent_grid_fx(int items, int max_wgs) {
  int grid = (max_wgs > 0 && items > max_wgs) ? max_wgs : items;
  return std::max(grid, std::min(items, 8));
}

}  // namespace

int launch_near_fx(const Plan* p, const double* fe, int nrhs, int max_wgs, hipStream_t s, std::string& err) {
  const HostPlan& H = p->H;
  const DevicePlan& D = p->D;
  const DeviceTables& DT = p->ctx->D;
  const long total = (long)H.L * kFxN, sNY = (long)H.np_src.size() * kFxN;
  hipLaunchKernelGGL(k_split4, dim3(H.L, nrhs), dim3(256), 0, s, H.L, fe, D.xs, D.xs_exp);
  if (!H.ml_cfg.empty()) {
    const int items = (int)H.ml_cfg.size();
    hipLaunchKernelGGL(k_near_fx<true>, dim3(persistent_grid_fx(items, max_wgs), nrhs), dim3(256), 0, s, items, 1,
                       D.ml_cfg, D.ml_first, D.ml_count, D.np_src, DT.lr_R, DT.fx_W, DT.fx_Wexp, DT.fx_Q,
                       DT.fx_Qexp, D.xs, D.xs_exp, total, H.L, D.near_y, sNY);
  }
  if (!H.mt_cfg.empty()) {
    const int items = 4 * (int)H.mt_cfg.size();
    hipLaunchKernelGGL(k_near_fx<false>, dim3(persistent_grid_fx(items, max_wgs), nrhs), dim3(256), 0, s, items, 4,
                       D.mt_cfg, D.mt_first, D.mt_count, D.np_src, DT.lr_R, DT.fx_A, DT.fx_Aexp, DT.fx_Q,
                       DT.fx_Qexp, D.xs, D.xs_exp, total, H.L, D.near_y, sNY);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("mixed near field: ") + hipGetErrorString(e);
    return VFX_EHIP;
  }
  return VFX_OK;
}

}  // namespace vfx
