// Mixed-precision near field on the int8 matrix cores (K = 16): the list-1
// table products of Section 4 (low-rank Q W for the 32 neighbour
// configurations, dense for the self operator) with results accurate to
// about 2^-34 of the operands' row maxima.
//
// Every operand row v (along the contraction) is cut into S = kF8Slices = 5
// fixed-point slices: with e the exponent of max |v| (max |v| < 2^e),
//     v = 2^e sum_{s<S} q_s 2^(-6-7s)  (+ a residual below 2^(e-7S)),
// q_s integers of magnitude <= 64.  A product of two rows is
//     2^(e_a + e_b - 12) sum_{d<S} 2^(-7d) sum_{i+j=d} <q_i(a), q_j(b)>
// (the pairs with i + j >= S are below the residual and are dropped: 15 of
// the 25 products are kept).  A slice product is at most 2^12 in magnitude,
// so over the whole contraction (256 terms) the at most five pairs of one d
// add up to less than 2^23: the int32 accumulation is exact with no
// intermediate widening, and the final sum over d in FP64 is exact too (51
// significant bits).  The results are FP64, stored as the FP64 path's
// per-pair products.  (Six slices keep 2^-41 and measured slower than the
// FP64 path on the wedge workload; the kernel is written for any S.)
//
// v_mfma_i32_16x16x64_i8: lane l holds A[l%16][16(l/16)+j], B[16(l/16)+j][l%16]
// (j = 0..15, one byte each) and the outputs D[4(l/16)+r][l%16], r = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "vfx_internal.h"

namespace vfx {

namespace {

typedef int f8_v4 __attribute__((ext_vector_type(4)));

constexpr int kF8N = 256;          // K^2
constexpr int kF8Slice = 64 * 64;  // one staged slice: 64 rows x 64 contraction bytes

// leaf data -> kF8Slices int8 slices per node and one exponent per leaf: one
// wavefront per leaf (four per work-group), lane l holds nodes 4l .. 4l+3
// (two 16-byte loads), the row maximum is a wavefront reduction, and each
// slice leaves as one 4-byte store per lane
__global__ void __launch_bounds__(256) k_split_i8(int L, const double* __restrict__ x, int8_t* __restrict__ xs,
                                                  int* __restrict__ xe) {
  const long total = (long)L * kF8N;
  x += blockIdx.y * total;  // right-hand side blockIdx.y
  xs += blockIdx.y * kF8Slices * total;
  xe += blockIdx.y * L;
  const int leaf = 4 * blockIdx.x + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (leaf >= L) return;  // uniform over the wavefront
  const double2* src = (const double2*)(x + (size_t)leaf * kF8N + 4 * lane);
  const double2 v01 = src[0], v23 = src[1];
  double v[4] = {v01.x, v01.y, v23.x, v23.y};
  double m = fmax(fmax(fabs(v[0]), fabs(v[1])), fmax(fabs(v[2]), fabs(v[3])));
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) m = fmax(m, __shfl_xor(m, o, 64));
  int e = 0;
  if (m > 0.0) frexp(m, &e);
  unsigned word[kF8Slices];
#pragma unroll
  for (int s = 0; s < kF8Slices; ++s) word[s] = 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double r = ldexp(v[k], 6 - e);  // |r| < 64
#pragma unroll
    for (int s = 0; s < kF8Slices; ++s) {
      if (s) r *= 128.0;
      const double q = rint(r);
      word[s] |= ((unsigned)(int)q & 0xffu) << (8 * k);
      r -= q;
    }
  }
#pragma unroll
  for (int s = 0; s < kF8Slices; ++s) *(unsigned*)(xs + (size_t)s * total + (size_t)leaf * kF8N + 4 * lane) = word[s];
  if (lane == 0) xe[leaf] = e;
}

__device__ __forceinline__ f8_v4 f8_mfma(f8_v4 a, f8_v4 b, f8_v4 c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// t[d] += the slice products of one 64-index block with i + j = d < S
template <int S>
__device__ __forceinline__ void f8_block(const f8_v4 a[S], const f8_v4 b[S], f8_v4 t[S]) {
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int i = 0; i <= d; ++i) t[d] = f8_mfma(a[i], b[d - i], t[d]);
}
template <int S>
__device__ __forceinline__ void f8_zero(f8_v4 t[S]) {
#pragma unroll
  for (int d = 0; d < S; ++d) t[d] = f8_v4{0, 0, 0, 0};
}
// the integer-scaled sum over d of 2^(-7d) times the d-sum of output r
template <int S>
__device__ __forceinline__ double f8_value(const f8_v4 t[S], int r) {
  double v = (double)t[S - 1][r];
#pragma unroll
  for (int d = S - 2; d >= 0; --d) v = (double)t[d][r] + 0x1p-7 * v;
  return v;
}

// B staging: 64 rows x 64 contraction bytes x S slices; per slice 256
// pieces of 16 bytes (piece p = bytes 16p .. 16p + 15 of a row), one per
// thread: wave w, lane l takes row 16 w + l % 16, piece l / 16 (each load
// instruction covers 16 rows x 64 contiguous bytes).  In LDS a slice is
// piece-major, [piece][row] at 16 bytes: a fragment read (rows 16 r + li,
// piece lk) and a store then cover 256 contiguous bytes per 16 lanes, which
// the LDS serves without bank conflicts (measured; a row-major 64-byte row
// with XOR-swizzled pieces costs four extra cycles per 128-bit read).
template <int S>
struct F8Stage {
  f8_v4 v[S];
};
template <int S>
__device__ __forceinline__ void f8_gload(F8Stage<S>& st, const int8_t* __restrict__ base, size_t slice, int ld,
                                         int row0, int c0, int nrows) {
  const int t = threadIdx.x, row = 16 * (t >> 6) + (t & 15), part = (t >> 4) & 3;
#pragma unroll
  for (int j = 0; j < S; ++j)
    st.v[j] = row < nrows ? *(const f8_v4*)(base + (size_t)j * slice + (size_t)(row0 + row) * ld + c0 + 16 * part)
                          : f8_v4{0, 0, 0, 0};
}
template <int S>
__device__ __forceinline__ void f8_lstore(const F8Stage<S>& st, int8_t* sb) {
  const int t = threadIdx.x, row = 16 * (t >> 6) + (t & 15), part = (t >> 4) & 3;
#pragma unroll
  for (int j = 0; j < S; ++j) *(f8_v4*)(sb + j * kF8Slice + part * 1024 + 16 * row) = st.v[j];
}
// B fragments (S slices) of row tile r from a staged block
template <int S>
__device__ __forceinline__ void f8_bfrag(const int8_t* sb, int r, f8_v4 b[S]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4, row = 16 * r + li;
#pragma unroll
  for (int s = 0; s < S; ++s) b[s] = *(const f8_v4*)(sb + s * kF8Slice + lk * 1024 + 16 * row);
}

// Phase 1: t[r] (r < MT1) = the slice d-sums of this lane's pair row of the
// leaf slices with B rows row0 + 16 r .. (B: [s][row][256], slice stride
// wslice) over the 256 nodes in four blocks of 64.  All A fragments (this
// lane's 16 bytes of every block and slice) are loaded at once; the B rows of
// block kb + 2 are loaded into registers once block kb + 1 is stored to the
// other LDS buffer.
template <int S, int MT1>
__device__ __forceinline__ void f8_phase1(const int8_t* __restrict__ xrow, long xs_slice,
                                          const int8_t* __restrict__ wbase, size_t wslice, int row0, int8_t* sbuf,
                                          f8_v4 t[4][S]) {
  constexpr int NKB = kF8N / 64, BUF = S * kF8Slice;
#pragma unroll
  for (int r = 0; r < MT1; ++r) f8_zero<S>(t[r]);
  f8_v4 a[NKB][S];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int s = 0; s < S; ++s) a[kb][s] = *(const f8_v4*)(xrow + (size_t)s * xs_slice + 64 * kb);
  F8Stage<S> st;
  f8_gload<S>(st, wbase, wslice, kF8N, row0, 0, 16 * MT1);
  __syncthreads();  // the previous user of sbuf is done
  f8_lstore<S>(st, sbuf);
  f8_gload<S>(st, wbase, wslice, kF8N, row0, 64, 16 * MT1);
  __syncthreads();
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    const int8_t* sb = sbuf + (kb & 1) * BUF;
#pragma unroll
    for (int r = 0; r < MT1; ++r) {
      f8_v4 b[S];
      f8_bfrag<S>(sb, r, b);
      f8_block<S>(a[kb], b, t[r]);
    }
    if (kb + 1 < NKB) f8_lstore<S>(st, sbuf + ((kb + 1) & 1) * BUF);
    if (kb + 2 < NKB) f8_gload<S>(st, wbase, wslice, kF8N, row0, 64 * (kb + 2), 16 * MT1);
    __syncthreads();
  }
}

// One work item: a tile of <= 64 pairs of one configuration (wave w owns
// pairs 16w..16w+15).  LR: Z = X W^T (R_c ranks) in FP64, cut into slices
// per pair row and staged in LDS as the A operand of Y = Z Q^T; dense (self
// operator): Y = X A^T for one block of 64 target rows (four row blocks per
// tile).  Results (FP64, exponents applied) go to the per-pair products Y.
// Tables and leaf slices hold kF8Slices slices per row (slice strides
// wslice, LM x n and xs_slice).
template <int S, bool LR>
__device__ __forceinline__ void f8_item(int item, int nrb, const int* __restrict__ t_cfg,
                                        const int* __restrict__ t_first, const int* __restrict__ t_count,
                                        const int* __restrict__ src, const int* __restrict__ lr_R,
                                        const int8_t* __restrict__ Wb, const int* __restrict__ Wexp,
                                        const int8_t* __restrict__ Qb, const int* __restrict__ Qexp,
                                        const int8_t* __restrict__ xs, const int* __restrict__ xe, long xs_slice,
                                        double* __restrict__ Y, int8_t* sbuf, int8_t* sZ8) {
  constexpr int n = kF8N, LM = kNearLrMax, BUF = S * kF8Slice;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tile = item / nrb, rb = item - tile * nrb;
  const int c = t_cfg[tile], p0 = t_first[tile], np = t_count[tile];
  const int ent = 16 * w + li;  // this lane's A-operand pair
  const int leaf = src[p0 + (ent < np ? ent : 0)];
  const int8_t* xrow = xs + (size_t)leaf * n + 16 * lk;
  const int my_ex = xe[leaf];
  // exponents of the output rows this lane holds: pairs 16w + 4lk + e
  int ex_out[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) ex_out[e] = __shfl(my_ex, 4 * lk + e, 16);
  const int MT1 = LR ? lr_R[c] / 16 : 4;
  const size_t wslice = LR ? (size_t)LM * n : (size_t)n * n;
  const int8_t* wbase = LR ? Wb + (size_t)c * kF8Slices * wslice : Wb;
  const int* wexp = LR ? Wexp + (size_t)c * LM : Wexp;
  const int row0 = LR ? 0 : 64 * rb;
  f8_v4 t[4][S];
  // padded ranks are 48 or 64 at K = 16; a smaller one takes the 48-row
  // product (the table rows past the rank are zero)
  if (MT1 <= 3)
    f8_phase1<S, 3>(xrow, xs_slice, wbase, wslice, row0, sbuf, t);
  else
    f8_phase1<S, 4>(xrow, xs_slice, wbase, wslice, row0, sbuf, t);
  if (!LR) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 64 * rb + 16 * r + li;
      const int ei = wexp[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pe = 16 * w + 4 * lk + e;
        if (pe < np) Y[(size_t)(p0 + pe) * n + i] = ldexp(f8_value<S>(t[r], e), ex_out[e] + ei - 12);
      }
    }
    return;
  }
  // Z (FP64) of this wave's pairs (ranks >= R zero); the exponent of every
  // pair's row of Z is the maximum over r and over the 16 lanes li that hold
  // the row.  Each lane cuts its 16 values into S slices under its row's
  // exponent and stores them to LDS as the A operand of the second product,
  // [slice][rank piece][pair][16 bytes] (piece-major, as the B staging)
  int ez_out[4];
  {
    double z[4][4], m[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ea = r < MT1 ? wexp[16 * r + li] : 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        z[r][e] = r < MT1 ? ldexp(f8_value<S>(t[r], e), ex_out[e] + ea - 12) : 0.0;
        m[e] = fmax(m[e], fabs(z[r][e]));
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) m[e] = fmax(m[e], __shfl_xor(m[e], o, 16));
      int ee = 0;
      if (m[e] > 0.0) frexp(m[e], &ee);
      ez_out[e] = ee;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int8_t* dst = sZ8 + r * 1024 + 16 * (16 * w + 4 * lk + e) + li;
        double q = ldexp(z[r][e], 6 - ez_out[e]);  // |q| < 64
#pragma unroll
        for (int s = 0; s < S; ++s) {
          if (s) q *= 128.0;
          const double qv = rint(q);
          dst[s * kF8Slice] = (int8_t)(int)qv;
          q -= qv;
        }
      }
  }
  // phase 2: Y = Z Q^T over the target rows in four chunks of 64 (stage g:
  // Q rows 64 g .. + 63, all 64 ranks, S slices), loaded two stages ahead
  // into registers and stored one stage ahead into the other buffer
  const int8_t* qbase = Qb + (size_t)c * kF8Slices * LM * n;
  const int* qexp = Qexp + (size_t)c * n;
  F8Stage<S> st[2];
  f8_gload<S>(st[0], qbase, (size_t)LM * n, LM, 0, 0, 64);
  f8_gload<S>(st[1], qbase, (size_t)LM * n, LM, 64, 0, 64);
  f8_lstore<S>(st[0], sbuf);  // the last phase-1 barrier freed sbuf
  f8_gload<S>(st[0], qbase, (size_t)LM * n, LM, 128, 0, 64);
  __syncthreads();  // the slices of Z and stage 0 are in LDS
  // A fragments of Z: this lane's pair 16w + li, ranks 16 lk + 0..15
  f8_v4 za[S];
#pragma unroll
  for (int s = 0; s < S; ++s) za[s] = *(const f8_v4*)(sZ8 + s * kF8Slice + lk * 1024 + 16 * (16 * w + li));
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int8_t* sb = sbuf + (g & 1) * BUF;
    if (g + 1 < 4) f8_lstore<S>(st[(g + 1) & 1], sbuf + ((g + 1) & 1) * BUF);
    if (g + 3 < 4) f8_gload<S>(st[(g + 1) & 1], qbase, (size_t)LM * n, LM, 64 * (g + 3), 0, 64);
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {  // one 16-row tile at a time: its products, then its outputs
      f8_v4 t2[S], b[S];
      f8_bfrag<S>(sb, r4, b);
      f8_zero<S>(t2);
      f8_block<S>(za, b, t2);
      const int i = 64 * g + 16 * r4 + li;
      const int ei = qexp[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pe = 16 * w + 4 * lk + e;
        if (pe < np) Y[(size_t)(p0 + pe) * n + i] = ldexp(f8_value<S>(t2, e), ez_out[e] + ei - 12);
      }
    }
    __syncthreads();
  }
}

// The tiles of one configuration list: work items (tiles x row blocks),
// row blocks per tile, the tile arrays and the phase-1 table.
struct F8List {
  int nitems, nrb;
  const int *cfg, *first, *count;
  const int8_t* W;
  const int* Wexp;
};

// Both item kinds in one persistent launch: each XCD takes an even share of
// the low-rank items (the heavier ones) and then an even share of the
// self-operator items, so the lighter items fill the tail of the heavier
// ones.  Items are configuration-major inside each kind, so an XCD's L2
// holds the slices of the few configurations it works on.
template <int S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_near_f8(F8List lr, F8List dn, const int* __restrict__ src, const int* __restrict__ lr_R,
          const int8_t* __restrict__ Qb, const int* __restrict__ Qexp, const int8_t* __restrict__ xs,
          const int* __restrict__ xe, long xs_slice, int L, double* __restrict__ Y, long sy) {
  xs += blockIdx.y * kF8Slices * xs_slice;  // right-hand side blockIdx.y
  xe += blockIdx.y * L;
  Y += blockIdx.y * sy;
  __shared__ __attribute__((aligned(16))) int8_t sbuf[2 * S * kF8Slice];
  __shared__ __attribute__((aligned(16))) int8_t sZ8[S * kF8Slice];
  const int nb = gridDim.x, bb = blockIdx.x;
  const int x = bb & 7;
  const int qa = lr.nitems >> 3, ra = lr.nitems & 7, qb = dn.nitems >> 3, rb = dn.nitems & 7;
  const int firstA = x * qa + min(x, ra), countA = qa + (x < ra ? 1 : 0);
  const int firstB = x * qb + min(x, rb), countB = qb + (x < rb ? 1 : 0);
  const int xwgs = (nb - x + 7) >> 3;
  for (int j = bb >> 3; j < countA + countB; j += xwgs) {
    if (j < countA)
      f8_item<S, true>(firstA + j, lr.nrb, lr.cfg, lr.first, lr.count, src, lr_R, lr.W, lr.Wexp, Qb, Qexp, xs, xe,
                       xs_slice, Y, sbuf, sZ8);
    else
      f8_item<S, false>(firstB + j - countA, dn.nrb, dn.cfg, dn.first, dn.count, src, lr_R, dn.W, dn.Wexp, Qb, Qexp,
                        xs, xe, xs_slice, Y, sbuf, sZ8);
  }
}

int persistent_grid_f8(int items, int max_wgs) {
  int grid = (max_wgs > 0 && items > max_wgs) ? max_wgs : items;
  return std::max(grid, std::min(items, 8));
}

}  // namespace

int launch_near_f8(const Plan* p, const double* fe, int nrhs, int max_wgs, hipStream_t s, std::string& err) {
  const HostPlan& H = p->H;
  const DevicePlan& D = p->D;
  const DeviceTables& DT = p->ctx->D;
  const long total = (long)H.L * kF8N, sNY = (long)H.np_src.size() * kF8N;
  // kF8Slices x L x n bytes per right-hand side fit the 4 x L x n bf16 slices' buffer
  static_assert(kF8Slices <= 8, "leaf slices exceed the slice buffer");
  int8_t* xs = (int8_t*)D.xs;
  hipLaunchKernelGGL(k_split_i8, dim3((H.L + 3) / 4, nrhs), dim3(256), 0, s, H.L, fe, xs, D.xs_exp);
  const F8List lr{(int)H.ml_cfg.size(), 1, D.ml_cfg, D.ml_first, D.ml_count, DT.f8_W, DT.f8_Wexp};
  const F8List dn{4 * (int)H.mt_cfg.size(), 4, D.mt_cfg, D.mt_first, D.mt_count, DT.f8_A, DT.f8_Aexp};
  const int items = lr.nitems + dn.nitems;
  // three quarters of the FP64 near-field kernels' work-group cap: this
  // kernel runs beside M2L on the caller's stream and finishes early, so
  // fewer resident work-groups leave M2L more room (wedge workload, int8
  // mixed step: 0.340 ms at 384 work-groups against 0.352 ms at 512)
  const int cap = max_wgs > 0 ? std::max(8, max_wgs * 3 / 4) : 0;
  if (items > 0)
    hipLaunchKernelGGL(k_near_f8<kF8Slices>, dim3(persistent_grid_f8(items, cap), nrhs), dim3(256), 0, s, lr, dn,
                       D.np_src, DT.lr_R, DT.f8_Q, DT.f8_Qexp, xs, D.xs_exp, total, H.L, D.near_y, sNY);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("mixed near field (int8): ") + hipGetErrorString(e);
    return VFX_EHIP;
  }
  return VFX_OK;
}

}  // namespace vfx
