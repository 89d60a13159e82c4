// Target-stationary near field (lists n, n+, n- of Section 4: the
// precomputed-table interactions of every leaf with its touching
// neighbours), K = 16, FP64.
//
// For a target leaf t of side h the near-field part of V is
//   h^2 sum_{(s, c) in list 1 of t} T_c f_s
// (plus the log(h) charge terms, which the far-field kernel adds).  The 32
// neighbour configurations form six classes under the symmetries of the
// square; with g mapping the class's base configuration b onto c,
// T_c = P_g T_b P_g^T, and T_b ~ Q_b W_b (low rank).  A table GEMM over the
// configuration-major pair tiles has already formed, for every pair,
// Z = (W_b P_g^T) f_s (the symmetry folded into the row factor's columns).
// This kernel finishes the sum per group of 16 consecutive targets, so each
// target's sum is formed in registers and written once:
//   self tile      acc += X T_self^T, row r = the group's target r;
//   class tiles    Y' = Z Q_b^T with row r = one pair of target r (at most
//                  one pair per target and tile, any configuration of the
//                  class); row r is written through its permutation,
//                  S[r][g_r(i)] = Y'[r][i], into an LDS stage in the target
//                  frame (a bijection per row, rows of distinct targets, so
//                  no two writes meet), and after one barrier every lane adds
//                  its own target nodes of S to its accumulators.
// The accumulation order is fixed by the plan (tile order), so results are
// bitwise repeatable and independent of the launch shape; no atomics.
//
// Layout (v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16],
// outputs D[(l/16) + 4r][l%16]): eight waves; wave w owns the target nodes
// 32w .. 32w+31 in two column tiles; acc[q][r] is target slot lk + 4r, node
// 32w + 16q + li (li = l%16, lk = l/16).  The A rows of a tile (the self
// rows, or the Z rows of up to four consecutive tiles of one class) are
// staged once in LDS for all waves; each wave streams its own B columns from
// L2 one block of 16 contraction indices ahead, and a run of class tiles
// shares every B block (a class's factor is read once per run, not per
// tile).  In MFMA step s of block
// kb, lane (li, lk) supplies index k = 16kb + 4lk + s on both sides (the B
// tables are stored contraction-fastest: self_T[i][j], cls_QT[k][i][a]).
// The LDS stage holds node (a, b) of a target at a*17 + b (rows of 16
// padded to 17), so the permuted writes of 16 lanes fall into distinct
// banks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "vfx_internal.h"

namespace vfx {

namespace {

typedef double ts_d4 __attribute__((ext_vector_type(4)));

constexpr int kTsN = 256;                // K^2
constexpr int kTsRow = 16 * 17;          // LDS stage: one target's nodes, rows of 16 padded to 17
constexpr int kTsThreads = 512;          // eight waves

__device__ __forceinline__ double ts_side(double root, int level) { return ldexp(root, -level); }
__device__ __forceinline__ int ts_pad(int i) { return (i >> 4) * 17 + (i & 15); }

constexpr int kTsLDA = 68;    // LDS row stride of staged A rows of a class tile (64 + 4)
constexpr int kTsLDX = 260;   // LDS row stride of the staged self rows (256 + 4)
constexpr int kTsMaxRun = 4;  // class tiles of one group sharing each B block

// Stage NR rows of KD values: row r <- src + rows[r] * ld (rows[r] < 0: a
// zero row), LDS stride lda; 16-byte pieces over the work-group, every
// thread issuing all its loads before its stores.
template <int NR, int KD>
__device__ __forceinline__ void ts_stage(double* sA, int lda, const double* __restrict__ src, const int* rows,
                                         int ld) {
  constexpr int PER = KD / 2, TOTAL = NR * PER, NT = (TOTAL + kTsThreads - 1) / kTsThreads;
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2 v[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int q = threadIdx.x + u * kTsThreads;
    v[u] = d2{0.0, 0.0};
    if (q < TOTAL) {
      const int r = q / PER, c = 2 * (q - r * PER);
      const int row = rows[r];
      if (row >= 0) v[u] = *(const d2*)(src + (size_t)row * ld + c);
    }
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int q = threadIdx.x + u * kTsThreads;
    if (q < TOTAL) {
      const int r = q / PER, c = 2 * (q - r * PER);
      *(d2*)(sA + r * lda + c) = v[u];
    }
  }
}

// y[u][q] += A_u (16 x 16 NKB, LDS rows u*16.. with stride lda) times
// B (16 NKB x this wave's two column tiles, columns at b0 and b1,
// contraction-fastest, offset by 4 lk), for NT tiles u sharing every B
// block.  Blocks are unrolled; each block's B loads are issued one block
// ahead.
template <int NT, int NKB>
__device__ __forceinline__ void ts_gemm(const double* sA, int lda, const double* __restrict__ b0,
                                        const double* __restrict__ b1, ts_d4 (*y)[2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  ts_d4 rb[2][2];
  rb[0][0] = *(const ts_d4*)b0;
  rb[0][1] = *(const ts_d4*)b1;
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    const int cur = kb & 1, nxt = cur ^ 1;
    if (kb + 1 < NKB) {
      rb[nxt][0] = *(const ts_d4*)(b0 + 16 * (kb + 1));
      rb[nxt][1] = *(const ts_d4*)(b1 + 16 * (kb + 1));
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const double a = sA[(16 * u + li) * lda + 16 * kb + 4 * lk + s];
        y[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rb[cur][0][s], y[u][0], 0, 0, 0);
        y[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rb[cur][1][s], y[u][1], 0, 0, 0);
      }
  }
}

// A run of NT class tiles (one class, consecutive in the plan): stage their
// Z rows, one product pass sharing each B block, then per tile the
// target-frame stage and the per-lane sums (two barriers per tile).
template <int NT>
__device__ __forceinline__ void ts_class_run(int R, const double* __restrict__ Z, const int* rows,
                                             const int* codes, const double* __restrict__ bc, double* sA,
                                             double* S, ts_d4 acc[2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int col0 = 32 * w + li;
  ts_d4 y[NT][2];
#pragma unroll
  for (int u = 0; u < NT; ++u) y[u][0] = y[u][1] = ts_d4{0.0, 0.0, 0.0, 0.0};
  // class ranks are padded to a multiple of 16 (48 or 64 here)
  if (R > 48) {
    ts_stage<16 * NT, 64>(sA, kTsLDA, Z, rows, kNearLrMax);
    __syncthreads();
    ts_gemm<NT, 4>(sA, kTsLDA, bc, bc + 16 * kNearLrMax, y);
  } else if (R > 32) {
    ts_stage<16 * NT, 48>(sA, kTsLDA, Z, rows, kNearLrMax);
    __syncthreads();
    ts_gemm<NT, 3>(sA, kTsLDA, bc, bc + 16 * kNearLrMax, y);
  } else if (R > 16) {
    ts_stage<16 * NT, 32>(sA, kTsLDA, Z, rows, kNearLrMax);
    __syncthreads();
    ts_gemm<NT, 2>(sA, kTsLDA, bc, bc + 16 * kNearLrMax, y);
  } else {
    ts_stage<16 * NT, 16>(sA, kTsLDA, Z, rows, kNearLrMax);
    __syncthreads();
    ts_gemm<NT, 1>(sA, kTsLDA, bc, bc + 16 * kNearLrMax, y);
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // row lk + 4e of tile u is target slot lk + 4e; its code holds g^-1
      const int g_ = d4_inverse(codes[16 * u + lk + 4 * e]);
      double* Sr = S + (lk + 4 * e) * kTsRow;
      Sr[ts_pad(d4_node(g_, 16, col0))] = y[u][0][e];
      Sr[ts_pad(d4_node(g_, 16, col0 + 16))] = y[u][1][e];
    }
    __syncthreads();  // the stage of tile u is complete
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double* Sr = S + (lk + 4 * e) * kTsRow;
      acc[0][e] += Sr[ts_pad(col0)];
      acc[1][e] += Sr[ts_pad(col0 + 16)];
    }
    __syncthreads();  // every lane has read the stage (and the A rows are consumed)
  }
}

__global__ void __launch_bounds__(kTsThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_near_ts(int ngroups, int L, const int* __restrict__ grp, const int* __restrict__ tcls,
          const int* __restrict__ trow, const int* __restrict__ tcode, const int* __restrict__ clsR,
          const double* __restrict__ selfT, const double* __restrict__ QT, const double* __restrict__ X,
          const double* __restrict__ Z, double root_size, const int* __restrict__ leaf_box,
          const int* __restrict__ box_level, double* __restrict__ out, long sx, long sz, long so) {
  X += blockIdx.y * sx;  // right-hand side blockIdx.y
  Z += blockIdx.y * sz;
  out += blockIdx.y * so;
  // staged A rows (a run of class tiles, or the self rows) and the
  // target-frame stage of one class tile
  __shared__ double sA[kTsMaxRun * 16 * kTsLDA > 16 * kTsLDX ? kTsMaxRun * 16 * kTsLDA : 16 * kTsLDX];
  __shared__ double S[kTsGroup * kTsRow];
  __shared__ int s_rows[kTsMaxRun * kTsGroup], s_codes[kTsMaxRun * kTsGroup];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int col0 = 32 * w + li;  // this lane's target node in column tile q: col0 + 16 q
  // persistent, XCD-aware: the work-groups of XCD x (blockIdx % 8 == x)
  // walk one contiguous range of groups (neighbouring targets share sources
  // and tables in that XCD's L2); the launch has at least min(8, groups)
  // work-groups, so every range has one
  const int nb = gridDim.x, bb = blockIdx.x, x = bb & 7;
  const int qg = ngroups >> 3, rg = ngroups & 7;
  const int xfirst = x * qg + min(x, rg), xcount = qg + (x < rg ? 1 : 0);
  const int xwgs = (nb - x + 7) >> 3;
  const double* bself = selfT + (size_t)col0 * kTsN + 4 * lk;
  for (int j = bb >> 3; j < xcount; j += xwgs) {
    const int g = xfirst + j;
    const int t0 = kTsGroup * g;
    ts_d4 acc[2];
    acc[0] = acc[1] = ts_d4{0.0, 0.0, 0.0, 0.0};
    const int tg1 = grp[g + 1];
    for (int tt = grp[g]; tt < tg1;) {
      const int k = tcls[tt];
      // the run of tiles of this class (at most kTsMaxRun)
      int nt = 1;
      while (nt < kTsMaxRun && tt + nt < tg1 && tcls[tt + nt] == k) ++nt;
      if (k == 0) nt = 1;
      if (tid < nt * kTsGroup) {
        s_rows[tid] = trow[kTsGroup * tt + tid];
        s_codes[tid] = tcode[kTsGroup * tt + tid];
      }
      __syncthreads();
      if (k == 0) {
        // the self operator on the group's own leaves, straight into acc
        ts_stage<16, kTsN>(sA, kTsLDX, X, s_rows, kTsN);
        __syncthreads();
        ts_d4 y1[1][2] = {{acc[0], acc[1]}};
#pragma unroll 1
        for (int c4 = 0; c4 < 4; ++c4)  // four runs of four blocks
          ts_gemm<1, 4>(sA + 64 * c4, kTsLDX, bself + 64 * c4, bself + 64 * c4 + 16 * kTsN, y1);
        acc[0] = y1[0][0];
        acc[1] = y1[0][1];
        __syncthreads();  // done with sA and the descriptors
      } else {
        const int R = clsR[k];
        const double* bc = QT + ((size_t)k * kTsN + col0) * kNearLrMax + 4 * lk;
        switch (nt) {
          case 1: ts_class_run<1>(R, Z, s_rows, s_codes, bc, sA, S, acc); break;
          case 2: ts_class_run<2>(R, Z, s_rows, s_codes, bc, sA, S, acc); break;
          case 3: ts_class_run<3>(R, Z, s_rows, s_codes, bc, sA, S, acc); break;
          default: ts_class_run<4>(R, Z, s_rows, s_codes, bc, sA, S, acc); break;
        }
      }
      tt += nt;
    }
    // h^2 times the sum, per target (raw: no 1/(2 pi), no log terms)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int t = t0 + lk + 4 * e;
      if (t >= L) continue;
      const double h = ts_side(root_size, box_level[leaf_box[t]]);
      out[(size_t)t * kTsN + col0] = h * h * acc[0][e];
      out[(size_t)t * kTsN + col0 + 16] = h * h * acc[1][e];
    }
  }
}

}  // namespace

int launch_near_ts(const Plan* p, const double* fe, double* V, int nrhs, int max_wgs, hipStream_t s,
                   std::string& err) {
  const HostPlan& H = p->H;
  const DevicePlan& D = p->D;
  const DeviceTables& DT = p->ctx->D;
  const int ngroups = (int)H.ts_grp.size() - 1;
  if (ngroups <= 0) return VFX_OK;
  const long sFL = (long)H.L * kTsN, sZ = (long)H.np_src.size() * kNearLrMax;
  // persistent grid: one work-group per CU fits (eight waves of up to 256
  // registers, 70 KB of LDS), so at most max_wgs / 2 work-groups, but at
  // least one per XCD range (min(8, groups)), since each range is walked by
  // its own XCD's groups
  const int cap = max_wgs > 0 ? std::max(1, max_wgs / 2) : 0;
  int grid = (cap > 0 && ngroups > cap) ? cap : ngroups;
  grid = std::max(grid, std::min(ngroups, 8));
  hipLaunchKernelGGL(k_near_ts, dim3(grid, nrhs), dim3(kTsThreads), 0, s, ngroups, H.L, D.ts_grp, D.ts_tcls,
                     D.ts_row, D.ts_code, DT.cls_R, DT.self_T, DT.cls_QT, fe, D.near_z, p->ctx->T.root_size,
                     D.leaf_box, D.box_level, V, sFL, sZ, sFL);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("k_near_ts: ") + hipGetErrorString(e);
    return VFX_EHIP;
  }
  return VFX_OK;
}

}  // namespace vfx
