// Internal declarations of the vfx library (host precompute, plan, kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vfx.h"

namespace vfx {

// Table indexing ------------------------------------------------------------
// Near field (list 1) configurations of a source leaf relative to a target
// leaf of side h (33 in a level-restricted tree):
//   0..8    same level, offset (dx, dy) in [-1,1]^2 -> (dx+1)*3 + (dy+1)
//   9..20   one level coarser, centre offset (ox, oy) in units h/2, odd
//           values in {-3,-1,1,3} with max(|ox|,|oy|) = 3
//   21..32  one level finer, centre offset in units h/4, same value set
constexpr int kNearConfigs = 33;
constexpr int kNearSelf = 4;  // the self interaction (colleague offset 0, 0)
// Near-field operators are applied in low-rank form Q W when the truncated
// pivoted QR at this relative tolerance has rank <= kNearLrMax and saves at
// least 40% of the dense work.
constexpr double kNearLrTol = 1e-14;
constexpr int kNearLrMax = 64;
// M2L (list 2): centre offset (dx, dy) in units h, |dx|,|dy| <= 3, index
// (dx+3)*7 + (dy+3); only max(|dx|,|dy|) >= 2 occurs.
constexpr int kM2LSlots = 49;
// P2L (list 4): a leaf one level coarser than the target box, centre offset
// in units h/2, odd values in {-5..5} with max(|ox|,|oy|) = 5; index
// ((ox+5)/2)*6 + (oy+5)/2.
constexpr int kP2LSlots = 36;
// M2P (list 3): a box one level finer than the target leaf, centre offset
// in units of its own half side, odd values in {-5..5} with
// max(|ox|,|oy|) = 5; the same 36-slot index ((ox+5)/2)*6 + (oy+5)/2.

// Symmetries of the square (the dihedral group D4) as 3-bit codes g:
// bit 0 swaps the axes, then bit 1 negates x and bit 2 negates y.  On the
// K x K first-kind grid (nodes symmetric about 0) g maps node (a, b) to
// node (a', b'): (A, B) = swap ? (b, a) : (a, b), a' = negx ? K-1-A : A,
// b' = negy ? K-1-B : B.
__host__ __device__ inline int d4_inverse(int g) {
  return (g & 1) ? (1 | (((g >> 2) & 1) << 1) | (((g >> 1) & 1) << 2)) : g;
}
__host__ __device__ inline void d4_point(int g, double x, double y, double* gx, double* gy) {
  const double X = (g & 1) ? y : x, Y = (g & 1) ? x : y;
  *gx = (g & 2) ? -X : X;
  *gy = (g & 4) ? -Y : Y;
}
__host__ __device__ inline int d4_node(int g, int K, int i) {
  const int a = i / K, b = i % K;
  int A = (g & 1) ? b : a, B = (g & 1) ? a : b;
  if (g & 2) A = K - 1 - A;
  if (g & 4) B = K - 1 - B;
  return A * K + B;
}
// Target-stationary near field: the 33 list-1 configurations fall into
// seven classes under D4 about the target centre: 0 self; 1 edge and 2
// corner colleagues; 3 corner and 4 edge coarse neighbours; 5 corner and 6
// edge fine neighbours.  A log-kernel table is invariant under an isometry
// applied to target and source alike, so with g mapping the class's base
// configuration b onto c,  T_c[g(i)][g(j)] = T_b[i][j].
constexpr int kNearClasses = 7;
constexpr int kTsGroup = 16;  // target leaves per group of the target-stationary near field

int near_config_coarse_index(int ox2, int oy2);  // -1 if invalid
int near_config_fine_index(int ox4, int oy4);
void near_config_geometry(int c, double* ox, double* oy, double* side);

struct Tables {
  int K = 0, n = 0, Kbar = 0, deg = 0, nG = 0, nX = 0, p = 0;
  double root_cx = 0, root_cy = 0, root_size = 0;
  std::vector<double> t, tbar;         // 1D first-kind nodes (ascending)
  std::vector<double> w2;              // n weights of the unit square, sum 1
  std::vector<double> stencil_xy;      // nX x 2 (Sbar frame)
  std::vector<double> A;               // nX x nG, row-major
  std::vector<double> AbarT;           // nG x Kbar^2 (transposed Sbar rows)
  std::vector<double> cbar;            // Kbar x Kbar values -> coefficients
  std::vector<double> near;            // 33 x n x n, [c][j][i]
  std::vector<double> near_s2;         // 33: (source side / target side)^2
  // low-rank near-field operators (near ~ Q W), see build_near_lowrank
  std::vector<int> lr_R, lr_rank;      // 33: padded rank (0 = dense), rank
  std::vector<double> lr_W;            // 33 x n x kNearLrMax, [c][j][a]
  std::vector<double> lr_Q;            // 33 x kNearLrMax x n, [c][a][i]
  // fixed-point bf16 slices of the K = 16 near-field operators as MFMA B
  // operands, contraction index fastest, 4 slices, one exponent per row:
  //   fx_W [c][s][a][j] = W[a][j] (exponent per rank a),
  //   fx_Q [c][s][i][a] = Q[i][a] (exponent per target node i),
  //   fx_A [s][i][j] = self table, row i (target node), column j
  // (v = 2^e sum_s q_s 2^(-8(s+1)), q_s integers of magnitude <= 256)
  std::vector<uint16_t> fx_W, fx_Q, fx_A;
  std::vector<int> fx_Wexp, fx_Qexp, fx_Aexp;
  // the same operands as kF8Slices int8 slices for the int8 matrix cores
  // (v = 2^e sum_s q_s 2^(-6-7s), q_s integers of magnitude <= 64)
  std::vector<int8_t> f8_W, f8_Q, f8_A;
  std::vector<int> f8_Wexp, f8_Qexp, f8_Aexp;
  std::vector<double> p2m;             // (p+1) x n complex, [k][j] (re,im)
  std::vector<double> l2p;             // n x (p+1) complex, [i][l]
  std::vector<double> m2m;             // 4 x (p+1) x (p+1) complex, [q][k][l]
  std::vector<double> l2l;             // 4 x (p+1) x (p+1) complex, [q][k][l]
  std::vector<double> m2l;             // 49 x (p+1) x (p+1) complex, [o][k][l]
  std::vector<double> p2l;             // 36 x (p+1) x n complex, [c][l][j]
  std::vector<double> p2l_area;        // 36: source area in units h^2 (0 if unused)
  // Scaled-Pascal forms of the translations (shared real matrices plus
  // diagonal complex scalings), used by the device kernels:
  //   M2L: b_l += t^l sum_{k>=1} C(k+l-1,l) (-t)^k a_k - a_0 t^l/l (l>=1),
  //        b_0 += a_0 log|d|, t = h/d
  //   M2M: b_l += w^l [ sum_{1<=k<=l} C(l-1,k-1) (2w)^-k a_k - a_0/l ],
  //        b_0 += a_0, w = (child - parent centre)/h_parent
  //   L2L: c_l  = (2w)^-l sum_{k>=l} C(k,l) w^k b_k
  std::vector<double> pas_m2l, pas_m2m, pas_l2l;  // P x P real, [k][l]
  std::vector<double> pas_m2l_t, pas_m2m_t, pas_l2l_t;  // the same, stored [l][k]
  std::vector<double> m2l_tpow, m2l_tneg;         // 49 x P complex: t^l, (-t)^k
  std::vector<double> m2l_logd;                   // 49: log|d/h|
  std::vector<double> m2m_in, m2m_out;            // 4 x P complex: (2w)^-k, w^l
  std::vector<double> l2l_in, l2l_out;            // 4 x P complex: w^k, (2w)^-l
  // P2L tables as real GEMM operands: [slot][j][row], row = 2l (re) or
  // 2l+1 (im), rows padded to p2l_rows (a multiple of 64)
  int p2l_rows = 0;
  std::vector<double> p2l_gemm;
  // P2M as a real GEMM operand: [j][row], rows as for P2L
  std::vector<double> p2m_gemm;
  // M2P (list 3) as a real GEMM operand: [slot][k][i], k < p2l_rows
  std::vector<double> m2p_gemm;
  // Target-stationary near field (K = 16; ts_ok when every non-self class
  // base is applied in low-rank form): class and D4 code of each
  // configuration (T_c = P_g T_b P_g^T), the base configuration and padded
  // rank of each class, the row factors of each configuration with the
  // symmetry folded into their columns, lr_Wp[c][j][a] = W_b[a][g^-1(j)]
  // (so Z = W_b P_g^T f), the column factor of each class as
  // cls_QT[k][i][a] = Q_b[i][a], and the self table as self_T[i][j] =
  // T_self[i][j].  ts_sym_err: max over c, i, j of
  // |T_c[g(i)][g(j)] - T_b[i][j]| relative to max |T_b|.
  bool ts_ok = false;
  std::vector<int> near_cls, near_g, cls_base, cls_R;
  std::vector<double> lr_Wp, cls_QT, self_T;
  double ts_sym_err = 0.0;
};

// Host precompute (quadrature.cpp, stencil.cpp)
void build_tables(Tables& T);
void gauss_legendre(int q, double* x, double* w);
void log_product_rule(int N, double* r, double* w, double* wl);
void padua_points(int deg, std::vector<double>& xy);
void build_stencil(Tables& T);
// pseudo-inverse of the m x n row-major matrix A (n x m row-major result),
// singular values below rel_cut * sigma_max dropped; returns the rank.
int pinv_jacobi(const double* A, int m, int n, double rel_cut, double* P);

// Device copy of the universal tables
struct DeviceTables {
  bool ready = false;
  int device = -1;
  double *t = nullptr, *tbar = nullptr, *w2 = nullptr, *AbarT = nullptr, *cbar = nullptr, *A = nullptr;
  double *near = nullptr, *near_s2 = nullptr;
  int* lr_R = nullptr;
  double *lr_W = nullptr, *lr_Q = nullptr;
  uint16_t *fx_W = nullptr, *fx_Q = nullptr, *fx_A = nullptr;
  int *fx_Wexp = nullptr, *fx_Qexp = nullptr, *fx_Aexp = nullptr;
  int8_t *f8_W = nullptr, *f8_Q = nullptr, *f8_A = nullptr;
  int *f8_Wexp = nullptr, *f8_Qexp = nullptr, *f8_Aexp = nullptr;
  double2 *p2m = nullptr, *l2p = nullptr, *m2m = nullptr, *l2l = nullptr, *m2l = nullptr, *p2l = nullptr;
  double* p2l_area = nullptr;
  double *pas_m2l = nullptr, *pas_m2m = nullptr, *pas_l2l = nullptr, *m2l_logd = nullptr, *p2l_gemm = nullptr;
  double *p2m_gemm = nullptr, *m2p_gemm = nullptr;
  double *pas_m2l_t = nullptr, *pas_m2m_t = nullptr, *pas_l2l_t = nullptr;
  double2 *m2l_tpow = nullptr, *m2l_tneg = nullptr, *m2m_in = nullptr, *m2m_out = nullptr, *l2l_in = nullptr,
          *l2l_out = nullptr;
  int* cls_R = nullptr;
  double *lr_Wp = nullptr, *cls_QT = nullptr, *self_T = nullptr;
};

// Device buffers that a captured HIP graph may refer to carry a generation
// count: every call that frees or reallocates them adds one, so a graph can
// tell at launch whether what it recorded still exists (see api.cpp).
struct Context {
  Tables T;
  DeviceTables D;
  uint64_t id = 0, gen = 0;
};

// Host-side plan ------------------------------------------------------------
struct HostPlan {
  int L = 0, B = 0, nlev = 0, ncut = 0;
  std::vector<int> box_level, box_ix, box_iy, box_parent, box_child0, box_leaf;
  std::vector<double> box_cx, box_cy;
  std::vector<int> level_start;              // nlev + 1
  std::vector<int> leaf_box;                 // L
  std::vector<int8_t> kind;                  // L
  std::vector<int> l1_ptr, l1_src, l1_cfg;   // per leaf
  std::vector<int> l1_srcbox;                // box of each list-1 source leaf
  std::vector<int> l2_ptr, l2_src, l2_off;   // per box
  std::vector<int> l2_tgt;                   // target box of each list-2 entry
  std::vector<int> m2l_grp;                  // groups of consecutive boxes (level >= 2):
                                             // <= 64 list-2 entries, <= 8 boxes
  std::vector<int> l3_ptr, l3_src, l3_cfg;   // per leaf (source boxes, M2P slot)
  // direct upward pass: non-leaf boxes at level >= 2, their leaf-descendant
  // pairs, wave groups {pos0, pos1, e0, e1, slot} and split boxes
  // {box, slot0, nslots}
  std::vector<int> up_box, up_ptr, up_src, up_pos, up_grp, up_split;
  std::vector<int> anc_ptr, anc, anc_leaf;   // per leaf: ancestors at level >= 2, nearest first
  std::vector<int> dn_grp;                   // leaf groups of the downward kernel
  int up_slots = 0;
  std::vector<int> l4_ptr, l4_src, l4_cfg;   // per box (source leaves)
  // list-1 pairs regrouped by table configuration (config-major, targets
  // ascending inside a configuration) for the batched near-field GEMM;
  // l1_slot maps each per-target list-1 entry to its pair index
  std::vector<int> np_src, np_tgt, l1_slot;
  std::vector<int> nt_cfg, nt_first, nt_count;  // dense GEMM tiles of <= 64 pairs
  std::vector<int> nl_cfg, nl_first, nl_count;  // low-rank tiles of <= 64 pairs
  // the same for the pairs applied in mixed precision (bf16 slices)
  std::vector<int> mt_cfg, mt_first, mt_count, ml_cfg, ml_first, ml_count;
  int precision = 0, mixed_min_level = 0;
  // target-stationary near field (FP64, K = 16): groups of kTsGroup
  // consecutive target leaves; per group a range of tiles (ts_grp); per tile
  // its class (0 self, 1..6 low-rank classes) and kTsGroup entries, one per
  // target slot: the A-operand row (the leaf itself for the self tile; for
  // a class tile the row of the list-1 factor products Z of one pair of
  // that target, i.e. the pair's index in the configuration-major order;
  // -1 for none) and d4_inverse(g) of the pair's configuration.  The
  // low-rank pairs' Z = W_b P_g^T f come from the table GEMM over the
  // configuration-major tiles nl_*.
  bool ts = false;
  int near_mode = 0;  // 0 pair-based near field, 1 target-stationary (vfx_plan_set_near_mode)
  std::vector<int> ts_grp, ts_tcls, ts_row, ts_code;
  // list-4 entries regrouped by P2L slot, the same way
  std::vector<int> p4_src, l4_slot, t4_cfg, t4_first, t4_count;
  // list-3 entries regrouped by M2P slot, the same way
  std::vector<int> p3_src, l3_slot, t3_cfg, t3_first, t3_count;
  // P2M over all leaves as one GEMM configuration
  std::vector<int> leaf_ids, t0_cfg, t0_first, t0_count;
  std::vector<int> cut_leaf;                 // ncut
  std::vector<int> owner;                    // L
  std::vector<int> ext_ptr, ext_tgt;         // per cut leaf (targets, itself first)
  std::vector<double> ext_geo;               // per target: x0, y0, scale in the Sbar frame
  std::vector<int> pinv_ptr;                 // ncut + 1 (in interior points)
  std::vector<uint16_t> pinv_idx;            // interior stencil indices
  std::vector<double> pinv_val;              // per cut: nG x N_I row-major
  bool factored = true;                      // false: P_i are computed on the GPU
  std::vector<uint8_t> sbar_given;           // ncut x Kbar^2
  double plan_seconds = 0;
};

struct DevicePlan {
  bool ready = false;
  int *box_level = nullptr, *box_child0 = nullptr, *box_leaf = nullptr, *box_parent = nullptr;
  double *box_cx = nullptr, *box_cy = nullptr;
  int* leaf_box = nullptr;
  int8_t* kind = nullptr;
  int8_t* fe_src = nullptr;  // per leaf: 2 written by the extension, 1 copied from f, 0 zero
  int *l1_ptr = nullptr, *l1_src = nullptr, *l1_cfg = nullptr, *l1_srcbox = nullptr;
  int *l2_ptr = nullptr, *l2_src = nullptr, *l2_off = nullptr, *l2_tgt = nullptr, *m2l_grp = nullptr;
  int *l3_ptr = nullptr, *l3_src = nullptr;
  int *up_box = nullptr, *up_ptr = nullptr, *up_src = nullptr, *up_pos = nullptr, *up_grp = nullptr,
      *up_split = nullptr;
  double2* up_part = nullptr;
  int *anc_ptr = nullptr, *anc = nullptr, *anc_leaf = nullptr, *dn_grp = nullptr;
  double2* locf = nullptr;  // full local expansion of every leaf, L x (p+1)  // partial multipoles of split boxes, up_slots x (p+1)
  int *l4_ptr = nullptr, *l4_src = nullptr, *l4_cfg = nullptr;
  int *np_src = nullptr, *l1_slot = nullptr, *nt_cfg = nullptr, *nt_first = nullptr, *nt_count = nullptr;
  int *nl_cfg = nullptr, *nl_first = nullptr, *nl_count = nullptr;
  int *mt_cfg = nullptr, *mt_first = nullptr, *mt_count = nullptr, *ml_cfg = nullptr, *ml_first = nullptr,
      *ml_count = nullptr;
  uint16_t* xs = nullptr;  // fixed-point slices of the leaf data: 4 x L x n bf16 (or 5 x L x n int8)
  int* xs_exp = nullptr;   // their exponent per leaf, L
  int cap = 0;             // right-hand sides the per-RHS buffers hold
  bool factored = false;   // pinv_val holds the P_i
  double* fac_ws = nullptr;  // scratch of the GPU factorisation
  double* near_y = nullptr;  // per-pair partial potentials, n_pairs x n
  double* near_z = nullptr;  // target-stationary path: per-pair factor products Z, n_pairs x 64
  int *ts_grp = nullptr, *ts_tcls = nullptr, *ts_row = nullptr, *ts_code = nullptr;
  int *p4_src = nullptr, *l4_slot = nullptr, *t4_cfg = nullptr, *t4_first = nullptr, *t4_count = nullptr;
  int *leaf_ids = nullptr, *t0_cfg = nullptr, *t0_first = nullptr, *t0_count = nullptr;
  double* p2l_y = nullptr;   // per-entry P2L partial locals, n_list4 x p2l_rows
  int *p3_src = nullptr, *l3_slot = nullptr, *t3_cfg = nullptr, *t3_first = nullptr, *t3_count = nullptr;
  double* m2p_y = nullptr;   // per-entry M2P values at the target nodes, n_list3 x n
  double* chg_part = nullptr;  // net-charge block partials, kChargeBlocks x chg_cap
  int chg_cap = 0;
  int *cut_leaf = nullptr, *ext_ptr = nullptr, *ext_tgt = nullptr, *pinv_ptr = nullptr;
  double* ext_geo = nullptr;
  uint16_t* pinv_idx = nullptr;
  double* pinv_val = nullptr;
  uint8_t* sbar_given = nullptr;
  double2 *mpole = nullptr, *local = nullptr;
  // batched extension (nrhs >= kExtGemmMinRhs): f_G of every (cut leaf,
  // right-hand side), ncut x cap x nG, and A_{Xbar,G} f_G on the Sbar grid,
  // ncut x cap x Kbar^2 (column c * nrhs + r)
  double *ext_fg = nullptr, *ext_g = nullptr;
};

struct Plan {
  Context* ctx = nullptr;
  HostPlan H;
  DevicePlan D;
  // P2L and the near field run on a side stream (default priority), forked
  // after the extension; M2L waits for P2L (p2l_ev), the far-field kernel
  // for the whole side stream (join_ev)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr, p2l_ev = nullptr, up_ev = nullptr;
  // per-phase timing: one set of kEvents events per timed execute
  static constexpr int kEvents = 14;
  // launch parameters chosen by vfx_plan_autotune
  struct Tune {
    int near_wgs = 512;  // work-group cap of the persistent near-field kernels (2 per CU,
                         // leaving room for the caller's stream beside them)
    int dense_mtb = 4;   // row tiles per block of the dense near-field GEMM (K = 16)
  } tune;
  bool timing = false;
  std::vector<hipEvent_t> ev;   // kEvents * capacity
  int n_timed = 0;
  uint64_t id = 0, gen = 0;     // identity and generation of the device buffers
};

// plan.cpp
int build_host_plan(const Tables& T, const vfx_tree* tree, HostPlan& H, std::string& err, bool defer_factor = false);
int factor_gpu(Plan* p, hipStream_t s, std::string& err);
int build_near_tiles(const Tables& T, HostPlan& H, int mode, int min_level, std::string& err);

// kernels.hip
int upload_tables(Context* c, std::string& err);
int upload_plan(Plan* p, std::string& err);
void free_plan_device(Plan* p);
void free_tables_device(Context* c);
int launch_execute(Plan* p, int nrhs, const double* f_leaf, const double* f_cut, double* fe, double* V,
                   hipStream_t s, std::string& err);
int ensure_rhs_capacity(Plan* p, int nrhs, std::string& err);
int launch_interp(Plan* p, const double* V, long npts, const double* px, const double* py, double* out,
                  hipStream_t s, std::string& err);
int launch_net_charge(Plan* p, const double* fe, int nrhs, double* out, hipStream_t s, std::string& err);
// ext_batch.hip: batches of at least this many right-hand sides compute
// the extension's two matrix products (A1 per cut leaf, A2 over every cut
// leaf and right-hand side) as FP64 MFMA GEMMs ahead of the extension kernel
constexpr int kExtGemmMinRhs = 8;
int launch_ext_gemm(const Plan* p, const double* f_cut, int nrhs, hipStream_t s, std::string& err);
int launch_ext_eval(const Plan* p, const double* f_cut, double* fe, int nrhs, hipStream_t s, std::string& err);
// mixed.hip
int launch_near_fx(const Plan* p, const double* fe, int nrhs, int max_wgs, hipStream_t s, std::string& err);
// int8 slices per operand row of the mixed-precision near field (mode 2)
constexpr int kF8Slices = 5;
int launch_near_f8(const Plan* p, const double* fe, int nrhs, int max_wgs, hipStream_t s, std::string& err);
// near.hip
int launch_near_ts(const Plan* p, const double* fe, double* V, int nrhs, int max_wgs, hipStream_t s,
                   std::string& err);
int launch_net_charge_noalloc(Plan* p, const double* fe, int nrhs, double* out, hipStream_t s, std::string& err);
int noalloc_max_rhs();

// mlp.hip (refinement classifier)
int mlp_param_count();
int mlp_forward(const float* th, const float* X, long B, float* logits, hipStream_t s);
long mlp_grad_work(long B);
int mlp_grad(const float* th, const float* X, const float* y, long B, float* grad, float* work, hipStream_t s);
int mlp_adam(float* th, const float* grad, float* m, float* v, int step, float lr, float b1, float b2, float eps,
             hipStream_t s);
int mlp_to_f16(const float* a, uint16_t* h, long n, hipStream_t s);
int mlp_infer_f16(const uint16_t* th, const uint16_t* X, long B, float* logits, hipStream_t s);

}  // namespace vfx
