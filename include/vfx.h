/*
 * vfx: function extension from cut leaves + adaptive volume FMM, on one GPU.
 *
 * The method (Fryklund & Greengard, "An FMM accelerated Poisson solver for
 * complicated geometries in the plane using function extension"):
 *   - the source f is sampled on K x K first-kind Chebyshev grids on the
 *     leaves of an adaptive, level-restricted quad-tree over a square root
 *     box (Section 4);
 *   - on every cut leaf (a leaf the boundary crosses) f is known only at the
 *     interior points of a universal stencil X = X_S u X_Sbar u G, and is
 *     extended by least squares through the universal interpolation matrix
 *     A_{X,G} (Section 3.2), resampled from its total-order Chebyshev
 *     expansion on the extension square onto every leaf of the cut leaf's
 *     extension list (Section 4.1, eq. chebexpbarS);
 *   - the volume potential V(x) = int (1/2pi) log|x-y| f^e(y) dy of the
 *     extended data is evaluated at every leaf node by a volume FMM
 *     (Section 1 eqs. volpot/greenf/volinte; Section 4, the near/far split
 *     of the VFMM remark and the tree-levels figure).
 *
 * Conventions
 *   - Root box: centre (root_cx, root_cy), side root_size.  A leaf at level
 *     l with integer position (ix, iy), 0 <= ix, iy < 2^l, has side
 *     h = root_size / 2^l and centre
 *     (root_cx - root_size/2 + (ix + 1/2) h, root_cy - root_size/2 + (iy + 1/2) h).
 *   - Leaf grid: 1D nodes t_a = -cos((2a+1) pi / (2K)), a = 0..K-1
 *     (ascending, first kind); node (a, b) of a leaf sits at
 *     (cx + h t_a / 2, cy + h t_b / 2) and has flat index a*K + b.
 *   - Stencil of a cut leaf (Section 3.2), in the reference frame of its
 *     extension square Sbar = [-1,1]^2 (side 3h, same centre), so the leaf
 *     itself is [-1/3,1/3]^2: first the K*K leaf nodes (t_a/3, t_b/3), then
 *     the Kbar*Kbar first-kind nodes of Sbar, then the N_G support nodes G
 *     (Padua points of degree deg, N_G = (deg+1)(deg+2)/2), |X| points in all.
 *     vfx_stencil_points returns their coordinates.
 *   - Cut leaves are numbered in ascending leaf order; that order is also the
 *     canonical order of the extension-list tie rule.
 *
 * Ownership and threading
 *   - Every pointer argument is owned by the caller.  Host arrays passed to
 *     vfx_create / vfx_plan_create are copied; device arrays passed to
 *     vfx_execute must stay valid until the work on the stream completes.
 *   - A context or plan must not be used from two threads at once.
 *   - Every call returns VFX_OK (0) or a negative status; vfx_last_error()
 *     returns a thread-local description of the last failure.  No C++
 *     exception crosses this interface.
 */
#ifndef VFX_H
#define VFX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VFX_OK 0
#define VFX_EINVAL (-1)  /* bad argument (null pointer, size out of range)    */
#define VFX_ETREE (-2)   /* tree not a quad-tree partition, not balanced, or  */
                         /* extension restriction violated                    */
#define VFX_EHIP (-4)    /* HIP runtime error                                 */
#define VFX_ENOMEM (-5)  /* host or device allocation failed                  */

typedef struct vfx_ctx vfx_ctx;
typedef struct vfx_plan vfx_plan;
typedef struct vfx_graph vfx_graph;

typedef struct {
  int32_t K;         /* leaf grid size: 4, 8, 12 or 16 (the paper fixes 8)   */
  int32_t Kbar;      /* grid size on the extension square, 2..16 (paper: 12)  */
  int32_t deg;       /* stencil degree; N_G = (deg+1)(deg+2)/2 (paper: 66)    */
  int32_t p;         /* FMM expansion order: terms 0..p, 4 <= p <= 60         */
  double root_cx, root_cy, root_size;
} vfx_params;

/* Create a context on the current HIP device: builds the universal tables
 * on the host and uploads them on first use:
 *   - the stencil matrix A_{X,G} of Section 3.2 (eq. defA; Gaussian basis in
 *     its flat limit, the total-degree-deg interpolant on the support nodes
 *     G), which every cut leaf shares;
 *   - the near-field tables of Section 4 (lists n, n+, n-: integrals of the
 *     log kernel against the leaf basis for the 33 neighbour configurations
 *     of a level-restricted tree, in units of the target side);
 *   - the expansion operators of the far field (multipole / local, order p).
 * Tables depend only on (K, Kbar, deg, p) and are cached for the process.
 * Errors: VFX_EINVAL for parameters out of range or a null argument,
 * VFX_ENOMEM if host memory runs out. */
int vfx_create(const vfx_params* prm, vfx_ctx** out);
int vfx_destroy(vfx_ctx* ctx);

/* Sizes of the stencil: |X| and N_G. */
int vfx_stencil_size(const vfx_ctx* ctx, int32_t* n_stencil, int32_t* n_support);
/* Stencil coordinates in the Sbar frame, xy[2*k], xy[2*k+1]; host array of
 * 2*|X| doubles. */
int vfx_stencil_points(const vfx_ctx* ctx, double* xy);
/* The K 1D leaf nodes t_a (host array of K doubles). */
int vfx_leaf_nodes(const vfx_ctx* ctx, double* t);

typedef struct {
  int32_t n_leaves;
  const int32_t* level;    /* host, n_leaves                                  */
  const int32_t* ix;       /* host, n_leaves                                  */
  const int32_t* iy;       /* host, n_leaves                                  */
  const int8_t* kind;      /* host, n_leaves: 0 exterior, 1 regular, 2 cut    */
  const uint8_t* cut_mask; /* host, n_cut x |X| bytes: 1 = stencil point lies */
                           /* inside the domain (cut leaves in leaf order)    */
} vfx_tree;

/* Build a plan for one tree (Section 4 data structures): the box hierarchy,
 * the FMM interaction lists, the extension lists (closest cut centre, later
 * cut leaf wins ties) and, per cut leaf, the pseudo-inverse of the interior
 * rows of A_{X,G} (singular values below 1e-13 sigma_max dropped).  Errors:
 * VFX_ETREE when the leaves do not tile the root, the tree is not level
 * restricted, or a cut leaf would extend onto a coarser neighbour. */
int vfx_plan_create(vfx_ctx* ctx, const vfx_tree* tree, vfx_plan** out);
int vfx_plan_destroy(vfx_plan* plan);

typedef struct {
  int32_t n_leaves, n_boxes, n_levels, n_cut, n_ext_targets;
  int64_t n_list1, n_list2, n_list3, n_list4;
  int64_t pinv_doubles;    /* size of the stored per-cut-leaf operators      */
  double plan_seconds;     /* host time spent in vfx_plan_create             */
} vfx_plan_stats;
int vfx_plan_stats_get(const vfx_plan* plan, vfx_plan_stats* out);

/* Owner cut leaf of every leaf (host array, n_leaves int32): the cut leaf
 * whose extension list contains it, itself for a cut leaf, -1 otherwise. */
int vfx_plan_ext_owner(const vfx_plan* plan, int32_t* owner);

/*
 * Run the extension and the volume FMM on `stream` (a hipStream_t; NULL for
 * the default stream):
 *   - on every cut leaf, f_G = A^+_{X^I,G} f_{X^I} and the values on the
 *     Kbar x Kbar grid of the extension square, A_{Xbar^E,G} f_G where no
 *     data is given (Section 3.2), the total-order Chebyshev expansion on the
 *     extension square (Section 4.1, eq. chebexpbarS) evaluated on the K x K
 *     grid of every leaf in the cut leaf's extension list;
 *   - V[f^e](x) = int (1/2pi) log|x - y| f^e(y) dy at every leaf node
 *     (Section 1, eqs. volpot, greenf, volinte), near field by the tables,
 *     far field by multipole and local expansions (Section 4).
 * All four arrays are device memory, row-major:
 *   f_leaf  n_leaves x K^2   samples of f on regular leaves (other rows
 *                            are not read)
 *   f_cut   n_cut x |X|      samples of f at the stencil points of each cut
 *                            leaf (exterior entries are not read)
 *   fe_out  n_leaves x K^2   extended data f^e (written)
 *   V_out   n_leaves x K^2   V[f^e] at every leaf node (written)
 * f_leaf, fe_out and V_out must be 16-byte aligned (they are accessed in
 * 16-byte pieces).
 * The arrays carry no sizes: the caller guarantees the extents above.
 * Inputs are not scanned: a NaN or Inf in a value that is read propagates
 * through IEEE arithmetic into f^e and V (the far field spreads it to every
 * leaf), and no other error results.
 * Asynchronous: returns after enqueueing.  Errors: VFX_EINVAL for null
 * or misaligned pointers, or a call under a stream capture that
 * vfx_graph_begin did not start on this stream; VFX_EHIP if a launch fails.
 */
int vfx_execute(vfx_plan* plan, const double* f_leaf, const double* f_cut, double* fe_out,
                double* V_out, void* stream);

/* ---- refinement classifier (learned refine/keep decision) --------------
 * A 64-64-64-1 perceptron with exact GELU activations whose input is the
 * last four rows (16 values each) of a K = 16 leaf's Chebyshev coefficient
 * array, in the order the host feature code fixes, and whose output logit
 * means "refine" (the refinement test it learns is the plain coefficient-
 * tail criterion of the tree; the host keeps that criterion as fallback and
 * judge).  Parameters: one flat FP32 vector of vfx_mlp_param_count() values,
 * W1 (64 x 64, [out][in]), b1, W2, b2, w3 (64), b3 (1).  All pointers are
 * device memory, row-major (x: batch x 64); calls are asynchronous on
 * `stream`; VFX_EINVAL for null pointers or bad sizes.
 *   vfx_mlp_forward   FP32 logits
 *   vfx_mlp_grad      gradient of the mean binary cross-entropy of the
 *                     logits against labels y (0/1); `work` holds
 *                     vfx_mlp_grad_work(batch) floats of per-tile partials,
 *                     summed in tile order (deterministic)
 *   vfx_mlp_adam      one Adam step (bias-corrected, step >= 1) on theta
 *                     with moment buffers m, v
 *   vfx_f32_to_f16    FP16 copy (round to nearest) of n floats
 *   vfx_mlp_infer_f16 logits from FP16 parameters and FP16 inputs with FP32
 *                     accumulation */
int vfx_mlp_param_count(void);
int64_t vfx_mlp_grad_work(int64_t batch);
int vfx_mlp_forward(const float* theta, const float* x, int64_t batch, float* logits, void* stream);
int vfx_mlp_grad(const float* theta, const float* x, const float* y, int64_t batch, float* grad, float* work,
                 int64_t work_floats, void* stream);
int vfx_mlp_adam(float* theta, const float* grad, float* m, float* v, int step, float lr, float beta1, float beta2,
                 float eps, void* stream);
int vfx_f32_to_f16(const float* a, uint16_t* h, int64_t n, void* stream);
int vfx_mlp_infer_f16(const uint16_t* theta_h, const uint16_t* x_h, int64_t batch, float* logits, void* stream);

/* Values at arbitrary points of data given on the leaf grids of the plan's
 * tree (e.g. V_out, at the boundary nodes a boundary-integral solve needs):
 * the tensor first-kind Chebyshev interpolant of the K x K samples of the
 * leaf that holds each point (the paper evaluates V off the grid by
 * interpolating the leaf expansions, \S4).  V: device, n_leaves x K^2 as in
 * vfx_execute; px, py: device, npts coordinates; out: device, npts values
 * (NaN for points outside the root box; a point on an edge between leaves
 * uses the upper/right one).  Asynchronous on `stream`.  VFX_EINVAL for null
 * pointers or npts < 0. */
int vfx_interp(vfx_plan* plan, const double* V, int64_t npts, const double* px, const double* py, double* out,
               void* stream);

/* Net charge A^e = integral of f^e over the tree, per right-hand side: the
 * coefficient of the log|x| growth of the volume potential, which the
 * exterior problem's boundary solve offsets in its constraint on the
 * densities (\S6, the exterior problem).  Each leaf contributes h^2 times
 * the tensor first-kind Chebyshev (Fejer) rule of the unit square applied to
 * its K x K samples.  fe: device, nrhs x n_leaves x K^2 as vfx_execute(_batch)
 * writes it; out: device, nrhs doubles (written).  The sum runs over a fixed
 * partition of the leaves, so the result is bitwise repeatable.  Asynchronous
 * on `stream`; the plan keeps a buffer of 2048 partial sums per right-hand
 * side, allocated by the first call that needs it (under stream capture that
 * call must already have happened).  VFX_EINVAL for null pointers or
 * nrhs < 1. */
int vfx_net_charge(vfx_plan* plan, const double* fe, int nrhs, double* out, void* stream);

/* The net charge of vfx_net_charge, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same result bit for bit, but the
 * block partials live in a fixed device array of the library (1 MiB per GPU,
 * held until the process ends) instead of a buffer of the plan, and the call
 * allocates nothing.  The plan's device data must already be resident on the
 * current device (one vfx_execute or vfx_net_charge before); nrhs may be at
 * most vfx_net_charge_noalloc_max_rhs() (64).  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (on different streams, or
 * from different threads) race and give wrong results; calls ordered on one
 * stream are safe.  VFX_EINVAL for null pointers, nrhs < 1 or above the
 * limit, a plan not yet on the device or on another device. */
int vfx_net_charge_noalloc(vfx_plan* plan, const double* fe, int nrhs, double* out, void* stream);
int vfx_net_charge_noalloc_max_rhs(void);

/* Precision of the near field (mode 0, 1 or 2; VFX_EINVAL otherwise).
 * mode 0: FP64 everywhere (the default).  mode 1: the list-1 interactions whose source
 * leaf is at level >= min_level are applied on the bf16 matrix cores (the
 * tables of Section 4): every operand row (leaf data, table rows, the
 * low-rank products Z) is cut into four 8-bit fixed-point slices under its
 * own exponent, the slice products are grouped by the sum of their slice
 * indices, and each group is summed exactly in FP32 over blocks of 128
 * contraction indices before being widened to FP64; the result keeps about
 * 2^-32 of the operands' row maxima and is stored in FP64 like the FP64
 * path's.  mode 2: the same interactions on the int8 matrix cores: every
 * operand row is cut into five 7-bit fixed-point slices (the leading one
 * 6 bits plus sign, each a signed integer of magnitude <= 64), the slice
 * pairs whose index sum is below 5 are multiplied and each group is summed
 * exactly in int32 over the whole contraction; the result keeps about
 * 2^-34 of the operands' row maxima (FP64 results as in mode 1).  In both
 * modes the log(h) terms, every multipole and local expansion, the M2L
 * log term and the final sums stay FP64.  The near-field contribution of a
 * source of side h scales like h^2, so a min_level bounds the error those
 * interactions can add.  Available for
 * K = 16 only (VFX_EINVAL otherwise, and the plan stays FP64).  The plan's
 * device data are rebuilt on the next vfx_execute; the call synchronises the
 * device and must not overlap an execute of the same plan. */
int vfx_plan_set_precision(vfx_plan* plan, int mode, int min_level);

/* Near-field strategy of the FP64 path at K = 16.  mode 0 (the default):
 * pair-based - every list-1 pair's table product is formed on its own
 * (configuration-major tiles of 32-64 pairs, operators shared through LDS)
 * and the far-field kernel sums each target's pair products.  mode 1:
 * target-stationary - the products of each group of 16 consecutive target
 * leaves are summed in registers and each leaf's near-field sum is written
 * once: the 32 neighbour configurations are folded onto six symmetry
 * classes of the square (T_c = P_g T_b P_g^T, Section 4 tables in
 * low-rank form Q_b W_b), a table GEMM forms every pair's W_b P_g^T f, and a
 * per-group kernel applies Q_b and the self table.  Both compute the same
 * sum (they differ by rounding); mode 1 reads and writes far less memory
 * but does more matrix work (tiles of one pair per target).  Other K and
 * mixed pairs keep mode 0.  The plan's device data are rebuilt on the next
 * vfx_execute (graphs that captured it are invalidated); the call must not
 * overlap an execute of the same plan.  VFX_EINVAL for other modes. */
int vfx_plan_set_near_mode(vfx_plan* plan, int mode);

/* Plan with the per-cut-leaf least-squares operators computed on the GPU
 * (the plan stage on the GPU).  flags = VFX_PLAN_DEFER_FACTOR: the host builds
 * only the lists and the interior index sets, and vfx_plan_factor_gpu then
 * computes every P_i = A_{X^I,G}^+ on the device, one work-group per cut
 * leaf: Householder QR of the N_I x N_G rows of A (the paper's QR per cut
 * square, \S7), one-sided Jacobi SVD of R, singular values below
 * 1e-13 sigma_max dropped (minimum-norm when N_I < N_G), P_i = pinv(R) Q^T,
 * all in FP64.  It is asynchronous on `stream`; executes on other streams
 * must be ordered after it by the caller.  vfx_execute on a deferred plan
 * that was not factored returns VFX_EINVAL.  Supports N_G <= 66 (stencil
 * degree <= 10; VFX_EINVAL otherwise).  flags = 0 is vfx_plan_create. */
#define VFX_PLAN_DEFER_FACTOR 1
int vfx_plan_create_ex(vfx_ctx* ctx, const vfx_tree* tree, int flags, vfx_plan** out);
int vfx_plan_factor_gpu(vfx_plan* plan, void* stream);

/* Many right-hand sides on one tree (batched execution).  Inputs and
 * outputs are stacked: f_leaf, fe_out, V_out are nrhs x n_leaves x K^2 and
 * f_cut is nrhs x n_cut x |X| (device, row-major).  Every kernel of the
 * path runs once for the whole batch with the right-hand side as a grid
 * dimension: the near-field and expansion GEMMs see nrhs times as many
 * pairs, and the latency-bound tree kernels fill the GPU.  The extension
 * (Section 3.2): below 8 right-hand sides one work-group per (cut leaf,
 * right-hand side), the work-groups of a cut leaf consecutive so that its
 * P_i is reused from L2, and the results are bitwise those of nrhs separate
 * vfx_execute calls; from 8 on, its two matrix products run as FP64 MFMA
 * GEMMs (f_G = P_i f_I per cut leaf over blocks of 64 right-hand sides, P_i
 * read once per block; A_{Xbar,G} f_G over every cut leaf and right-hand
 * side) and the Chebyshev step and target evaluation take eight right-hand
 * sides per work-group; the results then differ from separate executes by
 * rounding only (the products are summed in another order).  The plan
 * grows its per-right-hand-side buffers on first use (it synchronises the
 * device then); from 8 right-hand sides they include the extension's
 * intermediate products, n_cut x nrhs x (N_G + Kbar^2) doubles.  Errors as
 * vfx_execute, and VFX_EINVAL for nrhs < 1. */
int vfx_execute_batch(vfx_plan* plan, int nrhs, const double* f_leaf, const double* f_cut, double* fe_out,
                      double* V_out, void* stream);

/* Launch-parameter autotuner: times `reps` executes of the given batch
 * for each candidate (work-group cap of the persistent near-field kernels
 * 256/512/768/1024; row tiles per block of the dense near-field GEMM 4/8 at
 * K = 16) with HIP events on `stream` and keeps the fastest for later
 * executes of the plan; choice[0..1] (optional) receive it.  The choices
 * change only how work is distributed, not the arithmetic: results are
 * bitwise independent of them.  The buffers are overwritten. */
int vfx_plan_autotune(vfx_plan* plan, int nrhs, const double* f_leaf, const double* f_cut, double* fe_out,
                      double* V_out, void* stream, int reps, int32_t* choice);

/* Set the same two launch parameters directly (for example the choice an
 * earlier autotune made): the work-group cap of the persistent near-field
 * kernels (1..65535; default 512, two work-groups per CU; the int8 near
 * field of precision mode 2 takes three quarters of it) and the row
 * tiles per block of the dense near-field GEMM (4 or 8).  Results are
 * bitwise independent of them.  VFX_EINVAL outside those ranges. */
int vfx_plan_set_launch(vfx_plan* plan, int near_wgs, int dense_mtb);

/* HIP graph capture of a sequence of executes, possibly of many plans
 * (many uneven trees in one launch): vfx_graph_begin starts a capture
 * on `stream`; vfx_execute / vfx_execute_batch / vfx_net_charge calls on that
 * stream are recorded (each plan must have executed once before, with at
 * least as many right-hand sides, and have timing off); vfx_graph_end ends
 * the capture and instantiates the graph; vfx_graph_launch replays all of it
 * with one launch on a stream; vfx_graph_destroy frees it.  The graph holds
 * no memset nodes.
 *   Streams: while a capture is active, the library accepts calls only on
 * the stream vfx_graph_begin started it on.  A call on any other capturing
 * stream (a stream forked from that one by events, or a capture the caller
 * started without vfx_graph_begin) returns VFX_EINVAL and records nothing:
 * capturing executes on forked streams has ended in a crash inside
 * hipStreamEndCapture, so that mode is refused.
 *   Lifetime: a graph refers to the device buffers of the contexts and plans
 * it captured.  vfx_destroy, vfx_plan_destroy, vfx_plan_set_precision, a
 * vfx_execute_batch with more right-hand sides than the plan held, and a
 * vfx_net_charge with more right-hand sides than any earlier call free or
 * reallocate them; after any of these on a captured context or plan,
 * vfx_graph_launch returns VFX_EINVAL (capture again).
 * VFX_EHIP if the runtime refuses a step. */
int vfx_graph_begin(void* stream);
int vfx_graph_end(void* stream, vfx_graph** out);
int vfx_graph_launch(vfx_graph* graph, void* stream);
int vfx_graph_destroy(vfx_graph* graph);

/* Per-phase timing with HIP events.  The near-field kernels run on a side
 * stream of the plan (default priority), forked from `stream` after the
 * extension and joined before the far-field kernel; their phases are timed
 * with events on that side stream, the others on `stream`.  While enabled,
 * every vfx_execute records its events (at most 4096 executes are recorded;
 * enabling again restarts the count).  The query synchronises on the last
 * recorded event and returns, averaged over the recorded executes, the
 * milliseconds of eleven phases:
 *   ms[0] extension (the cut-leaf kernel, with the f^e initialisation of
 *         the other leaves)
 *   ms[1] P2M and the upward pass
 *   ms[2] M2L (with the wait for P2L)
 *   ms[3] downward pass (leaf local expansions)
 *   ms[4] near field, first kernel (side stream): the low-rank pairs, or on
 *         the target-stationary path (FP64, K = 16) the factor products
 *   ms[5] near field, second kernel (side stream): the dense pairs, or the
 *         per-target-group kernel of the target-stationary path
 *   ms[6] far field (list-1 and list-3 sums, L2P)   ms[7] total
 *   ms[8] P2L, list-4 products (side stream)
 *   ms[9] M2P, list-3 products (side stream, after the near field and the
 *         upward pass)
 *   ms[10] f^e initialisation: 0 (it runs inside the extension launch,
 *         which ms[0] times)
 * and ms[11] (if n_out >= 12) the number of executes averaged.  Phases on
 * the two streams overlap, so they do not add up to the total.  n_out must
 * be >= 11. */
int vfx_plan_set_timing(vfx_plan* plan, int enable);
int vfx_plan_timings(vfx_plan* plan, double* ms, int n_out);

/* ---- inspection (host only; for tests of the host logic) -------------- */
/* Copy a universal table into `out` (host, exactly `count` doubles):
 *   which 0: near-field table of configuration `index` (0..32), n x n, [j][i]
 *              = int_{S_c} log|x_i - y| l_j(y) dy in units of the target side
 *         1: A_{X,G}, |X| x N_G row-major
 *         2: P2M, (p+1) x n complex (re, im) pairs, [k][j]
 *         3: P2L of slot `index` (0..35), (p+1) x n complex, [l][j]
 *         4: M2L of slot `index` (0..48), (p+1) x (p+1) complex, [k][l]
 *         5: M2M of child `index` (0..3), (p+1) x (p+1) complex, [k][l]
 *         6: L2L of child `index` (0..3), (p+1) x (p+1) complex, [k][l]
 *         7: L2P, n x (p+1) complex, [i][l]
 *         8: unit-square quadrature weights, n
 *         9..19 (whole arrays, `index` ignored): the scaled-Pascal translation
 *           operands - 9 C(k+l-1,l) [k][l], 10 t^l and 11 (-t)^k per M2L slot
 *           (49 x (p+1) complex), 12 log|d/h| per M2L slot, 13 C(l-1,k-1),
 *           14 (2w)^-k and 15 w^l per child (4 x (p+1) complex), 16 C(k,l),
 *           17 w^k and 18 (2w)^-l per child, 19 the P2L GEMM operand
 *           (36 x n x rows, rows = 64 ceil(2(p+1)/64))
 *        20: low-rank factor W of near-field configuration `index`, n x 64,
 *            [j][a]; 21: its factor Q, 64 x n, [a][i]; table 0 of the
 *            configuration ~ sum_a Q[a][i] W[j][a] (zero padded beyond the
 *            rank; both zero for configurations applied densely)
 *        22 (`index` ignored): 66 values, the padded rank R (0 = dense) of
 *            each configuration, then its rank
 *        23: M2P (list 3) GEMM operand of slot `index` (0..35; the slot of
 *            a box one level finer than the target leaf, centre offset
 *            (ox, oy) in units of its half side, ((ox+5)/2)*6 + (oy+5)/2),
 *            rows x n, [k][i], rows as for table 19: row 0 log|z|, rows
 *            2k and 2k+1 Re z^-k and -Im z^-k (k >= 1), z = node i of the
 *            leaf minus the box centre in units of the box side
 *        24 (`index` ignored): 82 values describing the symmetry classes of
 *            the target-stationary near field (K = 16): the class (0..6) and
 *            the D4 code g of each of the 33 configurations, the base
 *            configuration and padded rank of each of the 7 classes, 1 if
 *            the path is available (else 0), and max |T_c[g(i)][g(j)] -
 *            T_b[i][j]| / max |T_b| over the configurations.  D4 code bits:
 *            1 swaps the axes, then 2 negates x and 4 negates y; on node
 *            (a, b) of the K x K grid: (A, B) = swapped ? (b, a) : (a, b),
 *            a' = (g & 2) ? K-1-A : A, b' = (g & 4) ? K-1-B : B
 *            (all -1 when K != 16)
 *        25, 27 (K = 16, `index` = configuration): the fixed-point slices
 *            of the mixed-precision kernels (25 int8, five slices; 27
 *            bf16, four slices; as doubles): W slices [s][a][j], 64 W
 *            exponents, Q slices [s][i][a], n Q exponents (64 ranks,
 *            padded); 26, 28 (`index` ignored): the self table's slices
 *            [s][i][j] and its n row exponents
 * VFX_EINVAL if `which`, `index` or `count` does not match. */
int vfx_debug_table(const vfx_ctx* ctx, int which, int index, double* out, int64_t count);
/* Interaction list `which` (1..4) of a plan as CSR arrays (host):
 * lists 1 and 3 are per leaf (ptr has n_leaves+1 entries), lists 2 and 4 per
 * box (n_boxes+1).  src: list 1 and 4 hold leaf indices, 2 and 3 box
 * indices.  cfg: table configuration (list 1: 0..32, list 2: M2L slot,
 * list 4: P2L slot, list 3: 0).  Sizes from vfx_plan_stats_get. */
int vfx_plan_lists(const vfx_plan* plan, int which, int32_t* ptr, int32_t* src, int32_t* cfg);
/* Boxes of a plan (n_boxes entries each): level, position, leaf index or -1. */
int vfx_plan_boxes(const vfx_plan* plan, int32_t* level, int32_t* ix, int32_t* iy, int32_t* leaf);

const char* vfx_last_error(void);
/* Fixed name of a status code ("VFX_OK", "VFX_EINVAL", ...; "unknown status"
 * for any other value).  The returned string is static; never fails. */
const char* vfx_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
