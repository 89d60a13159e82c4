// C-ABI entry points of the vfx library (declared in include/vfx.h).
#include <cstdint>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

#include "vfx_internal.h"

struct vfx_ctx {
  vfx::Context c;
};
struct vfx_plan {
  vfx::Plan p;
};

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Universal tables depend only on (K, Kbar, deg, p); building them costs
// seconds at K = 16, so they are kept for the life of the process.
std::mutex g_cache_mu;
std::map<std::tuple<int, int, int, int>, std::shared_ptr<const vfx::Tables>> g_cache;

// Live contexts and plans: id -> the generation count of their device
// buffers.  A captured graph records (id, generation) of everything its
// executes used; vfx_graph_launch refuses to replay it once one of them
// has been destroyed or has freed / reallocated those buffers.
std::mutex g_live_mu;
uint64_t g_next_id = 1;
std::unordered_map<uint64_t, const uint64_t*> g_live;

uint64_t register_live(const uint64_t* gen) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  const uint64_t id = g_next_id++;
  g_live[id] = gen;
  return id;
}

void unregister_live(uint64_t id) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.erase(id);
}

// Captures started by vfx_graph_begin: the stream, its capture id, and the
// (id, generation) pairs its executes used.
struct Capture {
  hipStream_t stream = nullptr;
  unsigned long long capture_id = 0;
  std::vector<std::pair<uint64_t, uint64_t>> used;
};
std::mutex g_cap_mu;
std::vector<Capture> g_captures;

// Under stream capture a call is accepted only on the stream vfx_graph_begin
// started the capture on (not on streams forked from it: capturing executes
// there has ended in a crash inside hipStreamEndCapture), and records what
// it uses.  Returns false (with the reason in msg) to refuse.
bool capture_admit(hipStream_t s, const vfx::Context* c, const vfx::Plan* p, std::string& msg) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long cid = 0;
  if (hipStreamGetCaptureInfo(s, &cs, &cid) != hipSuccess) {
    msg = "hipStreamGetCaptureInfo failed";
    return false;
  }
  if (cs != hipStreamCaptureStatusActive) return true;
  std::lock_guard<std::mutex> lk(g_cap_mu);
  for (Capture& k : g_captures) {
    if (k.capture_id != cid) continue;
    if (k.stream != s) break;
    k.used.emplace_back(c->id, c->gen);
    k.used.emplace_back(p->id, p->gen);
    return true;
  }
  msg = "under stream capture, calls must go to the stream vfx_graph_begin started the capture on "
        "(captures on other streams, or on streams forked from it, are not supported)";
  return false;
}

std::shared_ptr<const vfx::Tables> cached_tables(const vfx_params& prm) {
  auto key = std::make_tuple(prm.K, prm.Kbar, prm.deg, prm.p);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) return it->second;
  auto T = std::make_shared<vfx::Tables>();
  T->K = prm.K;
  T->Kbar = prm.Kbar;
  T->deg = prm.deg;
  T->p = prm.p;
  vfx::build_tables(*T);
  g_cache[key] = T;
  return T;
}
}  // namespace

extern "C" {

const char* vfx_last_error(void) { return g_err.c_str(); }

const char* vfx_status_string(int status) {
  switch (status) {
    case VFX_OK: return "VFX_OK";
    case VFX_EINVAL: return "VFX_EINVAL (bad argument)";
    case VFX_ETREE: return "VFX_ETREE (tree not a balanced quad-tree partition, or extension restriction violated)";
    case VFX_EHIP: return "VFX_EHIP (HIP runtime error)";
    case VFX_ENOMEM: return "VFX_ENOMEM (allocation failed)";
    default: return "unknown status";
  }
}

int vfx_create(const vfx_params* prm, vfx_ctx** out) {
  if (!prm || !out) return fail(VFX_EINVAL, "vfx_create: null argument");
  *out = nullptr;
  if (prm->K != 4 && prm->K != 8 && prm->K != 12 && prm->K != 16)
    return fail(VFX_EINVAL, "vfx_create: K must be 4, 8, 12 or 16");
  if (prm->Kbar < 2 || prm->Kbar > 16) return fail(VFX_EINVAL, "vfx_create: Kbar must be in 2..16");
  if (prm->deg < 1 || prm->deg > 15) return fail(VFX_EINVAL, "vfx_create: deg must be in 1..15");
  if (prm->p < 4 || prm->p > 60) return fail(VFX_EINVAL, "vfx_create: p must be in 4..60");
  if (!(prm->root_size > 0)) return fail(VFX_EINVAL, "vfx_create: root_size must be positive");
  try {
    auto T = cached_tables(*prm);
    std::unique_ptr<vfx_ctx> c(new vfx_ctx);
    c->c.T = *T;
    c->c.T.root_cx = prm->root_cx;
    c->c.T.root_cy = prm->root_cy;
    c->c.T.root_size = prm->root_size;
    c->c.id = register_live(&c->c.gen);
    *out = c.release();
    return VFX_OK;
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, "vfx_create: out of host memory");
  } catch (const std::exception& e) {
    return fail(VFX_EINVAL, std::string("vfx_create: ") + e.what());
  }
}

int vfx_destroy(vfx_ctx* ctx) {
  if (!ctx) return VFX_OK;
  unregister_live(ctx->c.id);
  vfx::free_tables_device(&ctx->c);
  delete ctx;
  return VFX_OK;
}

int vfx_stencil_size(const vfx_ctx* ctx, int32_t* nX, int32_t* nG) {
  if (!ctx || !nX || !nG) return fail(VFX_EINVAL, "vfx_stencil_size: null argument");
  *nX = ctx->c.T.nX;
  *nG = ctx->c.T.nG;
  return VFX_OK;
}

int vfx_stencil_points(const vfx_ctx* ctx, double* xy) {
  if (!ctx || !xy) return fail(VFX_EINVAL, "vfx_stencil_points: null argument");
  std::memcpy(xy, ctx->c.T.stencil_xy.data(), sizeof(double) * ctx->c.T.stencil_xy.size());
  return VFX_OK;
}

int vfx_leaf_nodes(const vfx_ctx* ctx, double* t) {
  if (!ctx || !t) return fail(VFX_EINVAL, "vfx_leaf_nodes: null argument");
  std::memcpy(t, ctx->c.T.t.data(), sizeof(double) * ctx->c.T.t.size());
  return VFX_OK;
}

static int plan_create(vfx_ctx* ctx, const vfx_tree* tree, int flags, vfx_plan** out, const char* who) {
  if (!ctx || !tree || !out) return fail(VFX_EINVAL, std::string(who) + ": null argument");
  if (flags & ~VFX_PLAN_DEFER_FACTOR) return fail(VFX_EINVAL, std::string(who) + ": unknown flags");
  *out = nullptr;
  try {
    std::unique_ptr<vfx_plan> p(new vfx_plan);
    p->p.ctx = &ctx->c;
    std::string err;
    int rc = vfx::build_host_plan(ctx->c.T, tree, p->p.H, err, (flags & VFX_PLAN_DEFER_FACTOR) != 0);
    if (rc) return fail(rc, std::string(who) + ": " + err);
    p->p.id = register_live(&p->p.gen);
    *out = p.release();
    return VFX_OK;
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, std::string(who) + ": out of host memory");
  }
}

int vfx_plan_create(vfx_ctx* ctx, const vfx_tree* tree, vfx_plan** out) {
  return plan_create(ctx, tree, 0, out, "vfx_plan_create");
}

int vfx_plan_create_ex(vfx_ctx* ctx, const vfx_tree* tree, int flags, vfx_plan** out) {
  return plan_create(ctx, tree, flags, out, "vfx_plan_create_ex");
}

int vfx_plan_factor_gpu(vfx_plan* plan, void* stream) {
  if (!plan) return fail(VFX_EINVAL, "vfx_plan_factor_gpu: null argument");
  vfx::Plan& p = plan->p;
  try {
    std::string err;
    int rc = VFX_OK;
    if (!p.ctx->D.ready) rc = vfx::upload_tables(p.ctx, err);
    if (!rc && !p.D.ready) rc = vfx::upload_plan(&p, err);
    if (!rc) rc = vfx::factor_gpu(&p, (hipStream_t)stream, err);
    if (rc) return fail(rc, "vfx_plan_factor_gpu: " + err);
    return VFX_OK;
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, "vfx_plan_factor_gpu: out of host memory");
  }
}

int vfx_plan_destroy(vfx_plan* plan) {
  if (!plan) return VFX_OK;
  unregister_live(plan->p.id);
  vfx::free_plan_device(&plan->p);
  delete plan;
  return VFX_OK;
}

int vfx_plan_stats_get(const vfx_plan* plan, vfx_plan_stats* o) {
  if (!plan || !o) return fail(VFX_EINVAL, "vfx_plan_stats_get: null argument");
  const vfx::HostPlan& H = plan->p.H;
  o->n_leaves = H.L;
  o->n_boxes = H.B;
  o->n_levels = H.nlev;
  o->n_cut = H.ncut;
  o->n_ext_targets = (int32_t)H.ext_tgt.size();
  o->n_list1 = (int64_t)H.l1_src.size();
  o->n_list2 = (int64_t)H.l2_src.size();
  o->n_list3 = (int64_t)H.l3_src.size();
  o->n_list4 = (int64_t)H.l4_src.size();
  o->pinv_doubles = (int64_t)H.pinv_val.size();
  o->plan_seconds = H.plan_seconds;
  return VFX_OK;
}

int vfx_plan_ext_owner(const vfx_plan* plan, int32_t* owner) {
  if (!plan || !owner) return fail(VFX_EINVAL, "vfx_plan_ext_owner: null argument");
  const vfx::HostPlan& H = plan->p.H;
  for (int i = 0; i < H.L; ++i) owner[i] = H.owner[i];
  return VFX_OK;
}

static int execute_checked(vfx_plan* plan, int nrhs, const double* f_leaf, const double* f_cut, double* fe_out,
                           double* V_out, void* stream, const char* who) {
  if (!plan || !f_leaf || !fe_out || !V_out || nrhs < 1)
    return fail(VFX_EINVAL, std::string(who) + ": null argument or nrhs < 1");
  if (reinterpret_cast<uintptr_t>(fe_out) % 16 || reinterpret_cast<uintptr_t>(f_leaf) % 16 ||
      reinterpret_cast<uintptr_t>(V_out) % 16)
    return fail(VFX_EINVAL, std::string(who) + ": f_leaf, fe_out and V_out must be 16-byte aligned");
  if (plan->p.H.ncut > 0 && !f_cut)
    return fail(VFX_EINVAL, std::string(who) + ": f_cut is null but the tree has cut leaves");
  vfx::Plan& p = plan->p;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive) {
    // no allocation or upload may be captured, and timing events neither
    if (!p.ctx->D.ready || !p.D.ready || nrhs > p.D.cap)
      return fail(VFX_EINVAL, std::string(who) + ": under stream capture the plan must already hold device data "
                                                 "for this many right-hand sides (execute it once before capturing)");
    if (p.timing) return fail(VFX_EINVAL, std::string(who) + ": timing must be off under stream capture");
    std::string msg;
    if (!capture_admit((hipStream_t)stream, p.ctx, &p, msg)) return fail(VFX_EINVAL, std::string(who) + ": " + msg);
  }
  try {
    std::string err;
    int rc = vfx::launch_execute(&p, nrhs, f_leaf, f_cut, fe_out, V_out, (hipStream_t)stream, err);
    if (rc) return fail(rc, std::string(who) + ": " + err);
    return VFX_OK;
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, std::string(who) + ": out of host memory");
  }
}

int vfx_execute(vfx_plan* plan, const double* f_leaf, const double* f_cut, double* fe_out, double* V_out,
                void* stream) {
  return execute_checked(plan, 1, f_leaf, f_cut, fe_out, V_out, stream, "vfx_execute");
}

int vfx_execute_batch(vfx_plan* plan, int nrhs, const double* f_leaf, const double* f_cut, double* fe_out,
                      double* V_out, void* stream) {
  return execute_checked(plan, nrhs, f_leaf, f_cut, fe_out, V_out, stream, "vfx_execute_batch");
}

int vfx_plan_autotune(vfx_plan* plan, int nrhs, const double* f_leaf, const double* f_cut, double* fe_out,
                      double* V_out, void* stream, int reps, int32_t* choice) {
  if (!plan || reps < 1) return fail(VFX_EINVAL, "vfx_plan_autotune: bad argument");
  vfx::Plan& p = plan->p;
  const bool was_timing = p.timing;
  p.timing = false;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(VFX_EHIP, "vfx_plan_autotune: hipEventCreate failed");
  const int wgs[] = {256, 512, 768, 1024};
  const int mtbs[] = {4, 8};
  const int n_mtb = p.ctx->T.n == 256 ? 2 : 1;
  float best = 1e30f;
  vfx::Plan::Tune bt = p.tune;
  int rc = VFX_OK;
  for (int a = 0; a < 4 && rc == VFX_OK; ++a)
    for (int b = 0; b < n_mtb && rc == VFX_OK; ++b) {
      p.tune.near_wgs = wgs[a];
      p.tune.dense_mtb = mtbs[b];
      rc = execute_checked(plan, nrhs, f_leaf, f_cut, fe_out, V_out, stream, "vfx_plan_autotune");  // warm-up
      if (rc) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && rc == VFX_OK; ++r)
        rc = execute_checked(plan, nrhs, f_leaf, f_cut, fe_out, V_out, stream, "vfx_plan_autotune");
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) rc = fail(VFX_EHIP, "vfx_plan_autotune: event wait failed");
      float ms = 0;
      if (rc == VFX_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best) {
        best = ms;
        bt = p.tune;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p.tune = bt;
  p.timing = was_timing;
  if (choice) {
    choice[0] = bt.near_wgs;
    choice[1] = bt.dense_mtb;
  }
  return rc;
}

int vfx_plan_set_launch(vfx_plan* plan, int near_wgs, int dense_mtb) {
  if (!plan || near_wgs < 1 || near_wgs > 65535 || (dense_mtb != 4 && dense_mtb != 8))
    return fail(VFX_EINVAL, "vfx_plan_set_launch: near_wgs must be in 1..65535 and dense_mtb 4 or 8");
  plan->p.tune.near_wgs = near_wgs;
  plan->p.tune.dense_mtb = dense_mtb;
  return VFX_OK;
}

struct vfx_graph {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  std::vector<std::pair<uint64_t, uint64_t>> used;  // (id, generation) of the contexts and plans
};

int vfx_graph_begin(void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return fail(VFX_EHIP, std::string("vfx_graph_begin: ") + hipGetErrorString(e));
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long cid = 0;
  e = hipStreamGetCaptureInfo(s, &cs, &cid);
  if (e != hipSuccess) {
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    return fail(VFX_EHIP, std::string("vfx_graph_begin: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_cap_mu);
  Capture k;
  k.stream = s;
  k.capture_id = cid;
  g_captures.push_back(std::move(k));
  return VFX_OK;
}

int vfx_graph_end(void* stream, vfx_graph** out) {
  if (!out) return fail(VFX_EINVAL, "vfx_graph_end: null argument");
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<vfx_graph> g(new vfx_graph);
  {
    std::lock_guard<std::mutex> lk(g_cap_mu);
    for (size_t i = 0; i < g_captures.size(); ++i)
      if (g_captures[i].stream == s) {
        g->used = std::move(g_captures[i].used);
        g_captures.erase(g_captures.begin() + i);
        break;
      }
  }
  hipError_t e = hipStreamEndCapture(s, &g->g);
  if (e != hipSuccess) return fail(VFX_EHIP, std::string("vfx_graph_end: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&g->e, g->g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g->g);
    return fail(VFX_EHIP, std::string("vfx_graph_end: instantiate: ") + hipGetErrorString(e));
  }
  *out = g.release();
  return VFX_OK;
}

int vfx_graph_launch(vfx_graph* g, void* stream) {
  if (!g) return fail(VFX_EINVAL, "vfx_graph_launch: null graph");
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    for (const auto& u : g->used) {
      auto it = g_live.find(u.first);
      if (it == g_live.end() || *it->second != u.second)
        return fail(VFX_EINVAL, "vfx_graph_launch: a context or plan captured in this graph has since been "
                                "destroyed or has freed / reallocated its device buffers; capture again");
    }
  }
  hipError_t e = hipGraphLaunch(g->e, (hipStream_t)stream);
  return e == hipSuccess ? VFX_OK : fail(VFX_EHIP, std::string("vfx_graph_launch: ") + hipGetErrorString(e));
}

int vfx_graph_destroy(vfx_graph* g) {
  if (!g) return VFX_OK;
  if (g->e) (void)hipGraphExecDestroy(g->e);
  if (g->g) (void)hipGraphDestroy(g->g);
  delete g;
  return VFX_OK;
}

int vfx_plan_set_precision(vfx_plan* plan, int mode, int min_level) {
  if (!plan || mode < 0 || mode > 2) return fail(VFX_EINVAL, "vfx_plan_set_precision: mode must be 0, 1 or 2");
  vfx::Plan& p = plan->p;
  try {
    std::string err;
    int rc = vfx::build_near_tiles(p.ctx->T, p.H, mode, mode >= 1 ? min_level : 0, err);
    if (rc) {
      vfx::build_near_tiles(p.ctx->T, p.H, 0, 0, err);
      return fail(rc, "vfx_plan_set_precision: " + err);
    }
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, "vfx_plan_set_precision: out of host memory");
  }
  vfx::free_plan_device(&p);  // re-uploaded by the next execute
  return VFX_OK;
}

int vfx_plan_set_near_mode(vfx_plan* plan, int mode) {
  if (!plan || (mode != 0 && mode != 1)) return fail(VFX_EINVAL, "vfx_plan_set_near_mode: mode must be 0 or 1");
  vfx::Plan& p = plan->p;
  try {
    std::string err;
    p.H.near_mode = mode;
    int rc = vfx::build_near_tiles(p.ctx->T, p.H, p.H.precision, p.H.mixed_min_level, err);
    if (rc) return fail(rc, "vfx_plan_set_near_mode: " + err);
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, "vfx_plan_set_near_mode: out of host memory");
  }
  vfx::free_plan_device(&p);  // re-uploaded by the next execute
  return VFX_OK;
}

int vfx_interp(vfx_plan* plan, const double* V, int64_t npts, const double* px, const double* py, double* out,
               void* stream) {
  if (!plan || npts < 0 || (npts > 0 && (!V || !px || !py || !out)))
    return fail(VFX_EINVAL, "vfx_interp: null argument or negative count");
  try {
    std::string err;
    int rc = vfx::launch_interp(&plan->p, V, (long)npts, px, py, out, (hipStream_t)stream, err);
    if (rc) return fail(rc, "vfx_interp: " + err);
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, "vfx_interp: out of host memory");
  }
  return VFX_OK;
}

int vfx_net_charge(vfx_plan* plan, const double* fe, int nrhs, double* out, void* stream) {
  if (!plan || !fe || !out || nrhs < 1) return fail(VFX_EINVAL, "vfx_net_charge: null argument or nrhs < 1");
  vfx::Plan& p = plan->p;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive) {
    if (!p.ctx->D.ready || !p.D.ready || nrhs > p.D.chg_cap)
      return fail(VFX_EINVAL, "vfx_net_charge: under stream capture the plan must already hold device data for "
                              "this many right-hand sides (call it once before capturing)");
    std::string msg;
    if (!capture_admit((hipStream_t)stream, p.ctx, &p, msg)) return fail(VFX_EINVAL, "vfx_net_charge: " + msg);
  }
  try {
    std::string err;
    int rc = vfx::launch_net_charge(&p, fe, nrhs, out, (hipStream_t)stream, err);
    if (rc) return fail(rc, "vfx_net_charge: " + err);
  } catch (const std::bad_alloc&) {
    return fail(VFX_ENOMEM, "vfx_net_charge: out of host memory");
  }
  return VFX_OK;
}

int vfx_net_charge_noalloc(vfx_plan* plan, const double* fe, int nrhs, double* out, void* stream) {
  if (!plan || !fe || !out || nrhs < 1)
    return fail(VFX_EINVAL, "vfx_net_charge_noalloc: null argument or nrhs < 1");
  vfx::Plan& p = plan->p;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive) {
    std::string msg;
    if (!capture_admit((hipStream_t)stream, p.ctx, &p, msg))
      return fail(VFX_EINVAL, "vfx_net_charge_noalloc: " + msg);
  }
  std::string err;
  int rc = vfx::launch_net_charge_noalloc(&p, fe, nrhs, out, (hipStream_t)stream, err);
  if (rc) return fail(rc, "vfx_net_charge_noalloc: " + err);
  return VFX_OK;
}

int vfx_net_charge_noalloc_max_rhs(void) { return vfx::noalloc_max_rhs(); }

int vfx_mlp_param_count(void) { return vfx::mlp_param_count(); }

int64_t vfx_mlp_grad_work(int64_t batch) { return batch > 0 ? (int64_t)vfx::mlp_grad_work((long)batch) : 0; }

int vfx_mlp_forward(const float* theta, const float* x, int64_t batch, float* logits, void* stream) {
  if (batch < 0 || (batch > 0 && (!theta || !x || !logits))) return fail(VFX_EINVAL, "vfx_mlp_forward: bad argument");
  int rc = vfx::mlp_forward(theta, x, (long)batch, logits, (hipStream_t)stream);
  return rc ? fail(rc, "vfx_mlp_forward: launch failed") : VFX_OK;
}

int vfx_mlp_grad(const float* theta, const float* x, const float* y, int64_t batch, float* grad, float* work,
                 int64_t work_floats, void* stream) {
  if (batch <= 0 || !theta || !x || !y || !grad || !work) return fail(VFX_EINVAL, "vfx_mlp_grad: bad argument");
  if (work_floats < (int64_t)vfx::mlp_grad_work((long)batch)) return fail(VFX_EINVAL, "vfx_mlp_grad: work too small");
  int rc = vfx::mlp_grad(theta, x, y, (long)batch, grad, work, (hipStream_t)stream);
  return rc ? fail(rc, "vfx_mlp_grad: launch failed") : VFX_OK;
}

int vfx_mlp_adam(float* theta, const float* grad, float* m, float* v, int step, float lr, float beta1, float beta2,
                 float eps, void* stream) {
  if (!theta || !grad || !m || !v || step < 1) return fail(VFX_EINVAL, "vfx_mlp_adam: bad argument");
  int rc = vfx::mlp_adam(theta, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
  return rc ? fail(rc, "vfx_mlp_adam: launch failed") : VFX_OK;
}

int vfx_f32_to_f16(const float* a, uint16_t* h, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!a || !h))) return fail(VFX_EINVAL, "vfx_f32_to_f16: bad argument");
  int rc = vfx::mlp_to_f16(a, h, (long)n, (hipStream_t)stream);
  return rc ? fail(rc, "vfx_f32_to_f16: launch failed") : VFX_OK;
}

int vfx_mlp_infer_f16(const uint16_t* theta_h, const uint16_t* x_h, int64_t batch, float* logits, void* stream) {
  if (batch < 0 || (batch > 0 && (!theta_h || !x_h || !logits)))
    return fail(VFX_EINVAL, "vfx_mlp_infer_f16: bad argument");
  int rc = vfx::mlp_infer_f16(theta_h, x_h, (long)batch, logits, (hipStream_t)stream);
  return rc ? fail(rc, "vfx_mlp_infer_f16: launch failed") : VFX_OK;
}

int vfx_plan_set_timing(vfx_plan* plan, int enable) {
  if (!plan) return fail(VFX_EINVAL, "vfx_plan_set_timing: null argument");
  plan->p.timing = enable != 0;
  plan->p.n_timed = 0;
  return VFX_OK;
}

int vfx_plan_timings(vfx_plan* plan, double* ms, int n_out) {
  constexpr int NP = 11;  // phases
  if (!plan || !ms || n_out < NP) return fail(VFX_EINVAL, "vfx_plan_timings: bad argument");
  vfx::Plan& p = plan->p;
  constexpr int NE = vfx::Plan::kEvents;
  if (p.n_timed == 0) return fail(VFX_EINVAL, "vfx_plan_timings: no timed execute recorded");
  hipError_t e = hipEventSynchronize(p.ev[(size_t)(p.n_timed - 1) * NE + 9]);
  if (e != hipSuccess) return fail(VFX_EHIP, std::string("vfx_plan_timings: ") + hipGetErrorString(e));
  // phase k runs from event a[k] to event b[k]
  static const int a_[NP] = {12, 1, 2, 3, 5, 6, 8, 0, 10, 13, 0};
  static const int b_[NP] = {1, 2, 3, 4, 6, 7, 9, 9, 5, 11, 12};
  double acc[NP] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = 0; r < p.n_timed; ++r) {
    const hipEvent_t* ev = &p.ev[(size_t)r * NE];
    for (int k = 0; k < NP; ++k) {
      float t = 0;
      e = hipEventElapsedTime(&t, ev[a_[k]], ev[b_[k]]);
      if (e != hipSuccess) return fail(VFX_EHIP, std::string("vfx_plan_timings: ") + hipGetErrorString(e));
      acc[k] += t;
    }
  }
  for (int k = 0; k < NP; ++k) ms[k] = acc[k] / p.n_timed;
  if (n_out > NP) ms[NP] = p.n_timed;
  return VFX_OK;
}

int vfx_debug_table(const vfx_ctx* ctx, int which, int index, double* out, int64_t count) {
  if (!ctx || !out) return fail(VFX_EINVAL, "vfx_debug_table: null argument");
  const vfx::Tables& T = ctx->c.T;
  const int64_t n = T.n, P = T.p + 1;
  const double* src = nullptr;
  int64_t size = 0;
  switch (which) {
    case 0:
      if (index < 0 || index >= vfx::kNearConfigs) break;
      src = T.near.data() + (size_t)index * n * n;
      size = n * n;
      break;
    case 1:
      src = T.A.data();
      size = (int64_t)T.A.size();
      break;
    case 2:
      src = T.p2m.data();
      size = (int64_t)T.p2m.size();
      break;
    case 3:
      if (index < 0 || index >= vfx::kP2LSlots) break;
      src = T.p2l.data() + (size_t)index * P * n * 2;
      size = P * n * 2;
      break;
    case 4:
      if (index < 0 || index >= vfx::kM2LSlots) break;
      src = T.m2l.data() + (size_t)index * P * P * 2;
      size = P * P * 2;
      break;
    case 5:
    case 6:
      if (index < 0 || index >= 4) break;
      src = (which == 5 ? T.m2m : T.l2l).data() + (size_t)index * P * P * 2;
      size = P * P * 2;
      break;
    case 7:
      src = T.l2p.data();
      size = (int64_t)T.l2p.size();
      break;
    case 8:
      src = T.w2.data();
      size = (int64_t)T.w2.size();
      break;
    case 20:
    case 21:
      if (index < 0 || index >= vfx::kNearConfigs) break;
      src = (which == 20 ? T.lr_W : T.lr_Q).data() + (size_t)index * n * vfx::kNearLrMax;
      size = n * vfx::kNearLrMax;
      break;
    case 22: {
      static thread_local std::vector<double> rk;
      rk.assign(2 * vfx::kNearConfigs, 0.0);
      for (int c = 0; c < vfx::kNearConfigs; ++c) {
        rk[c] = T.lr_R[c];
        rk[vfx::kNearConfigs + c] = T.lr_rank[c];
      }
      src = rk.data();
      size = (int64_t)rk.size();
      break;
    }
    case 24: {
      static thread_local std::vector<double> v;
      v.clear();
      if (T.near_cls.size() == (size_t)vfx::kNearConfigs) {
        for (int c = 0; c < vfx::kNearConfigs; ++c) v.push_back(T.near_cls[c]);
        for (int c = 0; c < vfx::kNearConfigs; ++c) v.push_back(T.near_g[c]);
        for (int k = 0; k < vfx::kNearClasses; ++k) v.push_back(T.cls_base[k]);
        for (int k = 0; k < vfx::kNearClasses; ++k) v.push_back(T.cls_R[k]);
      } else {
        v.assign(2 * vfx::kNearConfigs + 2 * vfx::kNearClasses, -1.0);
      }
      v.push_back(T.ts_ok ? 1.0 : 0.0);
      v.push_back(T.ts_sym_err);
      src = v.data();
      size = (int64_t)v.size();
      break;
    }
    case 25:
    case 26:
    case 27:
    case 28: {
      // fixed-point slices of the near-field operators as doubles: 25/27 the
      // low-rank factors of configuration `index` (W slices [s][a][j], W
      // exponents [a], Q slices [s][i][a], Q exponents [i]), 26/28 the self
      // table (slices [s][i][j], exponents [i]); 25/26 int8, 27/28 bf16
      static thread_local std::vector<double> v;
      v.clear();
      const bool i8 = which == 25 || which == 26, self = which == 26 || which == 28;
      const int ns = i8 ? vfx::kF8Slices : 4;
      if (T.f8_W.empty() || (!self && (index < 0 || index >= vfx::kNearConfigs))) break;
      auto bf = [](uint16_t h) {
        const uint32_t u = (uint32_t)h << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return (double)f;
      };
      const size_t SW = (size_t)vfx::kNearLrMax * n;
      if (self) {
        for (size_t k = 0; k < (size_t)ns * n * n; ++k) v.push_back(i8 ? (double)T.f8_A[k] : bf(T.fx_A[k]));
        for (int64_t i = 0; i < n; ++i) v.push_back(i8 ? T.f8_Aexp[i] : T.fx_Aexp[i]);
      } else {
        const size_t c = (size_t)index;
        for (size_t k = 0; k < (size_t)ns * SW; ++k)
          v.push_back(i8 ? (double)T.f8_W[c * ns * SW + k] : bf(T.fx_W[c * ns * SW + k]));
        for (int a = 0; a < vfx::kNearLrMax; ++a)
          v.push_back(i8 ? T.f8_Wexp[c * vfx::kNearLrMax + a] : T.fx_Wexp[c * vfx::kNearLrMax + a]);
        for (size_t k = 0; k < (size_t)ns * SW; ++k)
          v.push_back(i8 ? (double)T.f8_Q[c * ns * SW + k] : bf(T.fx_Q[c * ns * SW + k]));
        for (int64_t i = 0; i < n; ++i) v.push_back(i8 ? T.f8_Qexp[c * n + i] : T.fx_Qexp[c * n + i]);
      }
      src = v.data();
      size = (int64_t)v.size();
      break;
    }
    case 23:
      if (index < 0 || index >= vfx::kP2LSlots) break;
      src = T.m2p_gemm.data() + (size_t)index * T.p2l_rows * n;
      size = (int64_t)T.p2l_rows * n;
      break;
    case 9: case 10: case 11: case 12: case 13: case 14: case 15: case 16: case 17: case 18: case 19: {
      const std::vector<double>* v[] = {&T.pas_m2l, &T.m2l_tpow, &T.m2l_tneg, &T.m2l_logd, &T.pas_m2m,
                                        &T.m2m_in,  &T.m2m_out,  &T.pas_l2l,  &T.l2l_in,   &T.l2l_out,
                                        &T.p2l_gemm};
      src = v[which - 9]->data();
      size = (int64_t)v[which - 9]->size();
      break;
    }
    default:
      break;
  }
  if (!src || size != count) return fail(VFX_EINVAL, "vfx_debug_table: bad table, index or count");
  std::memcpy(out, src, sizeof(double) * size);
  return VFX_OK;
}

int vfx_plan_lists(const vfx_plan* plan, int which, int32_t* ptr, int32_t* src, int32_t* cfg) {
  if (!plan || !ptr || !src || !cfg) return fail(VFX_EINVAL, "vfx_plan_lists: null argument");
  const vfx::HostPlan& H = plan->p.H;
  const std::vector<int>*P = nullptr, *S = nullptr, *C = nullptr;
  switch (which) {
    case 1: P = &H.l1_ptr; S = &H.l1_src; C = &H.l1_cfg; break;
    case 2: P = &H.l2_ptr; S = &H.l2_src; C = &H.l2_off; break;
    case 3: P = &H.l3_ptr; S = &H.l3_src; break;
    case 4: P = &H.l4_ptr; S = &H.l4_src; C = &H.l4_cfg; break;
    default: return fail(VFX_EINVAL, "vfx_plan_lists: which must be 1..4");
  }
  for (size_t i = 0; i < P->size(); ++i) ptr[i] = (*P)[i];
  for (size_t i = 0; i < S->size(); ++i) {
    src[i] = (*S)[i];
    cfg[i] = C ? (*C)[i] : 0;
  }
  return VFX_OK;
}

int vfx_plan_boxes(const vfx_plan* plan, int32_t* level, int32_t* ix, int32_t* iy, int32_t* leaf) {
  if (!plan || !level || !ix || !iy || !leaf) return fail(VFX_EINVAL, "vfx_plan_boxes: null argument");
  const vfx::HostPlan& H = plan->p.H;
  for (int b = 0; b < H.B; ++b) {
    level[b] = H.box_level[b];
    ix[b] = H.box_ix[b];
    iy[b] = H.box_iy[b];
    leaf[b] = H.box_leaf[b];
  }
  return VFX_OK;
}

}  // extern "C"
