#!/usr/bin/env python3
"""Throughput of the extension + volume FMM path on one MI355X.

A step is one pass of the whole path (cut-leaf extension, P2M/M2M,
M2L/P2L, L2L, near field, far field) over the synthetic wedge workload
(square minus a wedge, K = 16 leaf grids, adaptive level-restricted tree of
ten levels, 3.65e6 leaf nodes, 1536 cut leaves), with every input already
resident in HBM.  The value is leaf points per second in FP64; beside it,
the same path with the mixed-precision near field (five fixed-point int8
slices per operand row on the int8 matrix cores, exact int32 sums, FP64
results) at every level threshold, each checked against the oracle, and the
four-slice bf16 form of the same products for comparison.  Per-phase times come from HIP events recorded by the library on the
execute stream during the timed steps; the roofline object describes the
dominant phase.  The CPU baseline times the oracle (direct quadrature of the
volume potential at a seeded sample of nodes plus its float64 extension of
every cut leaf) on the host's cores and scales it to the whole workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config NAME] [--p P]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "leaf points/s (ext + volume FMM) at 1e-10 rel L∞; mixed vs FP64 on 1 GPU"
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


# phase -> (kernel name as in a kernel trace, marker comment that opens its
# source block in kernels.hip); a phase of several kernels names the one
# that dominates it.  The roofline object describes, among the phases that
# are a single kernel launch (the others hold several launches, and their
# event-timed spans include waits for the other stream), the one with the
# most algorithmic work (the longest time at the roofline): event times of
# kernels that share the GPU with the other stream vary from run to run.
SINGLE_KERNEL_PHASES = ("extension", "down", "near_lowrank", "near_dense", "far", "p2l", "m2p")
PHASE_KERNEL = {
    "extension": ("k_extension", "// Extension of one cut leaf per work-group"),
    "p2m_up": ("k_up", "// Upward pass without the level-by-level chain."),
    "m2l": ("k_m2l_lanes", "// M2L: one lane per list-2 entry"),
    "p2l": ("k_tgemm", "// Table GEMMs with 64-entry tiles"),
    "m2p": ("k_tgemm", "// Table GEMMs with 64-entry tiles"),
    "down": ("k_down", "// Downward pass without the level-by-level chain"),
    "near_lowrank": ("k_near_lr", "// Near field in low-rank form"),
    "near_dense": ("k_tgemm", "// Table GEMMs with 64-entry tiles"),
    "far": ("k_far", "// Far field and the near-field reduction"),
}
# the same phases on the target-stationary path (FP64, K = 16)
PHASE_KERNEL_TS = dict(PHASE_KERNEL, near_lowrank=("k_tgemm", "// Table GEMMs with 64-entry tiles"),
                       near_dense=("k_near_ts", None))


def algorithmic_work(case, precision="fp64"):
    """Algorithmic FP64 flops and HBM bytes of one execute, per phase, with
    the stream each phase runs on.

    Flops count the arithmetic the method needs (a complex multiply-add is 8
    flops; low-rank operators at their true ranks), bytes the compulsory HBM
    traffic (every operand read once, every result written once)."""
    import numpy as np
    plan, ctx = case["plan"], case["ctx"]
    st = plan.stats()
    K = case["K"]
    n = K * K
    P = case["p"] + 1
    L, B = st["n_leaves"], st["n_boxes"]
    N2, N3, N4 = st["n_list2"], st["n_list3"], st["n_list4"]
    nG = 66
    ext_targets, ncut = st["n_ext_targets"], st["n_cut"]
    ptr, src, cfg = plan.lists(1)
    counts = np.bincount(cfg, minlength=33)
    rk = ctx.debug_table(22, 0, 66)
    lrR, rank = rk[:33].astype(int), rk[33:].astype(int)
    # pairs (box, leaf below it) of the direct upward/downward passes
    lev = np.asarray(case["tree"]["level"])
    n_pairs_ud = int(np.maximum(lev - 2, 0).sum())
    nI = case["interior"]
    n_reg = int(np.count_nonzero(np.asarray(case["tree"]["kind"]) == 1))
    work = {
        # the extension (P_i and f_I read, the Sbar grid data, every list
        # target written; ext_targets counts the cut leaves themselves) and,
        # in the same launch, the f^e initialisation of the other leaves
        "extension": (2.0 * nG * nI + ncut * (2 * nG * 144 + 4 * 144 * 12) + ext_targets * (2 * 12 * 12 * K + 2 * 12 * n),
                      8.0 * (nG * nI + nI + ncut * 144) + 8.0 * L * n + 8.0 * n_reg * n, "caller"),
        "p2m_up": (8.0 * P * n * L / 2 + 8.0 * P * P / 2 * n_pairs_ud, 8.0 * L * n + 16.0 * B * P, "caller"),
        # M2L sums the list-4 products of P2L with the list-2 translations
        "m2l": (8.0 * P * P * N2, 16.0 * 2 * B * P + 16.0 * N4 * P, "caller"),
        "p2l": (4.0 * P * n * N4, 8.0 * L * n + 16.0 * N4 * P, "side"),
        "down": (8.0 * P * P / 2 * n_pairs_ud, 16.0 * (B + L) * P, "caller"),
        "m2p": (2.0 * n * 2 * P * N3, 16.0 * N3 * P + 8.0 * n * N3 + 8.0 * 2 * P * n * 20, "side"),
    }
    info = ctx.debug_table(24, 0, 82)
    ts = precision == "fp64" and K == 16 and info[80] == 1.0
    if ts:
        cls = info[:33].astype(int)
        base = info[66:73].astype(int)
        r_cls = np.array([rank[base[cls[c]]] if cls[c] > 0 else 0 for c in range(33)])
        n_self = int(counts[4])
        zr = float((counts * r_cls).sum())  # sum over low-rank pairs of the class rank
        # phase 1, the factor products Z = (W_b P_g^T) f of every non-self
        # pair: each source leaf read once, Z written, the factors once
        work["near_lowrank"] = (2.0 * n * zr, 8.0 * L * n + 8.0 * zr + 8.0 * 32 * n * 64, "side")
        # phase 2 per target group: Q_b Z per pair and the self operator;
        # Z and the self rows read, each leaf's sum written once
        work["near_dense"] = (2.0 * n * zr + 2.0 * n * n * n_self,
                              8.0 * zr + 8.0 * n * n_self + 8.0 * L * n + 8.0 * (n * n + 6 * n * 64), "side")
        # the far-field kernel: M2P values of list 3, the near sums, L2P; V written
        work["far"] = (8.0 * P * n * L + n * N3, 8.0 * n * N3 + 16.0 * L * n + 16.0 * L * P, "caller")
    else:
        lr = lrR > 0
        n_lr, n_dense = int(counts[lr].sum()), int(counts[~lr].sum())
        work["near_lowrank"] = (float((counts * 4.0 * n * rank)[lr].sum()),
                                8.0 * (L * n + n * n_lr) + 8.0 * 2 * n * 64 * int(lr.sum()), "side")
        work["near_dense"] = (2.0 * n * n * n_dense, 8.0 * (L * n + n * n_dense) + 8.0 * n * n * int((~lr).sum()),
                              "side")
        work["far"] = (8.0 * P * n * L + n * (st["n_list1"] + N3),
                       8.0 * n * (st["n_list1"] + N3) + 8.0 * L * n + 16.0 * L * P, "caller")
    return work, ts


def kernel_digest(marker):
    """Digest of a kernel's source: the block of kernels.hip from its opening
    comment to the next separator line, or (marker None) all of near.hip."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2211_14537_amd", "csrc")
    if marker is None:
        return hashlib.sha256(open(os.path.join(csrc, "near.hip")).read().encode()).hexdigest()[:16]
    src = open(os.path.join(csrc, "kernels.hip")).read()
    i = src.find(marker)
    if i < 0:
        return None
    j = src.find("// ------", i + len(marker))
    return hashlib.sha256(src[i:j if j > 0 else len(src)].encode()).hexdigest()[:16]


def load_traffic(kernel, workload, digest, nbytes):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel factor), or
    None if there is none, the kernel source changed since, or the work of a
    launch did (the summary records the algorithmic bytes it was taken at)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("traffic:"):
            for kv in line[len("traffic:"):].split():
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("digest") != digest or float(vals.get("algorithmic_bytes", "nan")) != float(nbytes):
        return None
    return float(vals["bytes_per_launch"])


def oracle_sample(case, ns, seed, calibrate_seconds=None):
    """The oracle's float64 extension of every cut leaf and its direct
    quadrature of V at ns seeded leaf nodes (or, with calibrate_seconds, at
    as many as fit that time budget).  Returns the nodes, the values, the
    extended data and per-leaf records, and the two times."""
    import numpy as np
    from oracle import extension, geometry, volume

    cfg, tr, f_leaf, f_cut = case["cfg"], case["tree"], case["f_leaf"], case["f_cut"]
    K = cfg["K"]
    ot = geometry.Tree(tr["level"], tr["ix"], tr["iy"], cfg["root"])
    t0 = time.perf_counter()
    fe, info = extension.extend(ot, tr["kind"], f_leaf, f_cut, tr["mask"].astype(bool), K, precision="fp64")
    t_ext = time.perf_counter() - t0
    X, Y = ot.leaf_nodes(K)
    rng = np.random.default_rng(seed)
    if calibrate_seconds is not None:
        sel = rng.choice(X.size, 16, replace=False)
        t0 = time.perf_counter()
        volume.potential(ot, fe, K, X.ravel()[sel], Y.ravel()[sel])
        per = (time.perf_counter() - t0) / 16
        ns = int(max(16, min(4096, (calibrate_seconds - t_ext) / max(per, 1e-6))))
    sel2 = rng.choice(X.size, ns, replace=False)
    t0 = time.perf_counter()
    v = volume.potential(ot, fe, K, X.ravel()[sel2], Y.ravel()[sel2])
    t_v = time.perf_counter() - t0
    return sel2, v, fe, info, t_ext, t_v


def cpu_baseline(case, target_seconds=15.0):
    """Oracle timed on a bounded sample of the workload, scaled to it."""
    sel, v, fe, info, t_ext, t_v = oracle_sample(case, 0, 12345, calibrate_seconds=target_seconds)
    ns = sel.size
    N = case["tree"]["level"].size * case["K"] ** 2
    full = t_ext + t_v / ns * N
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": N / full, "unit": "leaf points/s", "cores": cores, "kind": "oracle",
        "sample": f"float64 extension of all {len(info)} cut leaves ({t_ext:.2f} s) + direct quadrature "
                  f"of V at {ns} seeded nodes ({t_v:.2f} s), scaled to {N} nodes "
                  f"(estimated full oracle time {full:.0f} s)",
    }, (sel, v, fe, info)


def accuracy_check(case, fe_gpu, V_gpu, sel, v_o, fe_o, info):
    """Accuracy of the timed plan's own execute against the oracle, at the
    sampled nodes sel:
      g1  V of the timed plan against the oracle's V of the GPU's own f^e
          (the volume FMM alone; the method's FP64 gate is 1e-10);
      g3  V of the timed plan against the oracle's V of the oracle's f^e
          (end to end, extension included);
      extension  the GPU's f^e against the oracle's float64 extension, as
          the worst ratio to the least-squares forward-error bound of two
          float64 routes, 32 u cond(A_I) max|f| (<= 1).
    V_o(fe_gpu) = V_o(fe_o) + V_o(fe_gpu - fe_o); the difference is nonzero
    only on extension targets.  g3 passes within 1e-10 plus the potential
    the allowed f^e differences can carry (|int_B log|x-y| d| <= |d| h^2
    (|log h| + 2) / 2 pi per target leaf of side h <= 1), relative to
    max |V|.  Returns the check record and V_o(fe_gpu)."""
    import numpy as np
    from oracle import extension, geometry, volume
    tr = case["tree"]
    feg = np.asarray(fe_gpu)
    ot = geometry.Tree(tr["level"], tr["ix"], tr["iy"], case["cfg"]["root"])
    d = feg - fe_o
    X, Y = ot.leaf_nodes(case["K"])
    tx, ty = X.ravel()[sel], Y.ravel()[sel]
    v_g = v_o + (volume.potential(ot, d, case["K"], tx, ty) if np.any(d != 0.0) else 0.0)
    Vs = np.asarray(V_gpu).ravel()[sel]
    g1 = float(np.abs(Vs - v_g).max() / np.abs(v_g).max())
    g3 = float(np.abs(Vs - v_o).max() / np.abs(v_o).max())
    worst, bound = 0.0, 0.0
    cut_ids = list(tr["cut_ids"])
    h = ot.h()
    for i, rec in info.items():
        tg = rec["targets"]
        r = cut_ids.index(i)
        f_int = case["f_cut"][r][tr["mask"][r] != 0]
        tol = 2.0 * extension.extension_tolerance(rec, fe_o[tg], f_int)
        worst = max(worst, float(np.abs(feg[tg] - fe_o[tg]).max()) / tol)
        for j in tg:
            bound += tol * h[j] ** 2 * (abs(math.log(h[j])) + 2.0) / (2.0 * math.pi)
    g3_allowed = 1e-10 + bound / float(np.abs(v_o).max())
    rec = {"volume_nodes": int(sel.size), "g1_rel_linf": g1, "g3_rel_linf": g3, "g3_allowed": g3_allowed,
           "extension_worst_error_over_bound": worst, "tolerance": 1e-10,
           "pass": bool(g1 <= 1e-10 and g3 <= g3_allowed and worst <= 1.0),
           "note": "timed plan's V against the oracle: g1 = V_oracle(GPU f^e) within 1e-10; g3 = "
                   "V_oracle(oracle f^e) (end to end) within 1e-10 plus the potential of the allowed f^e "
                   "differences; extension within 32 u cond(A_I) max|f| of the oracle's float64 extension"}
    return rec, v_g


def gpu_plan_stage(case, fl, fc, dev):
    """Plan + execute for one right-hand side with the least-squares
    operators computed on the GPU: host lists (no factorisation), device
    QR/SVD of every cut leaf, one execute."""
    import numpy as np
    import torch
    from paper_2211_14537_amd import vfx
    tr = case["tree"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = vfx.Plan(case["ctx"], tr["level"], tr["ix"], tr["iy"], tr["kind"], tr["mask"], defer_factor=True)
    t1 = time.perf_counter()
    plan.factor_gpu()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fe, V = torch.empty_like(fl), torch.empty_like(fl)
    plan.execute(fl, fc, fe, V)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    # second factorisation (device data already resident): the kernel alone
    plan.factor_gpu()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    return {"host_lists_s": t1 - t0, "gpu_factor_first_s": t2 - t1, "gpu_factor_ms": 1e3 * (t4 - t3),
            "plan_plus_execute_s": t3 - t0, "host_factored_plan_s": case["plan"].stats()["plan_seconds"]}


def bench_batch(args, dev):
    """Many right-hand sides on one tree, one vfx_execute_batch per step."""
    import numpy as np
    import torch
    from paper_2211_14537_amd import tree as T
    from paper_2211_14537_amd import vfx
    from workloads import get_config
    cfg = get_config("starfish_batch")
    nrhs = min(args.batch, len(cfg["rhs"]))
    ctx = vfx.Context(cfg["K"], cfg["p"], root=cfg["root"])
    P = ctx.stencil_points()
    tr = T.build_tree(cfg, P)
    plan = vfx.Plan(ctx, tr["level"], tr["ix"], tr["iy"], tr["kind"], tr["mask"])
    L, n = len(tr["level"]), cfg["K"] ** 2
    FL = torch.empty((nrhs, L, n), dtype=torch.float64, device=dev)
    FC = torch.empty((nrhs, len(tr["cut_ids"]), ctx.n_stencil), dtype=torch.float64, device=dev)
    for r in range(nrhs):
        c = dict(cfg)
        c["fun"] = cfg["rhs"][r]
        fl, fc = T.sample_inputs(c, tr, P)
        FL[r].copy_(torch.from_numpy(fl))
        FC[r].copy_(torch.from_numpy(fc))
    FE, V = torch.empty_like(FL), torch.empty_like(FL)
    choice = plan.autotune(nrhs, FL, FC, FE, V, reps=1) if args.autotune else None
    for _ in range(max(args.warmup, 1)):
        plan.execute_batch(nrhs, FL, FC, FE, V)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute_batch(nrhs, FL, FC, FE, V)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    # the same work one right-hand side at a time (first 8), for reference,
    # into buffers of their own (FE and V keep the batch's results)
    fe1, v1 = torch.empty_like(FL[0]), torch.empty_like(FL[0])
    t0 = time.perf_counter()
    k1 = min(8, nrhs)
    for r in range(k1):
        plan.execute(FL[r], FC[r], fe1, v1)
    torch.cuda.synchronize()
    el1 = (time.perf_counter() - t0) / k1
    # the extension phase (HIP events around it on the execute stream) per
    # right-hand side: in the batch (from 8 right-hand sides on its matrix
    # products run as MFMA GEMMs over the batch) and one at a time
    plan.set_timing(True)
    for _ in range(3):
        plan.execute_batch(nrhs, FL, FC, FE, V)
    torch.cuda.synchronize()
    ph_b = plan.timings()
    plan.set_timing(True)
    for r in range(k1):
        plan.execute(FL[r], FC[r], fe1, v1)
    torch.cuda.synchronize()
    ph_1 = plan.timings()
    plan.set_timing(False)
    ext = {"batch_ms_per_rhs": ph_b["extension"] / nrhs, "single_ms": ph_1["extension"],
           "speedup": ph_1["extension"] * nrhs / max(ph_b["extension"], 1e-12),
           "batch_phases_ms": {k: v for k, v in ph_b.items() if k != "count"}}
    # roofline of the low-rank near-field kernel in the batch: its
    # algorithmic flops for every right-hand side over its event time
    base = dict(cfg=cfg, K=cfg["K"], p=cfg["p"], ctx=ctx, tree=tr, plan=plan,
                interior=int(np.asarray(tr["mask"]).sum()))
    work, _ = algorithmic_work(base, "pairs")
    fl_nl = nrhs * work["near_lowrank"][0]
    t_nl = 1e-3 * ph_b["near_lowrank"]
    roof = {"bound": "mfma", "kernel": "k_near_lr", "phase": "near_lowrank", "achieved": fl_nl / t_nl / 1e12,
            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": fl_nl / t_nl / 1e12 / FP64_PEAK_TFLOPS,
            "traffic": None, "kernel_ms": 1e3 * t_nl, "algorithmic_flops": fl_nl}
    # the first and the last right-hand side against the oracle (as the
    # single-execute check: g1 = V against the oracle's V of the GPU's f^e)
    fe_h, v_h = FE.cpu().numpy(), V.cpu().numpy()
    checks, v_gs = [], {}
    for r in sorted({0, nrhs - 1}):
        c = dict(cfg)
        c["fun"] = cfg["rhs"][r]
        fl_r, fc_r = T.sample_inputs(c, tr, P)
        case_r = dict(base, cfg=c, f_leaf=fl_r, f_cut=fc_r)
        sel, v_o, fe_o, info, _, _ = oracle_sample(case_r, args.check_nodes or 48, 12345 + r)
        rec, v_g = accuracy_check(case_r, fe_h[r], v_h[r], sel, v_o, fe_o, info)
        v_gs[r] = (sel, v_g)
        checks.append(dict(rec, rhs=r))
    # the same batch with the mixed near field (int8 slices) for every level
    # threshold; the reported setting is the widest mixing meeting 1e-10
    rows = []
    for lmin in range(0, int(np.max(tr["level"])) + 1):
        plan.set_precision(2, lmin)
        for _ in range(max(args.warmup, 1)):
            plan.execute_batch(nrhs, FL, FC, FE, V)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.execute_batch(nrhs, FL, FC, FE, V)
        torch.cuda.synchronize()
        elm = (time.perf_counter() - t0) / args.steps
        vm = V.cpu().numpy()
        errm = max(float(np.abs(vm[r].ravel()[sel] - v_g).max() / np.abs(v_g).max()) for r, (sel, v_g) in v_gs.items())
        rows.append({"min_level": lmin, "ms_per_step": 1e3 * elm, "value": nrhs * L * n / elm, "rel_linf": errm})
    plan.set_precision(0)
    ok = [r for r in rows if r["rel_linf"] <= 1e-10]
    best = min(ok, key=lambda r: r["min_level"]) if ok else None
    mixed = {"error_against": "oracle V of the GPU's f^e, first and last right-hand side", "tolerance": 1e-10,
             "sweep": rows}
    if best is not None:
        mixed.update({"setting": f"near field of sources at level >= {best['min_level']} in {MIXED_SETTING[2]}; "
                                 "everything else FP64", "min_level": best["min_level"],
                      "ms_per_step": best["ms_per_step"], "value": best["value"],
                      "speedup_vs_fp64": el / (1e-3 * best["ms_per_step"]), "rel_linf": best["rel_linf"]})
    else:
        mixed.update({"setting": None, "value": None, "note": "no mixed setting meets the tolerance"})
    out = {"metric": "leaf points/s over a batch of right-hand sides (ext + volume FMM), FP64", "unit": "leaf points/s",
           "value": nrhs * L * n / el, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * el, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "starfish_batch", "rhs": nrhs, "leaves": L, "nodes_per_rhs": L * n,
                      "K": cfg["K"], "p": cfg["p"], "cut_leaves": len(tr["cut_ids"])},
           "single_rhs_ms": 1e3 * el1, "batch_speedup_per_rhs": el1 * nrhs / el, "extension": ext,
           "roofline": roof, "check": checks,
           "meets_tolerance": all(c["pass"] for c in checks),
           "mixed": mixed, "autotune": choice}
    print(json.dumps(out), flush=True)


def bench_trees(args, dev):
    """Many uneven trees (random Gaussian sums on the starfish, depth 3-7,
    1e3-1e5 nodes), every execute captured in one HIP graph: one launch."""
    import numpy as np
    import torch
    from paper_2211_14537_amd import tree as T
    from paper_2211_14537_amd import vfx
    from workloads import get_config
    from workloads.configs import batch_functions
    base = get_config("starfish_small")
    ctx = vfx.Context(16, 24, root=base["root"])
    P = ctx.stencil_points()
    rng = np.random.default_rng(21)
    funs = batch_functions(base["domain"], args.trees, seed=22)
    plans, bufs, nodes = [], [], 0
    for i in range(args.trees):
        c = dict(base)
        c["fun"] = funs[i]
        d = int(rng.integers(3, 8))
        c["tree"] = dict(kind="adaptive", tol=float(10 ** rng.uniform(-10, -6)), max_depth=d,
                         min_cut_level=int(rng.integers(min(3, d), d + 1)))
        tr = T.build_tree(c, P)
        L = len(tr["level"])
        if L * 256 > 1e5:
            continue
        fl, fc = T.sample_inputs(c, tr, P)
        plan = vfx.Plan(ctx, tr["level"], tr["ix"], tr["iy"], tr["kind"], tr["mask"])
        FL = torch.tensor(fl, device=dev)
        FC = torch.tensor(fc if fc.size else np.zeros((0, ctx.n_stencil)), device=dev)
        FE, V = torch.empty_like(FL), torch.empty_like(FL)
        plan.execute(FL, FC, FE, V)
        plans.append(plan)
        bufs.append((FL, FC, FE, V))
        nodes += L * 256
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for plan, (FL, FC, FE, V) in zip(plans, bufs):
                plan.execute(FL, FC, FE, V, stream=s)
        s.synchronize()
        el_eager = (time.perf_counter() - t0) / args.steps
        g = vfx.Graph()
        g.begin(s)
        for plan, (FL, FC, FE, V) in zip(plans, bufs):
            plan.execute(FL, FC, FE, V, stream=s)
        g.end(s)
        g.launch(s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.launch(s)
        s.synchronize()
        el_graph = (time.perf_counter() - t0) / args.steps
        g.close()
    out = {"metric": "leaf points/s over many trees in one HIP graph launch (ext + volume FMM), FP64",
           "unit": "leaf points/s", "value": nodes / el_graph, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * el_graph, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "uneven_trees", "trees": len(plans), "nodes": nodes,
                      "nodes_min": int(min(b[0].numel() for b in bufs)), "nodes_max": int(max(b[0].numel() for b in bufs))},
           "eager_ms": 1e3 * el_eager, "graph_speedup": el_eager / el_graph}
    print(json.dumps(out), flush=True)


def build_case(name, p):
    import numpy as np
    from paper_2211_14537_amd import tree as T
    from paper_2211_14537_amd import vfx
    from workloads import get_config

    cfg = get_config(name)
    K = cfg["K"]
    p = p if p is not None else cfg["p"]
    t0 = time.perf_counter()
    ctx = vfx.Context(K, p, root=cfg["root"])
    t_ctx = time.perf_counter() - t0
    P = ctx.stencil_points()
    t0 = time.perf_counter()
    tr = T.build_tree(cfg, P)
    t_tree = time.perf_counter() - t0
    f_leaf, f_cut = T.sample_inputs(cfg, tr, P)
    plan = vfx.Plan(ctx, tr["level"], tr["ix"], tr["iy"], tr["kind"], tr["mask"])
    return dict(cfg=cfg, K=K, p=p, ctx=ctx, tree=tr, f_leaf=f_leaf, f_cut=f_cut, plan=plan,
                t_ctx=t_ctx, t_tree=t_tree, interior=int(np.asarray(tr["mask"]).sum()))


def run_steps(plan, fl, fc, fe, V, stream, steps, warmup):
    """Warm-up executes, then `steps` timed executes back to back; seconds
    per execute."""
    import torch
    for _ in range(max(warmup, 1)):
        plan.execute(fl, fc, fe, V, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(fl, fc, fe, V, stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


MIXED_MODES = {"mixed": 2, "mixed-bf16": 1}
MIXED_SETTING = {
    2: "five fixed-point int8 slices per operand row on the int8 matrix cores (exact int32 sums, FP64 results)",
    1: "four fixed-point bf16 slices per operand row on the bf16 matrix cores (exact FP32 block sums, FP64 results)",
}


def mixed_sweep(case, plan, fl, fc, fe, V, stream, args, V64, sel=None, v_g=None):
    """The near field in mixed precision (int8 slices) for every level
    threshold (sources at level >= min_level mixed; 0 = all), each timed
    like the FP64 path and checked: against the oracle's V of the GPU's f^e
    at the sampled nodes when there is an oracle sample (g1), else against
    the FP64 GPU result.  The reported setting is the widest mixing
    (smallest threshold) whose error meets 1e-10; the bf16-slice form is
    timed and checked at every threshold too, for comparison."""
    import numpy as np
    import torch
    nlev = int(np.max(case["tree"]["level"]))

    def run(mode, lmin):
        plan.set_precision(mode, lmin)
        sec = run_steps(plan, fl, fc, fe, V, stream, args.steps, args.warmup)
        Vm = V.cpu().numpy()
        if v_g is not None:
            err = float(np.abs(Vm.ravel()[sel] - v_g).max() / np.abs(v_g).max())
        else:
            err = float(np.abs(Vm - V64).max() / np.abs(V64).max())
        return {"min_level": lmin, "ms_per_step": 1e3 * sec, "rel_linf": err}

    rows = [run(2, lmin) for lmin in range(0, nlev + 1)]
    rows_bf16 = [run(1, lmin) for lmin in range(0, nlev + 1)]
    plan.set_precision(0)
    torch.cuda.synchronize()
    N = case["tree"]["level"].size * case["K"] ** 2
    ok = [r for r in rows if r["rel_linf"] <= 1e-10]
    best = min(ok, key=lambda r: r["min_level"]) if ok else None
    out = {"error_against": "oracle V of the GPU's f^e at the sampled nodes" if v_g is not None
           else "FP64 GPU path (no oracle sample in this run)",
           "tolerance": 1e-10,
           "sweep": [dict(r, value=N / (1e-3 * r["ms_per_step"])) for r in rows],
           "sweep_bf16_slices": [dict(r, value=N / (1e-3 * r["ms_per_step"])) for r in rows_bf16]}
    if best is not None:
        out.update({"setting": f"near field of sources at level >= {best['min_level']} in {MIXED_SETTING[2]}; "
                               "everything else FP64",
                    "min_level": best["min_level"], "value": N / (1e-3 * best["ms_per_step"]),
                    "ms_per_step": best["ms_per_step"], "rel_linf": best["rel_linf"]})
    else:
        out.update({"setting": None, "value": None, "note": "no mixed setting meets the tolerance"})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="wedge_adaptive")
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--baseline-seconds", type=float, default=15.0)
    ap.add_argument("--precision", choices=("fp64", "mixed", "mixed-bf16"), default="fp64",
                    help="the timed path: FP64, or the near field in fixed-point int8 (mixed) or bf16 "
                         "(mixed-bf16) slices on the matrix cores")
    ap.add_argument("--min-level", type=int, default=0,
                    help="with --precision mixed: sources at this level or finer run mixed")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision sweep beside FP64")
    ap.add_argument("--near-mode", type=int, default=0, choices=(0, 1),
                    help="FP64 near field: 0 pair-based, 1 target-stationary")
    ap.add_argument("--check-nodes", type=int, default=0,
                    help="without the CPU baseline: oracle accuracy check at this many seeded nodes")
    ap.add_argument("--batch", type=int, default=0,
                    help="many right-hand sides on one tree (workload starfish_batch): vfx_execute_batch")
    ap.add_argument("--trees", type=int, default=0,
                    help="many uneven trees (1e3-1e5 nodes) captured in one HIP graph, against eager launches")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the near-field launch parameters before the timed steps")
    ap.add_argument("--launch", default=None,
                    help="near-field launch parameters W,M (work-group cap, dense row tiles) instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs the path on one GPU (one plan per device); --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    if args.batch > 0:
        return bench_batch(args, dev)
    if args.trees > 0:
        return bench_trees(args, dev)
    case = build_case(args.config, args.p)
    plan = case["plan"]
    if args.near_mode:
        plan.set_near_mode(args.near_mode)
    if args.precision != "fp64":
        plan.set_precision(MIXED_MODES[args.precision], args.min_level)
    st = plan.stats()
    fl = torch.tensor(case["f_leaf"], dtype=torch.float64, device=dev)
    fc = torch.tensor(case["f_cut"], dtype=torch.float64, device=dev)
    fe = torch.empty_like(fl)
    V = torch.empty_like(fl)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        plan.execute(fl, fc, fe, V, stream)
    torch.cuda.synchronize()
    if args.launch:
        w_, m_ = (int(v) for v in args.launch.split(","))
        plan.set_launch(w_, m_)
        choice = {"near_wgs": w_, "dense_mtb": m_, "set": True}
    else:
        choice = plan.autotune(1, fl, fc, fe, V, reps=20) if args.autotune else None
    sec = run_steps(plan, fl, fc, fe, V, stream, args.steps, 0)
    fe_t = fe.cpu().numpy()
    V_t = V.cpu().numpy()
    # per-phase times from separate executes with the timing events on (the
    # events themselves cost time, so the timed steps above run without them)
    plan.set_timing(True)
    for _ in range(min(args.steps, 20)):
        plan.execute(fl, fc, fe, V, stream)
    torch.cuda.synchronize()
    phases = plan.timings()
    plan.set_timing(False)
    if args.copy_calibration:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        bcopy = torch.empty_like(a)
        bcopy.copy_(a)
        torch.cuda.synchronize()
        del a, bcopy
    N = st["n_leaves"] * case["K"] ** 2
    value = N / sec

    work, ts = algorithmic_work(case, args.precision if args.near_mode == 1 else "pairs")
    kernels = PHASE_KERNEL_TS if ts else PHASE_KERNEL
    # per-phase rooflines: time at the roofline = the larger of flops at the
    # FP64 peak and bytes at the HBM peak; fraction = that / measured phase
    # time (HIP events on the phase's stream; spans of several kernels
    # include waits).  The step's fraction: the sum of the phase rooflines
    # over the measured step.
    rows = []
    for k, (fl_, by_, stream_) in work.items():
        if args.precision != "fp64" and k in ("near_lowrank", "near_dense"):
            continue  # int8 or bf16 kernels: not an FP64 roofline
        t_roof = max(fl_ / (FP64_PEAK_TFLOPS * 1e12), by_ / (HBM_PEAK_GBS * 1e9))
        ms = phases.get(k)
        rows.append({"phase": k, "kernel": kernels[k][0], "stream": stream_, "flops": fl_, "bytes": by_,
                     "bound": "mfma" if fl_ / (FP64_PEAK_TFLOPS * 1e12) >= by_ / (HBM_PEAK_GBS * 1e9) else "hbm",
                     "ms": ms, "roofline_ms": 1e3 * t_roof, "frac": (1e3 * t_roof / ms) if ms else None,
                     "single_kernel": k in SINGLE_KERNEL_PHASES})
    step_roof = sum(r["roofline_ms"] for r in rows)
    single = [r for r in rows if r["single_kernel"]]
    dom = max(single, key=lambda r: r["roofline_ms"])
    flops, nbytes, ksec = dom["flops"], dom["bytes"], dom["ms"] * 1e-3
    if dom["bound"] == "mfma":
        roof = {"bound": "mfma", "achieved": flops / ksec / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": nbytes / ksec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    kname, marker = kernels[dom["phase"]]
    roof["traffic"] = load_traffic(kname, case["cfg"]["name"], kernel_digest(marker), nbytes)
    roof["kernel"] = kname
    roof["phase"] = dom["phase"]
    roof["kernel_ms"] = dom["ms"]
    roof["algorithmic_flops"] = flops
    roof["algorithmic_bytes"] = nbytes
    roof["roofline_ms"] = dom["roofline_ms"]

    plan_stage = gpu_plan_stage(case, fl, fc, dev)
    out = {
        "metric": METRIC, "value": value, "unit": "leaf points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sec, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f64+i8", "mixed-bf16": "f64+bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": case["cfg"]["name"], "leaves": st["n_leaves"], "nodes": N, "K": case["K"],
                   "p": case["p"], "levels": st["n_levels"], "cut_leaves": st["n_cut"],
                   "ext_targets": st["n_ext_targets"],
                   "precision": "fp64" if args.precision == "fp64" else
                   (f"mixed: near field of sources at level >= {args.min_level} in "
                    f"{MIXED_SETTING[MIXED_MODES[args.precision]]}")},
        "phases_ms": {k: round(v, 4) for k, v in phases.items() if k != "count"},
        "autotune": choice,
        "plan_s": st["plan_seconds"], "tables_s": case["t_ctx"], "plan_stage": plan_stage,
        "roofline": roof,
        "roofline_phases": rows,
        "roofline_step": {"roofline_ms": step_roof, "ms_per_step": 1e3 * sec, "frac": step_roof / (1e3 * sec),
                          "note": "sum over phases of max(flops / 78.6 TFLOP/s, bytes / 8 TB/s), FP64 phases"},
    }
    sel = v_g = None
    if not args.no_cpu_baseline or args.check_nodes > 0:
        if not args.no_cpu_baseline:
            base, (sel, v_o, fe_o, info) = cpu_baseline(case, args.baseline_seconds)
            out["cpu_baseline"] = base
        else:
            sel, v_o, fe_o, info, _, _ = oracle_sample(case, args.check_nodes, 12345)
        out["check"], v_g = accuracy_check(case, fe_t, V_t, sel, v_o, fe_o, info)
        out["meets_tolerance"] = out["check"]["pass"]
    if args.precision == "fp64" and not args.no_mixed:
        out["mixed"] = mixed_sweep(case, plan, fl, fc, fe, V, stream, args, V_t, sel, v_g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
