#!/usr/bin/env python3
"""Throughput of the extension + volume FMM path on one MI355X.

A step is one pass of the whole path (cut-leaf extension, P2M/M2M,
M2L/P2L, L2L, near field, far field) over the synthetic starfish workload
(K = 16 leaf grids, adaptive level-restricted tree, about 1.08e6 leaf nodes),
with every input already resident in HBM.  The value is leaf points per
second.  Per-phase times come from HIP events recorded by the library on the
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


def algorithmic_work(stats, K, p, nX_total_interior):
    """Algorithmic flops and HBM bytes per launch of each phase (FP64)."""
    n = K * K
    P = p + 1
    L = stats["n_leaves"]
    B = stats["n_boxes"]
    N1, N2, N3, N4 = stats["n_list1"], stats["n_list2"], stats["n_list3"], stats["n_list4"]
    nG = 66
    ext_targets = stats["n_ext_targets"]
    ncut = stats["n_cut"]
    work = {
        # per pair: n x n table times n values (2 n^2 flops); the leaf data is
        # read once and V written once; the 33 tables are read once
        "near": (2.0 * n * n * N1, 8.0 * (2 * L * n + 33 * n * n)),
        # P_i (nG x N_I) streamed once, plus the gathered interior samples,
        # f_leaf read / f^e written for every leaf, and the list targets
        "extension": (2.0 * nG * nX_total_interior + ncut * (2 * nG * 144 + 4 * 144 * 12)
                      + ext_targets * (2 * 12 * 12 * K + 2 * 12 * n),
                      8.0 * (nG * nX_total_interior + nX_total_interior + 2 * L * n + ext_targets * n)),
        "p2m_m2m": (8.0 * P * n * L + 8.0 * P * P * 4 * (B - L) / 2, 8.0 * (L * n + 2 * B * P)),
        "m2l_p2l": (8.0 * P * P * N2 + 8.0 * P * n * N4, 16.0 * 2 * B * P),
        "l2l": (4.0 * P * P * B, 16.0 * 2 * B * P),
        "far": (8.0 * P * n * L + 8.0 * P * n * N3, 8.0 * 2 * L * n + 16.0 * B * P),
    }
    return work


def cpu_baseline(case, target_seconds=15.0):
    """Oracle timed on a bounded sample of the workload, scaled to it."""
    import numpy as np
    from oracle import extension, geometry, volume

    cfg, tr, f_leaf, f_cut = case["cfg"], case["tree"], case["f_leaf"], case["f_cut"]
    K = cfg["K"]
    ot = geometry.Tree(tr["level"], tr["ix"], tr["iy"], cfg["root"])
    t0 = time.perf_counter()
    fe, info = extension.extend(ot, tr["kind"], f_leaf, f_cut, tr["mask"].astype(bool), K, precision="fp64")
    t_ext = time.perf_counter() - t0
    X, Y = ot.leaf_nodes(K)
    rng = np.random.default_rng(12345)
    # calibrate, then size the sample to the time budget
    sel = rng.choice(X.size, 16, replace=False)
    t0 = time.perf_counter()
    v16 = volume.potential(ot, fe, K, X.ravel()[sel], Y.ravel()[sel])
    per = (time.perf_counter() - t0) / 16
    ns = int(max(16, min(4096, (target_seconds - t_ext) / max(per, 1e-6))))
    sel2 = rng.choice(X.size, ns, replace=False)
    t0 = time.perf_counter()
    v = volume.potential(ot, fe, K, X.ravel()[sel2], Y.ravel()[sel2])
    t_v = (time.perf_counter() - t0) / ns
    N = X.size
    full = t_ext + t_v * N
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": N / full, "unit": "leaf points/s", "cores": cores, "kind": "oracle",
        "sample": f"float64 extension of all {len(info)} cut leaves ({t_ext:.2f} s) + direct quadrature "
                  f"of V at {ns} seeded nodes ({t_v * ns:.2f} s), scaled to {N} nodes "
                  f"(estimated full oracle time {full:.0f} s)",
    }, (sel2, v, fe)


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="starfish_adaptive")
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--baseline-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs the path on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    case = build_case(args.config, args.p)
    plan = case["plan"]
    st = plan.stats()
    fl = torch.tensor(case["f_leaf"], dtype=torch.float64, device=dev)
    fc = torch.tensor(case["f_cut"], dtype=torch.float64, device=dev)
    fe = torch.empty_like(fl)
    V = torch.empty_like(fl)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        plan.execute(fl, fc, fe, V, stream)
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute(fl, fc, fe, V, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = plan.timings()
    plan.set_timing(False)
    elapsed = t1 - t0
    N = st["n_leaves"] * case["K"] ** 2
    value = N * args.steps / elapsed

    work = algorithmic_work(st, case["K"], case["p"], case["interior"])
    dom = max((k for k in work), key=lambda k: phases[k])
    flops, nbytes = work[dom]
    sec = phases[dom] * 1e-3
    intensity = flops / nbytes
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity >= ridge:
        roof = {"bound": "mfma", "achieved": flops / sec / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": nbytes / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = {"near": "k_near", "extension": "k_fe_init+k_extension", "p2m_m2m": "k_p2m+k_m2m",
                      "m2l_p2l": "k_m2l", "l2l": "k_l2l", "far": "k_far"}[dom]
    roof["phase_ms"] = phases[dom]
    roof["algorithmic_flops"] = flops
    roof["algorithmic_bytes"] = nbytes

    out = {
        "metric": METRIC, "value": value, "unit": "leaf points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": case["cfg"]["name"], "leaves": st["n_leaves"], "nodes": N, "K": case["K"],
                   "p": case["p"], "levels": st["n_levels"], "cut_leaves": st["n_cut"],
                   "ext_targets": st["n_ext_targets"], "precision": "fp64"},
        "phases_ms": {k: round(v, 4) for k, v in phases.items() if k != "count"},
        "plan_s": st["plan_seconds"], "tables_s": case["t_ctx"],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        base, (sel, v_o, fe_o) = cpu_baseline(case, args.baseline_seconds)
        out["cpu_baseline"] = base
        Vg = V.cpu().numpy().ravel()[sel]
        out["check"] = {"nodes": int(sel.size),
                        "rel_linf_vs_oracle": float(np.abs(Vg - v_o).max() / np.abs(v_o).max()),
                        "note": "GPU V against the oracle's V of the oracle's float64 extension"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
