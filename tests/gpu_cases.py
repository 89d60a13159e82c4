"""Shared set-up for the GPU parity tests: build a workload's tree and inputs,
run the HIP path through the C-ABI, and compute the oracle's answers."""
import sys

import numpy as np

from oracle import extension, geometry, volume
from paper_2211_14537_amd import tree as T
from paper_2211_14537_amd import vfx
from workloads import get_config

U = 2.0 ** -53


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def setup(name, p=None, all_regular=False, fun=None):
    cfg = get_config(name)
    if fun is not None:
        cfg["fun"] = fun
    K = cfg["K"]
    ctx = vfx.Context(K, p if p is not None else cfg["p"], root=cfg["root"])
    P = ctx.stencil_points()
    tr = T.build_tree(cfg, P)
    f_leaf, f_cut = T.sample_inputs(cfg, tr, P)
    kind = np.ones_like(tr["kind"]) if all_regular else tr["kind"]
    mask = None if all_regular else tr["mask"]
    plan = vfx.Plan(ctx, tr["level"], tr["ix"], tr["iy"], kind, mask)
    ot = geometry.Tree(tr["level"], tr["ix"], tr["iy"], cfg["root"])
    return dict(cfg=cfg, K=K, ctx=ctx, tree=tr, f_leaf=f_leaf, f_cut=f_cut, plan=plan, otree=ot, kind=kind)


def run_gpu(case, repeat=1):
    import torch
    dev = torch.device("cuda:0")
    fl = torch.tensor(case["f_leaf"], dtype=torch.float64, device=dev)
    fc = torch.tensor(case["f_cut"] if case["f_cut"].size else np.zeros((0, case["ctx"].n_stencil)),
                      dtype=torch.float64, device=dev)
    outs = []
    for _ in range(repeat):
        fe = torch.full_like(fl, float("nan"))
        V = torch.full_like(fl, float("nan"))
        case["plan"].execute(fl, fc, fe, V)
        torch.cuda.synchronize()
        outs.append((fe.cpu().numpy(), V.cpu().numpy()))
    return outs if repeat > 1 else outs[0]


def sample_targets(case, n_random, leaves=(), seed=0):
    X, Y = case["otree"].leaf_nodes(case["K"])
    rng = np.random.default_rng(seed)
    sel = set(rng.choice(X.size, min(n_random, X.size), replace=False).tolist())
    n = case["K"] ** 2
    for leaf in leaves:
        sel.update(range(leaf * n, (leaf + 1) * n))
    sel = np.array(sorted(sel))
    return sel, X.ravel()[sel], Y.ravel()[sel]


def oracle_extension(case, precision="fp64", cut_ids=None):
    tr = case["tree"]
    return extension.extend(case["otree"], tr["kind"], case["f_leaf"], case["f_cut"], tr["mask"].astype(bool),
                            case["K"], precision=precision, cut_ids=cut_ids)


def interior_values(case, i):
    tr = case["tree"]
    r = list(tr["cut_ids"]).index(i)
    return case["f_cut"][r][tr["mask"][r] != 0]


def oracle_potential(case, fe, tx, ty):
    return volume.potential(case["otree"], fe, case["K"], tx, ty)


def volume_checks(case, fe_gpu, V_gpu, sel, tx, ty, fe_o):
    """Rel Linf errors of V_gpu at the sampled nodes sel (coordinates tx, ty):
    g1 against the oracle's V of the GPU's own extended data fe_gpu (the
    volume FMM alone), g3 against the oracle's V of the oracle's extended
    data fe_o (end to end).  V_o(fe_gpu) = V_o(fe_o) + V_o(fe_gpu - fe_o),
    and the difference is nonzero only on extension targets, so the second
    potential is cheap.  Returns (g1, g3, v_o)."""
    v_o = oracle_potential(case, fe_o, tx, ty)
    d = np.asarray(fe_gpu, dtype=np.float64) - fe_o
    v_g = v_o + (oracle_potential(case, d, tx, ty) if np.any(d != 0.0) else 0.0)
    V = np.asarray(V_gpu).ravel()[sel]
    g1 = float(np.abs(V - v_g).max() / np.abs(v_g).max())
    g3 = float(np.abs(V - v_o).max() / np.abs(v_o).max())
    return g1, g3, v_o
