"""GPU parity at the full size of the benchmark workload (starfish_adaptive:
K = 16, p = 24, 4207 leaves, 1.08e6 leaf nodes, 730 cut leaves), in the
launch configuration bench.py times (FP64 near field, default launch
parameters), on sampled outputs the oracle computes one by one:

* V on given leaf data (every leaf regular): 96 seeded nodes plus all nodes
  of the coarsest and of the finest leaf, rel Linf <= 1e-10 against the
  oracle's direct quadrature;
* f^e of 40 seeded cut leaves (their whole extension lists) against the
  oracle's float64 extension, within the conditioning-aware bound of the
  other parity tests; regular leaves bit-exact.
"""
import numpy as np
import pytest

from gpu_cases import interior_values, oracle_extension, oracle_potential, run_gpu, say, setup
from oracle import extension
from paper_2211_14537_amd import vfx

pytestmark = pytest.mark.gpu


def test_full_size_starfish(gpu_device):
    say("[full size] starfish_adaptive p=24")
    case = setup("starfish_adaptive")
    tr = case["tree"]
    lv = np.asarray(tr["level"])
    assert len(lv) == 4207 and len(tr["cut_ids"]) == 730
    # extension on a seeded sample of cut leaves
    fe, _ = run_gpu(case)
    rng = np.random.default_rng(7)
    cuts = sorted(rng.choice(np.asarray(tr["cut_ids"]), 40, replace=False).tolist())
    ref, info = oracle_extension(case, "fp64", cut_ids=cuts)
    worst = 0.0
    for i in cuts:
        rec = info[i]
        tg = rec["targets"]
        tol = 2.0 * extension.extension_tolerance(rec, ref[tg], interior_values(case, i))
        err = float(np.abs(fe[tg] - ref[tg]).max())
        assert err <= tol, (i, err, tol)
        worst = max(worst, err / tol)
    reg = np.asarray(tr["kind"]) == 1
    assert np.array_equal(fe[reg], case["f_leaf"][reg])
    say(f"    extension: 40 cut leaves, worst error / bound = {worst:.3f}")
    # V on given data at sampled nodes, same tree, every leaf regular
    plan = vfx.Plan(case["ctx"], tr["level"], tr["ix"], tr["iy"], np.ones_like(tr["kind"]))
    reg_case = dict(case, plan=plan, f_cut=np.zeros((0, case["ctx"].n_stencil)))
    fe2, V = run_gpu(reg_case)
    assert np.array_equal(fe2, case["f_leaf"])
    n = case["K"] ** 2
    X, Y = case["otree"].leaf_nodes(case["K"])
    sel = set(rng.choice(X.size, 96, replace=False).tolist())
    for leaf in (int(np.argmin(lv)), int(np.argmax(lv))):
        sel.update(range(leaf * n, (leaf + 1) * n))
    sel = np.array(sorted(sel))
    vo = oracle_potential(case, case["f_leaf"], X.ravel()[sel], Y.ravel()[sel])
    rel = np.abs(V.ravel()[sel] - vo).max() / np.abs(vo).max()
    say(f"    V: rel Linf = {rel:.3e} over {sel.size} nodes")
    assert rel <= 1e-10


def test_full_size_wedge_mixed(gpu_device):
    """wedge_adaptive (14254 leaves, 3.65e6 nodes) on given data: the FP64
    path within 1e-10 and the all-mixed near field (bf16 slices, FP32
    accumulation) within 2e-6 of the oracle at sampled nodes."""
    say("[full size] wedge_adaptive p=24, FP64 and mixed")
    case = setup("wedge_adaptive", all_regular=True)
    assert len(case["tree"]["level"]) == 14254
    lv = np.asarray(case["tree"]["level"])
    n = case["K"] ** 2
    X, Y = case["otree"].leaf_nodes(case["K"])
    rng = np.random.default_rng(11)
    sel = set(rng.choice(X.size, 64, replace=False).tolist())
    sel.update(range(int(np.argmax(lv)) * n, (int(np.argmax(lv)) + 1) * n))
    sel = np.array(sorted(sel))
    vo = oracle_potential(case, case["f_leaf"], X.ravel()[sel], Y.ravel()[sel])
    _, V64 = run_gpu(case)
    rel64 = np.abs(V64.ravel()[sel] - vo).max() / np.abs(vo).max()
    case["plan"].set_precision(1, 0)
    _, Vmx = run_gpu(case)
    relmx = np.abs(Vmx.ravel()[sel] - vo).max() / np.abs(vo).max()
    say(f"    rel Linf over {sel.size} nodes: FP64 {rel64:.3e}, mixed {relmx:.3e}")
    assert rel64 <= 1e-10
    assert relmx <= 2e-6
