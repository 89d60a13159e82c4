"""GPU parity at the full size of the benchmark workloads, in the launch
configuration bench.py times (default launch parameters), on sampled outputs
the oracle computes one by one:

starfish_adaptive (K = 16, p = 24, 4207 leaves, 1.08e6 nodes, 730 cut leaves)
* the timed plan's own execute: f^e of every cut leaf against the oracle's
  float64 extension, within the conditioning-aware least-squares bound
  (regular leaves bit-exact); V against the oracle's V of the GPU's f^e
  (G1, rel Linf <= 1e-10) and against the oracle's V of the oracle's f^e
  (G3, end to end: 1e-10 max|V| plus the potential of the allowed extension
  differences) at 96 seeded nodes plus every node of a cut leaf, of an
  extension target, of the coarsest and of the finest leaf;
* V on given leaf data (every leaf regular), rel Linf <= 1e-10.

wedge_adaptive (14254 leaves, 3.65e6 nodes, 1536 cut leaves)
* the timed plan in FP64: G1 <= 1e-10 and G3 as above;
* the same plan with the mixed-precision near field at the setting bench.py
  reports: G1 within the gate stated below.
"""
import math

import numpy as np
import pytest

from gpu_cases import interior_values, oracle_extension, oracle_potential, run_gpu, say, setup, volume_checks
from oracle import extension
from paper_2211_14537_amd import vfx

pytestmark = pytest.mark.gpu


def _nodes(case, n_random, seed, leaves):
    X, Y = case["otree"].leaf_nodes(case["K"])
    rng = np.random.default_rng(seed)
    n = case["K"] ** 2
    sel = set(rng.choice(X.size, n_random, replace=False).tolist())
    for leaf in leaves:
        sel.update(range(int(leaf) * n, (int(leaf) + 1) * n))
    sel = np.array(sorted(sel))
    return sel, X.ravel()[sel], Y.ravel()[sel]


def _extension_and_bound(case, fe):
    """Every cut leaf against the oracle's float64 extension; returns the
    oracle's extended data, the worst error / bound, and the potential bound
    of the allowed differences (|int_B log|x-y| d| <= |d| h^2 (|log h| + 2)
    per target leaf, h <= 1)."""
    ref, info = oracle_extension(case, "fp64")
    h = case["otree"].h()
    worst, bound = 0.0, 0.0
    for i, rec in info.items():
        tg = rec["targets"]
        tol = 2.0 * extension.extension_tolerance(rec, ref[tg], interior_values(case, i))
        err = float(np.abs(fe[tg] - ref[tg]).max())
        assert err <= tol, (i, err, tol)
        worst = max(worst, err / tol)
        for j in tg:
            bound += tol * h[j] ** 2 * (abs(math.log(h[j])) + 2.0) / (2 * math.pi)
    return ref, worst, bound


def _sample_leaves(case, rng):
    tr = case["tree"]
    lv = np.asarray(tr["level"])
    owner = case["plan"].ext_owner()
    kind = np.asarray(tr["kind"])
    cut = rng.choice(np.asarray(tr["cut_ids"]))
    ext = rng.choice(np.nonzero((owner >= 0) & (kind == 0))[0])
    return [int(np.argmin(lv)), int(np.argmax(lv)), int(cut), int(ext)]


def test_full_size_starfish(gpu_device):
    say("[full size] starfish_adaptive p=24")
    case = setup("starfish_adaptive")
    tr = case["tree"]
    assert len(tr["level"]) == 4207 and len(tr["cut_ids"]) == 730
    fe, V = run_gpu(case)
    reg = np.asarray(tr["kind"]) == 1
    assert np.array_equal(fe[reg], case["f_leaf"][reg])
    ref, worst, bound = _extension_and_bound(case, fe)
    say(f"    extension: all 730 cut leaves, worst error / bound = {worst:.3f}")
    rng = np.random.default_rng(7)
    sel, tx, ty = _nodes(case, 96, 7, _sample_leaves(case, rng))
    g1, g3, v_o = volume_checks(case, fe, V, sel, tx, ty, ref)
    err3 = g3 * np.abs(v_o).max()
    say(f"    timed plan over {sel.size} nodes: G1 rel Linf {g1:.3e}, G3 rel Linf {g3:.3e} "
        f"(allowed {1e-10 + bound / np.abs(v_o).max():.3e})")
    assert g1 <= 1e-10
    assert err3 <= 1e-10 * np.abs(v_o).max() + bound
    # V on given data, every leaf regular
    plan = vfx.Plan(case["ctx"], tr["level"], tr["ix"], tr["iy"], np.ones_like(tr["kind"]))
    reg_case = dict(case, plan=plan, f_cut=np.zeros((0, case["ctx"].n_stencil)))
    fe2, V2 = run_gpu(reg_case)
    assert np.array_equal(fe2, case["f_leaf"])
    lv = np.asarray(tr["level"])
    sel, tx, ty = _nodes(case, 64, 8, (int(np.argmax(lv)),))
    vo = oracle_potential(case, case["f_leaf"], tx, ty)
    rel = np.abs(V2.ravel()[sel] - vo).max() / np.abs(vo).max()
    say(f"    given data: rel Linf = {rel:.3e} over {sel.size} nodes")
    assert rel <= 1e-10
    # the same with the target-stationary near field
    plan.set_near_mode(1)
    _, V3 = run_gpu(reg_case)
    rel3 = np.abs(V3.ravel()[sel] - vo).max() / np.abs(vo).max()
    say(f"    given data, target-stationary near field: rel Linf = {rel3:.3e}")
    assert rel3 <= 1e-10


# The mixed-precision setting bench.py reports beside FP64 on this workload
# (int8 slices, mode 2; the bf16 slices of mode 1 are checked too), and the
# gate on G1 of both: 10x the 8.4e-13 of the bf16 slices and 5x the 1.7e-12
# of the int8 slices over these nodes (the FP64 path: 4.5e-13).
WEDGE_MIXED = dict(min_level=0, modes=(2, 1), gate=8.5e-12)


def test_full_size_wedge(gpu_device):
    say("[full size] wedge_adaptive p=24, FP64 and mixed")
    case = setup("wedge_adaptive")
    tr = case["tree"]
    assert len(tr["level"]) == 14254
    fe, V64 = run_gpu(case)
    ref, worst, bound = _extension_and_bound(case, fe)
    say(f"    extension: all {len(tr['cut_ids'])} cut leaves, worst error / bound = {worst:.3f}")
    rng = np.random.default_rng(11)
    sel, tx, ty = _nodes(case, 64, 11, _sample_leaves(case, rng)[1:3])  # the finest leaf and a cut leaf
    g1, g3, v_o = volume_checks(case, fe, V64, sel, tx, ty, ref)
    say(f"    FP64 over {sel.size} nodes: G1 {g1:.3e}, G3 {g3:.3e} "
        f"(allowed {1e-10 + bound / np.abs(v_o).max():.3e})")
    assert g1 <= 1e-10
    assert g3 * np.abs(v_o).max() <= 1e-10 * np.abs(v_o).max() + bound
    for mode in WEDGE_MIXED["modes"]:
        case["plan"].set_precision(mode, WEDGE_MIXED["min_level"])
        fe_mx, Vmx = run_gpu(case)
        assert np.array_equal(fe_mx, fe)  # the extension is FP64 in every mode
        g1m, g3m, _ = volume_checks(case, fe, Vmx, sel, tx, ty, ref)
        say(f"    mixed mode {mode} (sources at level >= {WEDGE_MIXED['min_level']}): G1 {g1m:.3e}, G3 {g3m:.3e}")
        assert g1m <= WEDGE_MIXED["gate"]
