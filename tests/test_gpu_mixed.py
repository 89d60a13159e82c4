"""Mixed-precision near field against the oracle and the FP64 path.

The list-1 interactions of sources at level >= min_level run on the matrix
cores in fixed-point slices: mode 1 four bf16 slices per operand row (exact
FP32 sums per block of 128 contraction indices), mode 2 five int8 slices
(exact int32 sums over the whole contraction); FP64 results in both, and
everything else stays FP64.  The tests state the error of V against the oracle's direct
quadrature per setting, bound it, and check that raising min_level (fewer
mixed interactions, each with a smaller h^2 weight excluded) does not make
it worse than the all-mixed setting."""
import numpy as np
import pytest

from gpu_cases import oracle_potential, run_gpu, sample_targets, say, setup

pytestmark = pytest.mark.gpu


def _rel(case, V, sel, vo):
    return float(np.abs(V.ravel()[sel] - vo).max() / np.abs(vo).max())


@pytest.mark.parametrize("mode", [1, 2], ids=["bf16", "int8"])
def test_mixed_volume_against_oracle(gpu_device, mode):
    case = setup("starfish_small", p=24, all_regular=True)
    sel, tx, ty = sample_targets(case, 400, leaves=(0, case["otree"].n - 1))
    vo = oracle_potential(case, case["f_leaf"], tx, ty)
    _, V64 = run_gpu(case)
    e64 = _rel(case, V64, sel, vo)
    errs = {}
    for lmin in (0, 3, 4):  # the tree's leaves reach level 4
        case["plan"].set_precision(mode, lmin)
        fe, V = run_gpu(case)
        assert np.array_equal(fe, case["f_leaf"])
        errs[lmin] = _rel(case, V, sel, vo)
        say(f"    mixed mode {mode} (sources at level >= {lmin}): rel Linf vs oracle {errs[lmin]:.3e}  (FP64 path {e64:.3e})")
    case["plan"].set_precision(0)
    _, Vb = run_gpu(case)
    assert np.array_equal(Vb, V64)  # back to FP64: bitwise the FP64 result
    assert e64 <= 1e-11
    # measured all mixed: 4.5e-10 (bf16 slices, about 2^-32 of each operand
    # row's maximum), 1.8e-10 (int8 slices, about 2^-34); on this shallow
    # uniform tree the near field carries a large share of V
    assert errs[0] <= {1: 2e-9, 2: 1e-9}[mode]
    assert int(np.max(case["tree"]["level"])) == 4
    for lmin in (3, 4):
        assert e64 < errs[lmin] <= errs[0] * 1.01 + 1e-15


@pytest.mark.parametrize("mode", [1, 2], ids=["bf16", "int8"])
def test_mixed_mode_with_no_mixed_pair_is_bitwise_fp64(gpu_device, mode):
    """A mixed mode with a level threshold above every leaf mixes no list-1
    pair: the pairs keep the FP64 tiles and kernels and the result is the
    FP64 plan's, bit for bit; with the threshold at the finest level the two
    paths differ, by about the slices' truncation (2^-32 of the row maxima
    of the operands with bf16 slices, 2^-34 with int8 slices)."""
    case = setup("starfish_small", p=24, all_regular=True)
    lv = int(np.max(case["tree"]["level"]))
    _, V64 = run_gpu(case)
    case["plan"].set_precision(mode, lv + 1)
    _, V = run_gpu(case)
    assert np.array_equal(V, V64)
    case["plan"].set_precision(mode, lv)
    _, Vf = run_gpu(case)
    d = float(np.abs(Vf - V64).max() / np.abs(V64).max())
    say(f"    mixed mode {mode} only at level {lv}: rel Linf vs FP64 path {d:.3e}")
    assert 0 < d <= {1: 3e-9, 2: 2e-9}[mode]  # measured 7.3e-10 (bf16), 3.6e-10 (int8)


@pytest.mark.parametrize("mode", [1, 2], ids=["bf16", "int8"])
def test_mixed_end_to_end(gpu_device, mode):
    """Extension + volume with the mixed near field: V of the extended data
    against the oracle's V of the oracle's extension stays within the FP64
    path's error plus the mixed bound."""
    case = setup("starfish_small", p=24)
    sel, tx, ty = sample_targets(case, 300)
    fe64, V64 = run_gpu(case)
    case["plan"].set_precision(mode, 0)
    fe, V = run_gpu(case)
    assert np.array_equal(fe, fe64)  # the extension is FP64 in both modes
    d = float(np.abs(V - V64).max() / np.abs(V64).max())
    say(f"    mixed mode {mode} vs FP64 path, end to end: rel Linf {d:.3e}")
    assert d <= {1: 8e-9, 2: 3e-9}[mode]  # measured 1.7e-9 (bf16), 5.0e-10 (int8)


def test_mixed_rejects_other_grid_sizes(gpu_device):
    from paper_2211_14537_amd import vfx
    case = setup("disk_uniform3", p=20, all_regular=True)
    for mode in (1, 2):
        with pytest.raises(vfx.VfxError):
            case["plan"].set_precision(mode, 0)
    fe, V = run_gpu(case)  # the plan stays FP64 and usable
    assert np.isfinite(V).all()


# gates of the degenerate-tree test per mode: about 3-5x the measured
# 1.5e-9 (bf16 slices) and 8.0e-10 (int8 slices); on trees this shallow the
# near field is all of V, so the slices' truncation (about 2^-32 and 2^-34
# of each operand row's maximum) shows in full
DEGENERATE_GATE = {1: 5e-9, 2: 4e-9}


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["fp64", "bf16", "int8"])
def test_mixed_on_degenerate_trees(gpu_device, mode):
    """K = 16 trees of one leaf (the self pair only: the mixed kernels run
    their self-operator items alone), four leaves (near field only) and
    sixteen (low-rank neighbour pairs too), all sources mixed, against the
    oracle's direct quadrature at every node."""
    from oracle import geometry, volume
    from paper_2211_14537_amd import vfx
    import torch
    from workloads import GaussianSum
    fun = GaussianSum([[0.1, -0.1]], [0.2])
    ctx = vfx.Context(16, 24)
    d = torch.device("cuda:0")
    gate = {0: 1e-12, 1: DEGENERATE_GATE[1], 2: DEGENERATE_GATE[2]}[mode]
    trees = (([0], [0], [0]), ([1] * 4, [0, 1, 0, 1], [0, 0, 1, 1]),
             ([2] * 16, [i % 4 for i in range(16)], [i // 4 for i in range(16)]))
    for lv, ix, iy in trees:
        plan = vfx.Plan(ctx, lv, ix, iy, np.ones(len(lv), dtype=np.int8))
        if mode:
            plan.set_precision(mode, 0)
        ot = geometry.Tree(lv, ix, iy)
        X, Y = ot.leaf_nodes(16)
        f = fun.f(X, Y)
        fl = torch.tensor(f, device=d)
        fe, V = torch.empty_like(fl), torch.empty_like(fl)
        plan.execute(fl, torch.zeros((0, ctx.n_stencil), dtype=torch.float64, device=d), fe, V)
        torch.cuda.synchronize()
        vo = volume.potential(ot, f, 16, X.ravel(), Y.ravel())
        err = float(np.abs(V.cpu().numpy().ravel() - vo).max() / np.abs(vo).max())
        say(f"    mode {mode}, {len(lv)} leaves: rel Linf vs oracle {err:.3e}")
        assert err <= gate
