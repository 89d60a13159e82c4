"""Mixed-precision near field against the oracle and the FP64 path.

The list-1 interactions of sources at level >= min_level run on the bf16
matrix cores (three bf16 slices per operand, FP32 accumulation); everything
else stays FP64.  The tests state the error of V against the oracle's direct
quadrature per setting, bound it, and check that raising min_level (fewer
mixed interactions, each with a smaller h^2 weight excluded) does not make
it worse than the all-mixed setting."""
import numpy as np
import pytest

from gpu_cases import oracle_potential, run_gpu, sample_targets, say, setup

pytestmark = pytest.mark.gpu


def _rel(case, V, sel, vo):
    return float(np.abs(V.ravel()[sel] - vo).max() / np.abs(vo).max())


def test_mixed_volume_against_oracle(gpu_device):
    case = setup("starfish_small", p=24, all_regular=True)
    sel, tx, ty = sample_targets(case, 400, leaves=(0, case["otree"].n - 1))
    vo = oracle_potential(case, case["f_leaf"], tx, ty)
    _, V64 = run_gpu(case)
    e64 = _rel(case, V64, sel, vo)
    errs = {}
    for lmin in (0, 5):
        case["plan"].set_precision(1, lmin)
        fe, V = run_gpu(case)
        assert np.array_equal(fe, case["f_leaf"])
        errs[lmin] = _rel(case, V, sel, vo)
        say(f"    mixed (sources at level >= {lmin}): rel Linf vs oracle {errs[lmin]:.3e}  (FP64 path {e64:.3e})")
    case["plan"].set_precision(0)
    _, Vb = run_gpu(case)
    assert np.array_equal(Vb, V64)  # back to FP64: bitwise the FP64 result
    assert e64 <= 1e-11
    assert errs[0] <= 2e-6
    assert errs[5] <= errs[0] * 1.01 + 1e-15


def test_mixed_end_to_end(gpu_device):
    """Extension + volume with the mixed near field: V of the extended data
    against the oracle's V of the oracle's extension stays within the FP64
    path's error plus the mixed bound."""
    case = setup("starfish_small", p=24)
    sel, tx, ty = sample_targets(case, 300)
    fe64, V64 = run_gpu(case)
    case["plan"].set_precision(1, 0)
    fe, V = run_gpu(case)
    assert np.array_equal(fe, fe64)  # the extension is FP64 in both modes
    d = float(np.abs(V - V64).max() / np.abs(V64).max())
    say(f"    mixed vs FP64 path, end to end: rel Linf {d:.3e}")
    assert d <= 2e-6


def test_mixed_rejects_other_grid_sizes(gpu_device):
    from paper_2211_14537_amd import vfx
    case = setup("disk_uniform3", p=20, all_regular=True)
    with pytest.raises(vfx.VfxError):
        case["plan"].set_precision(1, 0)
    fe, V = run_gpu(case)  # the plan stays FP64 and usable
    assert np.isfinite(V).all()
