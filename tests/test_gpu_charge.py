"""GPU parity of the net charge A^e = int f^e (the log|x| growth of the
volume potential that the exterior problem's boundary solve offsets,
Section 6) against the oracle's exactly rounded Fejer-rule sum.

Tolerance: both sides sum the same h^2 w_j f_j terms in FP64 (the kernel in
a fixed tree order, the oracle exactly rounded), so they agree to a few
units of 2^-53 times the sum of the terms' magnitudes; 1e-13 of that sum is
written in the tests.  With the extension in front, the f^e of the two sides
differ by at most the extension bound per target leaf, and the weights are
positive with sum h^2 per leaf, which bounds the charge difference."""
import numpy as np
import pytest

from gpu_cases import oracle_extension, interior_values, run_gpu, say, setup
from oracle import extension, geometry, volume

pytestmark = pytest.mark.gpu


def _abs_sum(otree, fe, K):
    return float(volume.net_charge(otree, np.abs(fe), K).max())


def _gpu_charge(plan, fe):
    import torch
    d = torch.device("cuda:0")
    fe_t = torch.tensor(np.ascontiguousarray(fe), dtype=torch.float64, device=d)
    nrhs = fe_t.numel() // (plan.n_leaves * fe_t.shape[-1])
    out = torch.full((nrhs,), float("nan"), dtype=torch.float64, device=d)
    plan.net_charge(fe_t, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name", ["disk_uniform3", "starfish_small", "starfish_adaptive"])
def test_net_charge_given_data(gpu_device, name):
    """Given data on every leaf, one and three right-hand sides (the second
    stack entry shifted and scaled, the third random), bitwise repeatable."""
    say(f"[net charge] {name}")
    case = setup(name, all_regular=True)
    K, ot = case["K"], case["otree"]
    f = case["f_leaf"]
    rng = np.random.default_rng(3)
    stack = np.stack([f, -2.0 * f + 1.0, rng.standard_normal(f.shape)])
    ref = volume.net_charge(ot, stack, K)
    one = _gpu_charge(case["plan"], f)
    three = _gpu_charge(case["plan"], stack)
    again = _gpu_charge(case["plan"], stack)
    assert np.array_equal(three, again)
    assert one[0] == three[0]  # the batch sums each right-hand side alike
    for r in range(3):
        tol = 1e-13 * _abs_sum(ot, stack[r], K)
        say(f"    rhs {r}: A = {three[r]: .15e}, |gpu - oracle| = {abs(three[r] - ref[r]):.2e} (tol {tol:.2e})")
        assert abs(three[r] - ref[r]) <= tol


@pytest.mark.parametrize("K", [4, 12])
def test_net_charge_other_grids_and_degenerate_trees(gpu_device, K):
    """The root alone and a depth-1 tree (fewer leaves than partial-sum
    blocks), f = 1 gives the root's area and f = x^3 y^2 its closed form."""
    from paper_2211_14537_amd import vfx
    ctx = vfx.Context(K, 20)
    for lv, ix, iy in (([0], [0], [0]), ([1] * 4, [0, 1, 0, 1], [0, 0, 1, 1])):
        plan = vfx.Plan(ctx, lv, ix, iy, np.ones(len(lv), dtype=np.int8))
        ot = geometry.Tree(lv, ix, iy)
        X, Y = ot.leaf_nodes(K)
        a = _gpu_charge(plan, np.stack([np.ones_like(X), X ** 3 * Y ** 2 + 0.25]))
        area = ot.size ** 2
        x0, x1 = ot.cx0 - 0.5 * ot.size, ot.cx0 + 0.5 * ot.size
        exact = (x1 ** 4 - x0 ** 4) / 4 * (x1 ** 3 - x0 ** 3) / 3 + 0.25 * area
        say(f"    K={K}, {len(lv)} leaves: A(1) = {a[0]!r}, A(x^3 y^2 + 1/4) - exact = {a[1] - exact:.2e}")
        assert abs(a[0] - area) <= 1e-14 * area
        assert abs(a[1] - exact) <= 1e-14 * area


def test_net_charge_of_the_extension(gpu_device):
    """End to end on starfish_small: the charge of the library's f^e against
    the charge of the oracle's float64 extension, within the extension's
    per-target bound summed over the targets (h^2 each) plus the summation
    tolerance."""
    say("[net charge] starfish_small with the extension")
    case = setup("starfish_small")
    K, ot = case["K"], case["otree"]
    fe, _ = run_gpu(case)
    ref, info = oracle_extension(case, "fp64")
    kind = case["tree"]["kind"]
    assert np.array_equal(ref[kind == 1], case["f_leaf"][kind == 1])
    h = ot.h()
    bound = 0.0
    for i, rec in info.items():
        tg = rec["targets"]
        tol = 2.0 * extension.extension_tolerance(rec, ref[tg], interior_values(case, i))
        bound += tol * float(np.sum(h[tg] ** 2))
    bound += 1e-13 * _abs_sum(ot, ref, K)
    a = _gpu_charge(case["plan"], fe)[0]
    a_ref = volume.net_charge(ot, ref, K)[0]
    say(f"    A^e = {a:.15e}, oracle {a_ref:.15e}, diff {abs(a - a_ref):.2e} (bound {bound:.2e})")
    assert abs(a - a_ref) <= bound
