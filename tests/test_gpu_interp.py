"""Interpolation of leaf-grid data to arbitrary points (vfx_interp)."""
import numpy as np
import pytest

from gpu_cases import oracle_potential, run_gpu, say, setup

pytestmark = pytest.mark.gpu


def _interp(case, V, x, y):
    import torch
    dev = torch.device("cuda:0")
    Vt = torch.tensor(V, dtype=torch.float64, device=dev)
    px = torch.tensor(x, dtype=torch.float64, device=dev)
    py = torch.tensor(y, dtype=torch.float64, device=dev)
    out = torch.empty_like(px)
    case["plan"].interp(Vt, px, py, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_interp_reproduces_polynomials(gpu_device):
    """Tensor polynomials of degree K-1 are reproduced exactly (up to
    rounding) at random points, on an adaptive tree."""
    case = setup("starfish_small", p=24, all_regular=True)
    K = case["K"]
    X, Y = case["otree"].leaf_nodes(K)

    def poly(x, y):
        return (1.0 + 0.3 * x - 0.7 * y) ** 5 + 0.2 * x ** 15 - 0.1 * (x * y) ** 7 + y ** 15

    V = poly(X, Y).reshape(-1, K * K)
    rng = np.random.default_rng(3)
    x, y = rng.uniform(-1, 1, 5000), rng.uniform(-1, 1, 5000)
    # include exact node coordinates and points on leaf edges
    x[:50], y[:50] = X.ravel()[:50], Y.ravel()[:50]
    x[50:60], y[50:60] = 0.0, np.linspace(-0.9, 0.9, 10)
    got = _interp(case, V, x, y)
    ref = poly(x, y)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"    polynomial reproduction: rel Linf {err:.2e}")
    assert err < 1e-13


def test_interp_volume_potential_off_grid(gpu_device):
    """V interpolated from the leaf grids matches the oracle's direct
    quadrature of V at off-grid points (domain and boundary-like points)."""
    case = setup("starfish_small", p=24, all_regular=True)
    _, V = run_gpu(case)
    rng = np.random.default_rng(5)
    th = rng.uniform(0, 2 * np.pi, 120)
    r = 0.5 + 0.15 * np.cos(5 * th)
    x = np.concatenate([r * np.cos(th), rng.uniform(-0.95, 0.95, 80)])
    y = np.concatenate([r * np.sin(th), rng.uniform(-0.95, 0.95, 80)])
    got = _interp(case, V, x, y)
    ref = oracle_potential(case, case["f_leaf"], x, y)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"    off-grid V vs oracle: rel Linf {err:.2e}")
    assert err < 1e-10


def test_interp_outside_root_is_nan(gpu_device):
    case = setup("disk_uniform3", p=20, all_regular=True)
    V = np.zeros((case["otree"].n, case["K"] ** 2))
    got = _interp(case, V, np.array([1.5, 0.0, -1.0000001]), np.array([0.0, 2.0, 0.0]))
    assert np.isnan(got).all()
