"""Pins for the oracle's Chebyshev and stencil pieces (CPU).

What is pinned against what:
* first-kind nodes and coefficients against T_m(cos th) = cos(m th) and exact
  polynomial interpolation;
* Fejer weights against the exact integrals 2/(1-m^2) of T_m;
* the flat-limit interpolation matrix against its definition as the total
  degree-10 polynomial interpolant (reproduction; degree 11 is a negative
  control) and against the Gaussian form of eq. (defA) evaluated directly at
  small eps in high precision (reading R1: flat limit).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import cheb, stencil


def test_nodes_are_first_kind_and_ascending():
    for K in (4, 8, 12, 16):
        t = cheb.nodes(K)
        assert np.all(np.diff(t) > 0)
        assert np.all(np.abs(t) < 1)
        # T_K vanishes at the first-kind nodes
        assert np.abs(np.cos(K * np.arccos(t))).max() < 1e-13


@pytest.mark.parametrize("K", [5, 8, 16])
def test_coefficients_reproduce_polynomials(K):
    rng = np.random.default_rng(K)
    c = rng.standard_normal((K, K))
    t = cheb.nodes(K)
    tx, ty = np.meshgrid(t, t, indexing="ij")
    vals = cheb.eval2d(c, tx.ravel(), ty.ravel()).reshape(K, K)
    assert np.allclose(cheb.coeffs2d(vals), c, atol=1e-13, rtol=0)
    # T_m by recurrence equals cos(m arccos t)
    V = cheb.vander(t, K + 3)
    for m in range(K + 4):
        assert np.abs(V[:, m] - np.cos(m * np.arccos(t))).max() < 1e-13


@pytest.mark.parametrize("K", [4, 8, 16])
def test_fejer_weights_integrate_exactly(K):
    w = cheb.fejer1_weights(K)
    t = cheb.nodes(K)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(K):
        exact = 0.0 if m % 2 else 2.0 / (1.0 - m * m)
        assert abs(np.dot(w, np.cos(m * np.arccos(t))) - exact) < 1e-14
    assert np.all(w > 0)


def test_padua_points_unisolvent():
    G = stencil.padua_points(10)
    assert G.shape == (66, 2)
    assert len({(round(a, 14), round(b, 14)) for a, b in G}) == 66
    basis = stencil.total_degree_basis(10)
    V = np.array([[math.cos(m * math.acos(x)) * math.cos(n * math.acos(y)) for (m, n) in basis]
                  for x, y in G])
    s = np.linalg.svd(V, compute_uv=False)
    assert s[-1] / s[0] > 1e-3


@pytest.mark.parametrize("K", [8, 16])
def test_interp_matrix_reproduces_degree_10_not_11(K):
    A = stencil.interp_matrix(K)
    P = stencil.stencil_points(K)
    assert A.shape == (K * K + 144 + 66, 66)
    G = P[-66:]
    # the G rows are the identity (interpolation at the support nodes)
    assert np.abs(A[-66:] - np.eye(66)).max() < 1e-13
    rng = np.random.default_rng(0)
    for deg, ok in ((10, True), (11, False)):
        err = 0.0
        for _ in range(3):
            cf = {(m, n): rng.standard_normal() for m in range(deg + 1) for n in range(deg + 1 - m)}

            def f(x, y):
                return sum(v * np.cos(m * np.arccos(np.clip(x, -1, 1))) *
                           np.cos(n * np.arccos(np.clip(y, -1, 1))) for (m, n), v in cf.items())
            err = max(err, np.abs(A @ f(G[:, 0], G[:, 1]) - f(P[:, 0], P[:, 1])).max())
        if ok:
            assert err < 1e-12
        else:
            assert err > 1e-3
    # bounded universal map (the paper's argument for a stable universal step)
    assert np.abs(A).sum(axis=1).max() < 6.0


@pytest.mark.slow
def test_flat_limit_of_gaussian_matrix():
    """eq. (defA) with Gaussians at eps -> 0 tends to the polynomial matrix."""
    K = 8
    Pm = stencil.stencil_points_mp(K, 12, 10)
    rows = [0, 9, 27, 63, 64 + 5, 64 + 70, 64 + 143]
    with mp.workdps(60):
        A0 = stencil.interp_matrix_mp(K, 12, 10, dps=60)
    errs = []
    for eps, dps in ((2e-2, 90), (4e-3, 110)):
        Ag = stencil.gaussian_interp_matrix_mp([Pm[r] for r in rows], Pm[-66:], eps, dps)
        e = max(abs(float(Ag[i, j] - A0[r, j])) for i, r in enumerate(rows) for j in range(66))
        errs.append(e)
    # O(eps^2) convergence to the flat limit
    assert errs[1] < errs[0]
    ratio = errs[0] / errs[1]
    assert 15.0 < ratio < 40.0, (errs, ratio)
    assert errs[1] < 1e-3
