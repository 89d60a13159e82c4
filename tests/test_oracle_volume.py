"""Pins for the oracle's volume-potential quadrature (CPU).

Each check fixes the result by something other than the quadrature itself:
* constant density: the closed-form antiderivative of log(x^2 + y^2),
  F(x,y) = xy log(x^2+y^2) - 3xy + x^2 atan(y/x) + y^2 atan(x/y);
* polynomial density on one box: mpmath tanh-sinh quadrature split at the
  target (brute force in 20-digit arithmetic); for K = 8 and 16 and targets
  on every branch of the oracle (inside, near an edge, off a corner, at the
  far-rule threshold), a semi-analytic reference: the y2 integral in closed
  form, the y1 integral by tanh-sinh in 30-digit arithmetic;
* the Gauss-Legendre rules: exact on monomials, and equal to numpy's
  independent implementation;
* radial source f = Laplacian(u) with u a narrow Gaussian: Newton's theorem
  gives V = u up to the leaf interpolation error of f;
* scaling: V_s(s x) = s^2 V_1(x) + s^2 log(s) int f / (2 pi);
* symmetry: rotating the data by 90 degrees rotates the potential;
* the potential satisfies Laplacian(V) = f inside a leaf (loose, spectral).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import cheb, geometry, volume


def F(x, y):
    r2 = x * x + y * y
    t1 = x * y * math.log(r2) if r2 > 0 else 0.0
    t3 = x * x * math.atan(y / x) if x != 0 else 0.0
    t4 = y * y * math.atan(x / y) if y != 0 else 0.0
    return t1 - 3 * x * y + t3 + t4


def v_const(X, Y, a, b, c, d):
    return (F(b - X, d - Y) - F(a - X, d - Y) - F(b - X, c - Y) + F(a - X, c - Y)) / (4 * math.pi)


def small_adaptive_tree():
    # level-2 grid with two leaves refined (balanced)
    lv, ix, iy = [], [], []
    for a in range(4):
        for b in range(4):
            if (a, b) in ((1, 1), (2, 1)):
                for dx in (0, 1):
                    for dy in (0, 1):
                        lv.append(3), ix.append(2 * a + dx), iy.append(2 * b + dy)
            else:
                lv.append(2), ix.append(a), iy.append(b)
    return geometry.Tree(lv, ix, iy, (0.1, -0.05, 2.0))


def test_gauss_legendre_rule():
    for q in (1, 2, 5, 12, 24, 32, 48):
        x, w = volume.gauss_legendre(q)
        for k in range(2 * q):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(np.dot(w, x ** k) - exact) < 1e-14
        xn, wn = np.polynomial.legendre.leggauss(q)
        # numpy's weights carry up to ~5e-14 relative error at q = 48
        assert np.abs(x - xn).max() <= 2e-16 and np.abs(w - wn).max() <= 1e-13 * wn.max()


def test_constant_density_closed_form():
    t = small_adaptive_tree()
    K = 6
    assert t.check_partition() and t.is_balanced()
    rng = np.random.default_rng(0)
    on = rng.random(t.n) < 0.6
    fe = np.zeros((t.n, K * K))
    fe[on] = 1.0
    X, Y = t.leaf_nodes(K)
    pick = rng.choice(t.n * K * K, 40, replace=False)
    tx, ty = X.ravel()[pick], Y.ravel()[pick]
    # also a few points on box edges/corners and far away
    tx = np.concatenate([tx, [0.1, -0.4, 3.0, 0.6]])
    ty = np.concatenate([ty, [-0.05, 0.45, -2.0, -0.55]])
    v = volume.potential(t, fe, K, tx, ty)
    cx, cy = t.centers()
    h = t.h()
    ex = np.zeros(tx.size)
    for i in np.nonzero(on)[0]:
        a, b = cx[i] - h[i] / 2, cx[i] + h[i] / 2
        c, d = cy[i] - h[i] / 2, cy[i] + h[i] / 2
        ex += np.array([v_const(x, y, a, b, c, d) for x, y in zip(tx, ty)])
    assert np.abs(v - ex).max() < 2e-15 * max(1.0, np.abs(ex).max())


@pytest.mark.slow
def test_polynomial_density_brute_force():
    K = 4
    rng = np.random.default_rng(1)
    c = rng.standard_normal((K, K))
    tgt = (0.13, -0.21)     # inside the box [-0.5,0.5]^2

    def p(x, y):
        tx = [mp.mpf(1), 2 * x]
        ty = [mp.mpf(1), 2 * y]
        for _ in range(2, K):
            tx.append(4 * x * tx[-1] - tx[-2])
            ty.append(4 * y * ty[-1] - ty[-2])
        return sum(c[a, b] * tx[a] * ty[b] for a in range(K) for b in range(K))

    with mp.workdps(18):
        f = lambda x, y: mp.log((x - tgt[0]) ** 2 + (y - tgt[1]) ** 2) / 2 * p(x, y)  # noqa: E731
        ref = float(mp.quad(f, [-0.5, tgt[0], 0.5], [-0.5, tgt[1], 0.5]) / (2 * mp.pi))
    v = volume.potential_boxes([tgt[0]], [tgt[1]], [0.0], [0.0], [1.0], c[None], K)[0]
    assert abs(v - ref) < 1e-15


def _semi_analytic(c, K, cx, cy, h, tx, ty, dps=30):
    """(1/2 pi) int_B log|t - y| p(y) dy for the box B of centre (cx, cy)
    and side h and p = sum c[a, b] T_a(xi) T_b(eta).  With s = y2 - t2 and
    u = y1 - t1, p is a polynomial sum_k e_k(y1) s^k (T_b(alpha s + beta)
    expanded in monomials), and
      M_k(u) = int log(u^2 + s^2) s^k ds
             = [s^(k+1) log(u^2 + s^2)] / (k+1) - 2 A_(k+2)(u) / (k+1),
      A_m(u) = int s^m / (u^2 + s^2) ds = int s^(m-2) ds - u^2 A_(m-2)(u),
      A_0 = (atan(s1/u) - atan(s0/u)) / u,  A_1 = log((u^2+s1^2)/(u^2+s0^2)) / 2,
    so the y2 integral is closed-form and only the y1 integral is numerical
    (tanh-sinh, split at t1 when it lies over the box)."""
    with mp.workdps(dps):
        cx, cy, h, tx, ty = (mp.mpf(float(v)) for v in (cx, cy, h, tx, ty))
        x0, x1 = cx - h / 2, cx + h / 2
        s0, s1 = cy - h / 2 - ty, cy + h / 2 - ty
        al, be = 2 / h, 2 * (ty - cy) / h
        Tm = [[mp.mpf(1)], [be, al]]  # monomial coefficients of T_b(al s + be)
        for b in range(2, K):
            nxt = [mp.mpf(0)] * (b + 1)
            for k, v in enumerate(Tm[-1]):
                nxt[k] += 2 * be * v
                nxt[k + 1] += 2 * al * v
            for k, v in enumerate(Tm[-2]):
                nxt[k] -= v
            Tm.append(nxt)
        cm = [[mp.mpf(float(c[a, b])) for b in range(K)] for a in range(K)]

        def inner(y1):
            u2 = (y1 - tx) ** 2
            xi = 2 * (y1 - cx) / h
            Ta = [mp.mpf(1), xi]
            for _ in range(2, K):
                Ta.append(2 * xi * Ta[-1] - Ta[-2])
            g = [mp.fsum(cm[a][b] * Ta[a] for a in range(K)) for b in range(K)]
            e = [mp.fsum(g[b] * Tm[b][k] for b in range(k, K)) for k in range(K)]
            u = mp.sqrt(u2)
            A = [(mp.atan(s1 / u) - mp.atan(s0 / u)) / u, mp.log((u2 + s1 ** 2) / (u2 + s0 ** 2)) / 2]
            for m in range(2, K + 2):
                A.append((s1 ** (m - 1) - s0 ** (m - 1)) / (m - 1) - u2 * A[m - 2])
            L1, L0 = mp.log(u2 + s1 ** 2), mp.log(u2 + s0 ** 2)
            M = [(s1 ** (k + 1) * L1 - s0 ** (k + 1) * L0) / (k + 1) - 2 * A[k + 2] / (k + 1) for k in range(K)]
            return mp.fsum(e[k] * M[k] for k in range(K)) / 2

        pts = [x0, tx, x1] if x0 < tx < x1 else [x0, x1]
        return float(mp.quad(inner, pts) / (2 * mp.pi))


@pytest.mark.parametrize("K", [8, 16])
def test_polynomial_density_every_branch(K):
    """Degree-(K-1) polynomial density on one box, targets inside it, near
    an edge (distance 0.3 h and 0.999 h: the graded near rule), off a corner
    (0.18 h) and at the far-rule threshold (distance exactly h: the tensor
    rule), against the semi-analytic reference to 1e-14."""
    rng = np.random.default_rng(K)
    c = rng.standard_normal((K, K)) / (1.0 + np.add.outer(np.arange(K), np.arange(K)))
    cx, cy, h = 0.1, -0.2, 0.5
    targets = {"inside": (cx + 0.13 * h, cy - 0.21 * h), "near": (cx + 0.1 * h, cy + 0.8 * h),
               "near_edge": (cx - 1.499 * h, cy + 0.3 * h), "corner": (cx + 0.65 * h, cy + 0.6 * h),
               "far_threshold": (cx + 0.2 * h, cy - 1.5 * h)}
    for name, (tx, ty) in targets.items():
        ref = _semi_analytic(c, K, cx, cy, h, tx, ty)
        v = volume.potential_boxes([tx], [ty], [cx], [cy], [h], c[None], K)[0]
        assert abs(v - ref) <= 1e-14 * max(1.0, abs(ref)), (name, v, ref)


def test_radial_gaussian_newton():
    # u = exp(-r^2/w) centred in the root; f = Lap u has zero net charge and
    # decays, so V = u (to the piecewise-polynomial resolution of f)
    w = 0.01
    K = 16
    d = 4
    n = 2 ** d
    lv = [d] * (n * n)
    ix = [a for a in range(n) for b in range(n)]
    iy = [b for a in range(n) for b in range(n)]
    t = geometry.Tree(lv, ix, iy, (0.03, -0.02, 2.0))
    X, Y = t.leaf_nodes(K)
    x0, y0 = 0.0, 0.0
    r2 = (X - x0) ** 2 + (Y - y0) ** 2
    fe = (4 * r2 / w ** 2 - 4 / w) * np.exp(-r2 / w)
    fe[np.abs(fe).max(axis=1) < 1e-30] = 0.0
    rng = np.random.default_rng(2)
    tx = rng.uniform(-0.3, 0.3, 12)
    ty = rng.uniform(-0.3, 0.3, 12)
    v = volume.potential(t, fe, K, tx, ty)
    u = np.exp(-((tx - x0) ** 2 + (ty - y0) ** 2) / w)
    assert np.abs(v - u).max() < 1e-8


def test_scaling_and_rotation():
    K = 8
    rng = np.random.default_rng(5)
    coef = rng.standard_normal((3, K, K)) / (1 + np.add.outer(np.arange(K), np.arange(K))) ** 2
    cx = np.array([0.0, 1.0, 0.0])
    cy = np.array([0.0, 0.0, 1.0])
    h = np.ones(3)
    tx = np.array([0.1, 0.7, -0.3, 0.45])
    ty = np.array([0.2, -0.1, 0.9, 0.45])
    v1 = volume.potential_boxes(tx, ty, cx, cy, h, coef, K)
    s = 0.37
    vs = volume.potential_boxes(s * tx, s * ty, s * cx, s * cy, s * h, coef, K)
    w = cheb.fejer1_weights(K)
    charge = sum(np.einsum("i,ab,ai,bj,j->", w, coef[k], cheb.vander(cheb.nodes(K), K - 1).T,
                           cheb.vander(cheb.nodes(K), K - 1).T, w) / 4.0 for k in range(3))
    assert np.abs(vs - (s * s * v1 + s * s * math.log(s) * charge / (2 * math.pi))).max() < 1e-15
    # rotation by 90 degrees: (x, y) -> (-y, x); T_b(eta) with eta -> -eta
    # multiplies c[a, b] by (-1)^b and swaps the axes
    sign = (-1.0) ** np.arange(K)
    crot = np.stack([(coef[k] * sign[None, :]).T for k in range(3)])
    vr = volume.potential_boxes(-ty, tx, -cy, cx, h, crot, K)
    assert np.abs(vr - v1).max() < 1e-15


def test_laplacian_of_potential_is_density():
    # V from one box at its own interior nodes; spectral Laplacian of the
    # leaf interpolant of V approximates f (V is smooth inside the box)
    K = 12
    rng = np.random.default_rng(7)
    c = np.zeros((K, K))
    c[:3, :3] = rng.standard_normal((3, 3))
    hbox = 0.5
    t = cheb.nodes(K)
    # sample V on a small box strictly inside the source box
    hs = 0.1
    tx = (hs / 2 * t)[:, None] + 0.0 * t[None, :]
    ty = 0.0 * t[:, None] + (hs / 2 * t)[None, :]
    v = volume.potential_boxes(tx.ravel(), ty.ravel(), [0.0], [0.0], [hbox], c[None], K)
    cv = cheb.coeffs2d(v.reshape(K, K))
    # second derivatives of the Chebyshev series on [-hs/2, hs/2]
    D = np.zeros((K, K))
    for m in range(K):
        for j in range(m - 1, -1, -2):
            D[j, m] = 2.0 * m
    D[0, :] *= 0.5
    D2 = (D @ D) * (2.0 / hs) ** 2
    lap = D2 @ cv + cv @ D2.T
    lapv = cheb.eval2d(lap, np.array([0.0]), np.array([0.0]))[0]
    f0 = cheb.eval2d(c, np.array([0.0]), np.array([0.0]))[0]
    assert abs(lapv - f0) < 1e-6 * max(1.0, abs(f0))


def test_net_charge_closed_forms():
    """The oracle's net charge (integral of the leaf data over the tree):
    f = 1 gives the root's area; f = x^3 y^2 (degree below K in each
    variable, so every leaf interpolant is f itself) gives the product of
    the one-dimensional integrals; a Gaussian gives its erf closed form up
    to the leaf interpolation error; two right-hand sides are summed apart."""
    t = small_adaptive_tree()
    K = 6
    X, Y = t.leaf_nodes(K)
    x0, x1 = t.cx0 - 0.5 * t.size, t.cx0 + 0.5 * t.size
    y0, y1 = t.cy0 - 0.5 * t.size, t.cy0 + 0.5 * t.size
    one = volume.net_charge(t, np.ones_like(X), K)
    assert abs(one[0] - t.size ** 2) <= 1e-15 * t.size ** 2
    poly = volume.net_charge(t, X ** 3 * Y ** 2, K)[0]
    exact = (x1 ** 4 - x0 ** 4) / 4 * (y1 ** 3 - y0 ** 3) / 3
    assert abs(poly - exact) <= 1e-14 * abs(exact)
    # x^K is not integrated exactly by the rule on one leaf: the check is sharp
    bad = volume.net_charge(t, X ** (2 * K), K)[0]
    assert abs(bad - (x1 ** (2 * K + 1) - x0 ** (2 * K + 1)) / (2 * K + 1) * t.size) > 1e-10
    # a Gaussian on a finer uniform tree (K = 16, level 3)
    lv = np.full(64, 3)
    ix, iy = np.divmod(np.arange(64), 8)
    u = geometry.Tree(lv, ix, iy, (0.0, 0.0, 2.0))
    K = 16
    X, Y = u.leaf_nodes(K)
    cx, cy, beta = 0.13, -0.21, 0.05
    g = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / beta)
    sb = math.sqrt(beta)
    ex = math.sqrt(math.pi) * sb / 2 * (math.erf((1 - cx) / sb) - math.erf((-1 - cx) / sb))
    ey = math.sqrt(math.pi) * sb / 2 * (math.erf((1 - cy) / sb) - math.erf((-1 - cy) / sb))
    two = volume.net_charge(u, np.stack([g, -2.0 * g]), K)
    assert abs(two[0] - ex * ey) <= 1e-12 * ex * ey
    assert two[1] == -2.0 * two[0]  # scaling by 2 is exact
