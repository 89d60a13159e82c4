"""Pins for the oracle's cut-leaf extension (CPU).

* Polynomial reproduction: for f of total degree <= 10 the extension equals f
  on every square of the list of a full-rank cut leaf, up to the
  conditioning bound c * u * ||B|| * ||f_I|| (B = composite extension
  operator); degree 11 is not reproduced (negative control).
* Flat-limit identity (reading R1): with full rank, the values on Xbar^E equal
  the degree-10 least-squares polynomial fit to the interior samples, whatever
  the support nodes G are.
* Rank-deficient leaves (N_I < 66): f_G is the minimum-norm solution
  (consistent and in the row space of A_I).
* The float64 route agrees with the extended-precision route within the
  forward-error bound of a backward-stable least-squares solve,
  16 u cond(A_I) max|values|.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import extension, geometry, stencil
from workloads import Disk

U = 2.0 ** -53
K = 8


@pytest.fixture(scope="module")
def disk3():
    n = 8
    lv = [3] * (n * n)
    ix = [a for a in range(n) for b in range(n)]
    iy = [b for a in range(n) for b in range(n)]
    t = geometry.Tree(lv, ix, iy, (0.0, 0.0, 2.0))
    d = Disk(0.6)
    cx, cy = t.centers()
    kinds = d.classify_boxes(cx, cy, t.h())
    cuts = [i for i in range(t.n) if kinds[i] == 2]
    masks = geometry.cut_masks(t, cuts, d, K)
    return t, kinds, cuts, masks


def _inputs(t, cuts, fun):
    X, Y = t.leaf_nodes(K)
    fl = fun(X, Y)
    fc = np.zeros((len(cuts), K * K + 144 + 66))
    for r, i in enumerate(cuts):
        sx, sy = geometry.stencil_world(t, i, K)
        fc[r] = fun(sx, sy)
    return X, Y, fl, fc


def _pick(masks, cuts, n_int):
    for r, i in enumerate(cuts):
        if masks[r].sum() == n_int:
            return i
    raise AssertionError(n_int)


def poly10(x, y):
    return 1.0 + 0.7 * x ** 3 * y ** 7 - 0.5 * x ** 10 + 2.0 * y ** 4 * x ** 2 - 0.3 * y ** 9


@pytest.mark.slow
def test_polynomial_reproduction_and_negative_control(disk3):
    t, kinds, cuts, masks = disk3
    sel = [_pick(masks, cuts, 135), _pick(masks, cuts, 107)]
    X, Y, fl, fc = _inputs(t, cuts, poly10)
    fe, info = extension.extend(t, kinds, fl, fc, masks, K, precision="mp", cut_ids=sel,
                                want_operator_norms=True)
    for i in sel:
        tg = info[i]["targets"]
        assert info[i]["rank"] == 66
        fI = np.abs(fc[cuts.index(i)][masks[cuts.index(i)]]).max()
        bound = 64 * U * info[i]["op_norm_inf"] * fI
        err = np.abs(fe[tg] - poly10(X[tg], Y[tg])).max()
        assert err <= bound, (i, err, bound)
    # degree 11 (T_6 T_5 in the frame of Sbar) is not reproduced on the
    # well-conditioned leaf
    cx, cy = t.centers()
    i0 = sel[0]
    s = 1.5 * t.h()[i0]

    def p11(x, y):
        xi, eta = (x - cx[i0]) / s, (y - cy[i0]) / s
        return poly10(x, y) + np.cos(6 * np.arccos(np.clip(xi, -1, 1))) * \
            np.cos(5 * np.arccos(np.clip(eta, -1, 1)))

    X, Y, fl, fc = _inputs(t, cuts, p11)
    fe, info = extension.extend(t, kinds, fl, fc, masks, K, precision="mp", cut_ids=sel[:1])
    tg = info[i0]["targets"]
    assert np.abs(fe[tg] - p11(X[tg], Y[tg])).max() > 1e-2


@pytest.mark.slow
def test_flat_limit_identity_and_min_norm(disk3):
    t, kinds, cuts, masks = disk3
    A = stencil.interp_matrix_mp(K)
    with mp.workdps(50):
        pts = stencil.stencil_points_mp(K, 12, 10)
    rng = np.random.default_rng(3)
    for n_int in (135, 62):
        i = _pick(masks, cuts, n_int)
        m = masks[cuts.index(i)]
        I = np.nonzero(m)[0]
        fI = rng.standard_normal(I.size)
        with mp.workdps(40):
            AI = [[A[int(k), c] for c in range(66)] for k in I]
            fG, rank = extension.pinv_apply_mp(AI, fI, 66)
            ext_rows = [64 + a for a in range(144) if not m[64 + a]]
            g = [mp.fdot([A[k, c] for c in range(66)], fG) for k in ext_rows]
            if n_int >= 66:
                assert rank == 66
                # direct LS fit in the total-degree-10 Chebyshev basis, no G
                P = stencil.poly_vander_mp([pts[int(k)] for k in I], 10)
                Prows = [[P[r, c] for c in range(66)] for r in range(P.rows)]
                cf, r2 = extension.pinv_apply_mp(Prows, fI, 66)
                Pe = stencil.poly_vander_mp([pts[k] for k in ext_rows], 10)
                g2 = [mp.fdot([Pe[r, c] for c in range(66)], cf) for r in range(len(ext_rows))]
                scale = max(abs(v) for v in g)
                assert max(abs(a - b) for a, b in zip(g, g2)) < 1e-20 * max(scale, 1)
            else:
                assert rank == n_int
                # consistent: A_I f_G = f_I
                res = max(abs(mp.fdot(row, fG) - mp.mpf(float(v))) for row, v in zip(AI, fI))
                assert res < mp.mpf(10) ** -20
                # minimum norm: f_G lies in the row space of A_I, i.e. it is
                # orthogonal to every null vector; test against random null
                # vectors built as (I - A_I^+ A_I) z
                for _ in range(2):
                    z = [mp.mpf(float(v)) for v in rng.standard_normal(66)]
                    Az = [mp.fdot(row, z) for row in AI]
                    pz, _ = extension.pinv_apply_mp(AI, Az, 66)
                    nz = [a - b for a, b in zip(z, pz)]
                    nrm = mp.sqrt(mp.fdot(nz, nz))
                    assert nrm > 1e-3
                    assert abs(mp.fdot(nz, fG)) < mp.mpf(10) ** -20 * nrm * mp.sqrt(mp.fdot(fG, fG))


@pytest.mark.slow
def test_fp64_route_within_conditioning_bound(disk3):
    t, kinds, cuts, masks = disk3
    sel = [_pick(masks, cuts, 137), _pick(masks, cuts, 64)]

    def fun(x, y):
        r2 = (x - 0.1) ** 2 + (y + 0.2) ** 2
        return (4 * r2 / 0.05 ** 2 - 4 / 0.05) * np.exp(-r2 / 0.05)

    X, Y, fl, fc = _inputs(t, cuts, fun)
    fm, info = extension.extend(t, kinds, fl, fc, masks, K, precision="mp", cut_ids=sel,
                                want_operator_norms=True)
    fd, _ = extension.extend(t, kinds, fl, fc, masks, K, precision="fp64", cut_ids=sel)
    for i in sel:
        tg = info[i]["targets"]
        fI = fc[cuts.index(i)][masks[cuts.index(i)]]
        tol = extension.extension_tolerance(info[i], fm[tg], fI)
        err = np.abs(fm[tg] - fd[tg]).max()
        assert err <= tol, (i, err, tol)
        # the float64 route is not exact: its error is visible
        assert err > 0.0
    # leaves outside every list: regular copied, exterior zero
    own, _ = geometry.extension_owner(t, kinds)
    for j in range(t.n):
        if kinds[j] == 1:
            assert np.array_equal(fd[j], fl[j])
        elif own[j] < 0:
            assert not fd[j].any()
