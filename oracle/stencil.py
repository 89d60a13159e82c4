"""Universal extension stencil and interpolation matrix (oracle only).

Section 3.2: for a cut square S of side L the extension square Sbar has side
3L and the same centre.  The stencil is X = X_S u X_Sbar u G, where X_S is the
K x K first-kind grid on S, X_Sbar the Kbar x Kbar first-kind grid on Sbar and
G the N_G Gaussian support nodes.  All coordinates here are in the reference
frame of Sbar, [-1,1]^2, so S = [-1/3, 1/3]^2.

Ordering (a convention shared with the caller through the input layout):
X_S row-major (x index major), then X_Sbar row-major, then G.

Readings of the paper taken here:
* G: the paper only says the nodes come from a near-uniform triangulation and
  that N_G = 66 (Sections 3.2, 6).  66 = dim P_10, and a unisolvent choice is
  the Padua points of degree 10 (first family, j-major order).
* Interpolation matrix, eq. (defA): A_{X,G} = Phi_{X,G} Phi_{G,G}^{-1} with
  Gaussian Phi.  The paper evaluates it with RBF-QR at eps ~ 1e-5 on the unit
  box; in the flat limit eps -> 0 it tends to the polynomial interpolant on G
  of total degree 10, A = P_X P_G^{-1} for any basis of P_10.  The oracle uses
  that limit, computed in extended precision with the Chebyshev product basis
  T_m(x) T_n(y), m + n <= 10.  ``gaussian_interp_matrix_mp`` evaluates the
  finite-eps Gaussian form directly so a test can pin the limit.
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

from . import cheb


def padua_points(n):
    """Padua points of degree n: (cos(j pi/n), cos(k pi/(n+1))), 0<=j<=n,
    0<=k<=n+1, j+k even; (n+1)(n+2)/2 points, j-major."""
    pts = []
    for j in range(n + 1):
        for k in range(n + 2):
            if (j + k) % 2 == 0:
                pts.append((np.cos(j * np.pi / n), np.cos(k * np.pi / (n + 1))))
    return np.array(pts)


def padua_points_mp(n):
    pts = []
    for j in range(n + 1):
        for k in range(n + 2):
            if (j + k) % 2 == 0:
                pts.append((mp.cos(j * mp.pi / n), mp.cos(k * mp.pi / (n + 1))))
    return pts


def _cheb_nodes_mp(K):
    return [-mp.cos((2 * k - 1) * mp.pi / (2 * K)) for k in range(1, K + 1)]


def stencil_points_mp(K, Kbar, deg):
    t = _cheb_nodes_mp(K)
    tb = _cheb_nodes_mp(Kbar)
    pts = [(t[a] / 3, t[b] / 3) for a in range(K) for b in range(K)]
    pts += [(tb[a], tb[b]) for a in range(Kbar) for b in range(Kbar)]
    pts += padua_points_mp(deg)
    return pts


def stencil_points(K, Kbar=12, deg=10):
    """|X| x 2 array of stencil points in Sbar reference coordinates."""
    t = cheb.nodes(K)
    tb = cheb.nodes(Kbar)
    xs = np.array([(t[a] / 3.0, t[b] / 3.0) for a in range(K) for b in range(K)])
    xb = np.array([(tb[a], tb[b]) for a in range(Kbar) for b in range(Kbar)])
    return np.vstack([xs, xb, padua_points(deg)])


def total_degree_basis(deg):
    return [(m, n) for m in range(deg + 1) for n in range(deg + 1 - m)]


def _T_mp(m, x):
    # three-term recurrence in mp arithmetic
    if m == 0:
        return mp.mpf(1)
    a, b = mp.mpf(1), x
    for _ in range(m - 1):
        a, b = b, 2 * x * b - a
    return b


def poly_vander_mp(pts, deg):
    basis = total_degree_basis(deg)
    M = mp.matrix(len(pts), len(basis))
    for i, (x, y) in enumerate(pts):
        Tx = [_T_mp(m, x) for m in range(deg + 1)]
        Ty = [_T_mp(m, y) for m in range(deg + 1)]
        for j, (m, n) in enumerate(basis):
            M[i, j] = Tx[m] * Ty[n]
    return M


@lru_cache(maxsize=8)
def interp_matrix_mp(K, Kbar=12, deg=10, dps=50):
    """A_{X,G} = P_X P_G^{-1} (flat Gaussian limit) as an mp.matrix."""
    with mp.workdps(dps):
        pts = stencil_points_mp(K, Kbar, deg)
        nG = (deg + 1) * (deg + 2) // 2
        P = poly_vander_mp(pts, deg)
        PG = P[len(pts) - nG:, :]
        # A P_G = P_X  =>  A = P_X P_G^{-1}
        return P * mp.inverse(PG)


@lru_cache(maxsize=8)
def interp_matrix(K, Kbar=12, deg=10):
    """float64 copy of the flat-limit A_{X,G} (rows: stencil points)."""
    A = interp_matrix_mp(K, Kbar, deg)
    return np.array(A.tolist(), dtype=np.float64)


def gaussian_interp_matrix_mp(pts_X, pts_G, eps, dps):
    """A = Phi_{X,G} Phi_{G,G}^{-1} for Gaussians exp(-eps^2 |x-c|^2),
    evaluated directly in dps-digit arithmetic (eq. defA)."""
    with mp.workdps(dps):
        e2 = mp.mpf(eps) ** 2

        def phi(p, c):
            return mp.exp(-e2 * ((p[0] - c[0]) ** 2 + (p[1] - c[1]) ** 2))

        nX, nG = len(pts_X), len(pts_G)
        PX = mp.matrix(nX, nG)
        PG = mp.matrix(nG, nG)
        for i in range(nX):
            for j in range(nG):
                PX[i, j] = phi(pts_X[i], pts_G[j])
        for i in range(nG):
            for j in range(nG):
                PG[i, j] = phi(pts_G[i], pts_G[j])
        return PX * mp.inverse(PG)
