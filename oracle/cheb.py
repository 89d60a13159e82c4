"""First-kind Chebyshev grids (test infrastructure; oracle only).

The paper samples f on tensor-product Chebyshev grids of the first kind on
every leaf (Section 4; first-kind nodes, so no node lies on a leaf edge).
Plain definitions:

* nodes  t_k = -cos((2k-1) pi / (2K)), k = 1..K  (ascending on (-1,1));
* T_m(t) = cos(m arccos t);
* coefficients of the degree-(K-1) interpolant through (t_k, g_k):
  c_m = (2/K) sum_k g_k T_m(t_k), with c_0 halved (discrete orthogonality of
  T_0..T_{K-1} on the first-kind nodes).
"""
import numpy as np


def nodes(K):
    k = np.arange(1, K + 1)
    return -np.cos((2 * k - 1) * np.pi / (2 * K))


def T(m, t):
    """Chebyshev polynomial T_m at t (|t| <= 1 via cos/arccos, else cosh)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty(np.broadcast(t, m).shape)
    inside = np.abs(t) <= 1.0
    mt = np.broadcast_to(m, out.shape)
    tt = np.broadcast_to(t, out.shape)
    out[inside] = np.cos(mt[inside] * np.arccos(tt[inside]))
    o = ~inside
    out[o] = np.sign(tt[o]) ** mt[o] * np.cosh(mt[o] * np.arccosh(np.abs(tt[o])))
    return out


def vander(t, deg):
    """Matrix [T_0(t) ... T_deg(t)] (rows = points), by the three-term recurrence."""
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    V = np.empty((t.size, deg + 1))
    V[:, 0] = 1.0
    if deg >= 1:
        V[:, 1] = t
    for m in range(2, deg + 1):
        V[:, m] = 2.0 * t * V[:, m - 1] - V[:, m - 2]
    return V


def coef_matrix(K):
    """C with c = C g: 1D values at the K first-kind nodes -> coefficients."""
    t = nodes(K)
    C = (2.0 / K) * vander(t, K - 1).T
    C[0, :] *= 0.5
    return C


def coeffs2d(G):
    """2D coefficients c[a, b] of the tensor interpolant of values G[i, j]
    (i indexes x, j indexes y) on the K x K first-kind grid."""
    K = G.shape[0]
    C = coef_matrix(K)
    return C @ G @ C.T


def eval2d(c, x, y):
    """Evaluate sum_ab c[a,b] T_a(x) T_b(y) at matching arrays x, y."""
    Vx = vander(x, c.shape[0] - 1)
    Vy = vander(y, c.shape[1] - 1)
    return np.einsum("pa,ab,pb->p", Vx, c, Vy)


def fejer1_weights(K):
    """Weights of the K-point first-kind (Fejer) rule on [-1,1]:
    the exact integrals of the Lagrange basis of the first-kind nodes."""
    # integrate the interpolant exactly: int_{-1}^{1} T_m = 2/(1-m^2) for even m, 0 odd
    I = np.zeros(K)
    for m in range(0, K, 2):
        I[m] = 2.0 / (1.0 - m * m)
    return coef_matrix(K).T @ I
