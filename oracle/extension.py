"""Cut-leaf extension of f (oracle only; Sections 3.2 and 4.1).

For every cut leaf S, in the paper's order of operations:

1. Interior stencil points X^I of X = X_S u X_Sbar u G (mask = inside test).
2. f_G = A_{X^I,G}^+ f_{X^I}: minimum-norm least squares through the
   pseudo-inverse of the interior rows of the universal matrix A_{X,G}.
   Singular values below 1e-13 * sigma_max count as zero (the paper does not
   say how rank deficiency is treated; cut leaves with fewer than N_G interior
   stencil points are rank deficient by construction).
3. Values on the Kbar x Kbar grid of Sbar: the given data at interior nodes,
   A_{X_Sbar^E,G} f_G at exterior nodes.
4. The (Kbar-1)-th total-order Chebyshev expansion on Sbar, eq. (chebexpbarS):
   tensor interpolation on the first-kind grid, then coefficients with
   m + n >= Kbar dropped.
5. That expansion evaluated on the K x K grid of every square in the
   extension list of S (S itself included; its interior samples are
   overwritten too).

Regular leaves keep their data; exterior leaves in no list get zero.

``precision='mp'`` does steps 2-5 in mpmath (40 digits; the pseudo-inverse by
the normal equations of the full-rank side, or by an eigen-decomposition when
the cutoff bites); ``precision='fp64'`` uses numpy's SVD-based pinv and plain
float64 for the rest.
"""
import mpmath as mp
import numpy as np

from . import cheb
from . import stencil
from .geometry import extension_owner

REL_CUT = 1e-13


def _mp_gram(rows_a, rows_b):
    """Gram-type product sum_k a[k][i] b[k][j] for lists of mp rows."""
    n = len(rows_a[0])
    m = len(rows_b[0])
    cols_a = [[r[i] for r in rows_a] for i in range(n)]
    cols_b = cols_a if rows_a is rows_b else [[r[j] for r in rows_b] for j in range(m)]
    G = mp.matrix(n, m)
    for i in range(n):
        for j in range(m):
            if cols_b is cols_a and j < i:
                G[i, j] = G[j, i]
            else:
                G[i, j] = mp.fdot(cols_a[i], cols_b[j])
    return G


def pinv_apply_mp(AI_rows, fI, nG, dps=40):
    """f_G = A_I^+ f_I in mp arithmetic; AI_rows is a list of N_I rows of
    length nG.  Returns (f_G as list of mpf, numerical rank)."""
    with mp.workdps(dps):
        NI = len(AI_rows)
        if NI == 0:
            return [mp.mpf(0)] * nG, 0
        fI = [mp.mpf(v) for v in fI]
        if NI >= nG:
            Gm = _mp_gram(AI_rows, AI_rows)                      # A^T A, nG x nG
            rhs = mp.matrix([mp.fdot([r[i] for r in AI_rows], fI) for i in range(nG)])
            try:
                Gi = mp.inverse(Gm)
                cond = mp.norm(Gm, 1) * mp.norm(Gi, 1)
            except ZeroDivisionError:
                cond = mp.inf
            if cond * nG < mp.mpf(REL_CUT) ** -2:
                x = Gi * rhs
                return [x[i] for i in range(nG)], nG
        # general route: eigen-decomposition of A^T A with the cutoff
        Gm = _mp_gram(AI_rows, AI_rows)
        E, Q = mp.eigsy(Gm)
        lmax = max(abs(E[i]) for i in range(nG))
        keep = [i for i in range(nG) if E[i] > (mp.mpf(REL_CUT) ** 2) * lmax]
        rhs = [mp.fdot([r[i] for r in AI_rows], fI) for i in range(nG)]
        x = [mp.mpf(0)] * nG
        for k in keep:
            qk = [Q[i, k] for i in range(nG)]
            c = mp.fdot(qk, rhs) / E[k]
            for i in range(nG):
                x[i] += c * qk[i]
        return x, len(keep)


def _tcoef_mp(Kbar):
    t = [-mp.cos((2 * k - 1) * mp.pi / (2 * Kbar)) for k in range(1, Kbar + 1)]
    C = [[(mp.mpf(2) / Kbar) * mp.cos(m * mp.acos(t[j])) for j in range(Kbar)] for m in range(Kbar)]
    C[0] = [c / 2 for c in C[0]]
    return C


def _cheb_vals_mp(x, deg):
    v = [mp.mpf(1), x]
    for _ in range(2, deg + 1):
        v.append(2 * x * v[-1] - v[-2])
    return v[:deg + 1]


def extend(tree, kinds, f_leaf, f_cut, masks, K, Kbar=12, deg=10, precision="mp",
           cut_ids=None, want_operator_norms=False):
    """Extended data f^e on every leaf, shape (L, K*K).

    tree     oracle.geometry.Tree
    kinds    per leaf: 0 exterior, 1 regular, 2 cut
    f_leaf   (L, K*K) samples of f on regular leaves (other rows ignored)
    f_cut    (n_cut, |X|) samples of f at the stencil points of each cut leaf
             (canonical order = ascending leaf index); exterior entries ignored
    masks    (n_cut, |X|) interior flags
    cut_ids  optional subset of cut leaves to process (others left as NaN)
    """
    kinds = np.asarray(kinds)
    L = tree.n
    n = K * K
    nG = (deg + 1) * (deg + 2) // 2
    nSbar = Kbar * Kbar
    all_cuts = [i for i in range(L) if kinds[i] == 2]
    owner, viol = extension_owner(tree, kinds)
    if viol:
        raise ValueError(f"extension restriction violated: {viol[:5]}")
    lists = {i: [] for i in all_cuts}
    for j in range(L):
        if owner[j] >= 0:
            lists[int(owner[j])].append(j)
    fe = np.zeros((L, n))
    reg = kinds == 1
    fe[reg] = np.asarray(f_leaf)[reg]
    todo = all_cuts if cut_ids is None else list(cut_ids)
    if cut_ids is not None:
        for i in all_cuts:
            for j in lists[i]:
                fe[j] = np.nan
    X, Y = tree.leaf_nodes(K)
    cx, cy = tree.centers()
    h = tree.h()
    info = {}
    A64 = stencil.interp_matrix(K, Kbar, deg)
    Amp = stencil.interp_matrix_mp(K, Kbar, deg) if precision == "mp" else None
    rowpos = {i: r for r, i in enumerate(all_cuts)}
    for i in todo:
        r = rowpos[i]
        m = np.asarray(masks[r], dtype=bool)
        I = np.nonzero(m)[0]
        fI = np.asarray(f_cut[r], dtype=np.float64)[I]
        sbar_rows = np.arange(n, n + nSbar)
        targets = lists[i]
        xi = np.concatenate([(X[j] - cx[i]) / (1.5 * h[i]) for j in targets])
        eta = np.concatenate([(Y[j] - cy[i]) / (1.5 * h[i]) for j in targets])
        if precision == "mp":
            with mp.workdps(40):
                AI = [[Amp[int(k), c] for c in range(nG)] for k in I]
                fG, rank = pinv_apply_mp(AI, fI, nG)
                g = []
                for a in range(nSbar):
                    k = n + a
                    if m[k]:
                        g.append(mp.mpf(float(f_cut[r][k])))
                    else:
                        g.append(mp.fdot([Amp[k, c] for c in range(nG)], fG))
                C = _tcoef_mp(Kbar)
                # coefficients c[a][b] = sum_ij C[a][i] g[i,j] C[b][j]
                Gm = [[g[ii * Kbar + jj] for jj in range(Kbar)] for ii in range(Kbar)]
                tmp = [[mp.fdot(C[a], [Gm[ii][jj] for ii in range(Kbar)]) for jj in range(Kbar)]
                       for a in range(Kbar)]
                coef = [[mp.fdot(tmp[a], C[b]) if a + b < Kbar else mp.mpf(0) for b in range(Kbar)]
                        for a in range(Kbar)]
                vals = []
                for p in range(xi.size):
                    tx = _cheb_vals_mp(mp.mpf(float(xi[p])), Kbar - 1)
                    ty = _cheb_vals_mp(mp.mpf(float(eta[p])), Kbar - 1)
                    s = mp.mpf(0)
                    for a in range(Kbar):
                        s += tx[a] * mp.fdot(coef[a][:Kbar - a], ty[:Kbar - a])
                    vals.append(float(s))
                vals = np.array(vals)
        else:
            AI = A64[I]
            P = np.linalg.pinv(AI, rcond=REL_CUT) if I.size else np.zeros((nG, 0))
            fG = P @ fI
            rank = int(np.linalg.matrix_rank(AI, tol=REL_CUT * np.linalg.norm(AI, 2))) if I.size else 0
            g = A64[sbar_rows] @ fG
            gi = m[sbar_rows]
            g[gi] = np.asarray(f_cut[r], dtype=np.float64)[sbar_rows][gi]
            coef = cheb.coeffs2d(g.reshape(Kbar, Kbar))
            aa, bb = np.meshgrid(np.arange(Kbar), np.arange(Kbar), indexing="ij")
            coef[aa + bb >= Kbar] = 0.0
            vals = cheb.eval2d(coef, xi, eta)
        for q, j in enumerate(targets):
            fe[j] = vals[q * n:(q + 1) * n]
        rec = {"n_interior": int(I.size), "rank": int(rank), "targets": list(targets),
               "cond": condition_number(A64[I])}
        if want_operator_norms:
            rec["op_norm_inf"] = composite_norm(A64, m, xi, eta, K, Kbar, deg)
        info[i] = rec
    return fe, info


def condition_number(AI):
    """2-norm condition number of A_I over the singular values that the
    pseudo-inverse keeps (sigma > 1e-13 sigma_max)."""
    if AI.shape[0] == 0:
        return 1.0
    s = np.linalg.svd(AI, compute_uv=False)
    s = s[s > REL_CUT * s[0]]
    return float(s[0] / s[-1])


def extension_tolerance(rec, fe_targets, f_interior, c=16.0):
    """Parity tolerance for the extended values of one cut leaf between two
    float64 implementations: a backward-stable least-squares solve has a
    forward error of order u * cond(A_I) relative to the solution, which the
    well-conditioned universal stages carry to the targets."""
    u = 2.0 ** -53
    scale = max(float(np.abs(fe_targets).max()), float(np.abs(f_interior).max()) if f_interior.size else 0.0)
    return c * u * rec["cond"] * scale


def composite_norm(A64, m, xi, eta, K, Kbar, deg):
    """Infinity norm of the linear map f_{X^I} -> extended values on the
    targets (float64), used to scale the extension parity tolerance."""
    n = K * K
    nSbar = Kbar * Kbar
    I = np.nonzero(m)[0]
    if I.size == 0:
        return 0.0
    P = np.linalg.pinv(A64[I], rcond=REL_CUT)
    sbar = np.arange(n, n + nSbar)
    Mg = A64[sbar] @ P                       # (144, N_I)
    gi = m[sbar]
    pos = {int(k): q for q, k in enumerate(I)}
    for a in np.nonzero(gi)[0]:
        Mg[a, :] = 0.0
        Mg[a, pos[int(sbar[a])]] = 1.0
    C = cheb.coef_matrix(Kbar)
    Vx = cheb.vander(xi, Kbar - 1)
    Vy = cheb.vander(eta, Kbar - 1)
    aa, bb = np.meshgrid(np.arange(Kbar), np.arange(Kbar), indexing="ij")
    keep = (aa + bb < Kbar).astype(np.float64)
    # value_p = sum_ab Vx[p,a] keep[a,b] (C G C^T)[a,b] Vy[p,b]
    # with G = reshape(Mg @ f); build the operator column by column
    Op = np.empty((xi.size, I.size))
    for c in range(I.size):
        Gc = Mg[:, c].reshape(Kbar, Kbar)
        cf = (C @ Gc @ C.T) * keep
        Op[:, c] = np.einsum("pa,ab,pb->p", Vx, cf, Vy)
    return float(np.abs(Op).sum(axis=1).max())
