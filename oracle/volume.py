"""Volume potential by direct quadrature (oracle only).

V(x) = (1/2 pi) sum_B int_B log|x - y| p_B(y) dy over every leaf B with
nonzero data, where p_B is the degree-(K-1) tensor Chebyshev interpolant of
the leaf's K x K samples (Section 1, eqs. volpot and greenf; Section 4.1:
the VFMM computes exactly this for the piecewise-polynomial f^e up to its
far-field tolerance).  The double sum runs in plain C (volume.c), compiled on
first use with gcc; the Gauss-Legendre rules it applies come from
gauss_legendre() below.
"""
import ctypes
import functools
import os
import subprocess
import threading

import mpmath as mp

import numpy as np

from . import cheb

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "volume.c")
_LIB = os.path.join(_HERE, "_volume.so")
_lock = threading.Lock()
_lib = None


def build(force=False):
    """Compile volume.c into _volume.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            d = ctypes.POINTER(ctypes.c_double)
            lib.oracle_volume.argtypes = [ctypes.c_int, d, d, ctypes.c_int, d, d, d, ctypes.c_int, d,
                                          d, d, ctypes.c_int, d, d, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, d]
            lib.oracle_volume.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@functools.lru_cache(maxsize=None)
def _gauss_legendre(q):
    # Golub-Welsch: the nodes are the eigenvalues of the symmetric Jacobi
    # matrix of the Legendre recurrence (off-diagonal k / sqrt(4k^2 - 1)).
    # Each eigenvalue seeds a root search on mpmath's Legendre function in
    # 34-digit arithmetic; the weight is 2 / ((1 - x^2) P_q'(x)^2) with
    # P_q'(x) = q P_{q-1}(x) / (1 - x^2) at a root of P_q.  Rounded to
    # double once, and made exactly symmetric.
    k = np.arange(1, q)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    seeds = np.linalg.eigvalsh(np.diag(beta, 1) + np.diag(beta, -1))
    x = np.zeros(q)
    w = np.zeros(q)
    with mp.workdps(34):
        for i in range(q // 2, q):
            if q % 2 and i == q // 2:
                r = mp.mpf(0)
            else:
                r = mp.findroot(lambda t: mp.legendre(q, t), mp.mpf(float(seeds[i])))
            dp = q * mp.legendre(q - 1, r) / (1 - r * r)
            x[i], w[i] = float(r), float(2 / ((1 - r * r) * dp * dp))
            x[q - 1 - i], w[q - 1 - i] = -x[i], w[i]
    x.setflags(write=False)
    w.setflags(write=False)
    return x, w


def gauss_legendre(q):
    """q-point Gauss-Legendre rule on [-1, 1] (nodes ascending, weights)."""
    if not 1 <= q <= 48:
        raise ValueError("bad order")
    return _gauss_legendre(int(q))


def leaf_coefficients(values, K):
    """Chebyshev coefficients c[a, b] of each leaf's tensor interpolant;
    values has shape (L, K*K) with node (a, b) at flat a*K + b."""
    C = cheb.coef_matrix(K)
    V = np.asarray(values, dtype=np.float64).reshape(-1, K, K)
    return np.einsum("ai,lij,bj->lab", C, V, C)


def potential_boxes(tx, ty, cx, cy, h, coef, K, qf=None, qn=12, M=28, far_ratio=1.0):
    """V at targets from boxes given by centres, sides and coefficients."""
    tx = np.ascontiguousarray(tx, dtype=np.float64).reshape(-1)
    ty = np.ascontiguousarray(ty, dtype=np.float64).reshape(-1)
    cx = np.ascontiguousarray(cx, dtype=np.float64).reshape(-1)
    cy = np.ascontiguousarray(cy, dtype=np.float64).reshape(-1)
    h = np.ascontiguousarray(np.broadcast_to(h, cx.shape), dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64).reshape(cx.size, K * K)
    if qf is None:
        qf = K + 16
    out = np.zeros(tx.size)
    gxf, gwf = (np.ascontiguousarray(a) for a in gauss_legendre(int(qf)))
    gxn, gwn = (np.ascontiguousarray(a) for a in gauss_legendre(int(qn)))
    rc = _load().oracle_volume(tx.size, _ptr(tx), _ptr(ty), cx.size, _ptr(cx), _ptr(cy), _ptr(h), K,
                               _ptr(coef), _ptr(gxf), _ptr(gwf), int(qf), _ptr(gxn), _ptr(gwn), int(qn),
                               int(M), float(far_ratio), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_volume: bad parameters")
    return out


def potential(tree, fe, K, tx, ty, sources=None, **kw):
    """V at targets (tx, ty) from the leaves of ``tree`` carrying data fe
    (shape (L, K*K)); leaves whose data is identically zero are skipped;
    ``sources`` optionally restricts the source leaves."""
    fe = np.asarray(fe, dtype=np.float64)
    cx, cy = tree.centers()
    h = tree.h()
    idx = np.arange(tree.n) if sources is None else np.asarray(sources)
    idx = idx[np.any(fe[idx] != 0.0, axis=1)]
    coef = leaf_coefficients(fe[idx], K)
    return potential_boxes(tx, ty, cx[idx], cy[idx], h[idx], coef, K, **kw)


def net_charge(tree, fe, K):
    """Net charge A^e = int f^e over the leaves of ``tree`` (Section 6, the
    exterior problem: the volume potential of f^e grows like A^e log|x|).
    Each leaf integrates its tensor Chebyshev interpolant exactly: the
    K-point first-kind (Fejer) rule in each variable, mapped from [-1,1]^2 to
    the leaf of side h (Jacobian (h/2)^2).  fe has shape (L, K*K), or
    (nrhs, L, K*K); the leaf contributions are summed exactly rounded."""
    import math
    w = cheb.fejer1_weights(K)
    W = np.outer(w, w).ravel()
    h = tree.h()
    fe = np.asarray(fe, dtype=np.float64).reshape(-1, tree.n, K * K)
    out = []
    for r in range(fe.shape[0]):
        per_leaf = (0.5 * h) ** 2 * (fe[r] @ W)
        out.append(math.fsum(per_leaf.tolist()))
    return np.array(out)
