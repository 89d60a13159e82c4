"""Host-side quad-tree construction (the solver's input preparation).

Builds the adaptive, level-restricted quad-tree of Section 4 for a domain and
a right-hand side: refinement on the decay of each leaf's Chebyshev
coefficients, 2:1 balance, cut/regular/exterior labels, the extension
restriction (a cut leaf may not extend onto a coarser leaf; such leaves are
split, as in the paper's extension figure), and the interior flags of every
cut leaf's stencil points.  None of this is on the GPU path; its output is
the `vfx_tree` the library consumes.

Reading of the refinement rule (the paper's wording is garbled): a leaf that
meets the domain is split while the l2 norm of its Chebyshev coefficients of
total order >= K-1 exceeds tol * max|f| (max over the domain, so that
near-zero regions are not over-refined) and the level is below max_depth;
cut leaves are in addition split down to min_cut_level (in place of the
paper's rule tying the cut-leaf size to the boundary panel length).
"""
import numpy as np

from workloads.domains import CUT, EXTERIOR, REGULAR

DMAX = 28


def cheb_nodes(K):
    a = np.arange(K)
    return -np.cos((2 * a + 1) * np.pi / (2 * K))


def _coef_matrix(K):
    t = cheb_nodes(K)
    C = (2.0 / K) * np.cos(np.outer(np.arange(K), np.arccos(t)))
    C[0] *= 0.5
    return C


def _morton(x, y):
    r = 0
    for b in range(DMAX + 1):
        r |= ((x >> b) & 1) << (2 * b)
        r |= ((y >> b) & 1) << (2 * b + 1)
    return r


def leaf_order_key(l, x, y):
    """Canonical leaf order: Morton order of the lower-left corner."""
    return _morton(x << (DMAX - l), y << (DMAX - l))


class TreeBuilder:
    def __init__(self, root, K, domain, fun):
        self.cx0, self.cy0, self.size = (float(v) for v in root)
        self.K = K
        self.domain = domain
        self.fun = fun
        self.t = cheb_nodes(K)
        self.C = _coef_matrix(K)

    def geom(self, keys):
        keys = np.asarray(keys, dtype=np.int64).reshape(-1, 3)
        l, x, y = keys[:, 0], keys[:, 1], keys[:, 2]
        h = self.size / (2.0 ** l)
        cx = self.cx0 - 0.5 * self.size + (x + 0.5) * h
        cy = self.cy0 - 0.5 * self.size + (y + 0.5) * h
        return cx, cy, h

    def classify(self, keys):
        cx, cy, h = self.geom(keys)
        return self.domain.classify_boxes(cx, cy, h)

    def tails(self, keys):
        cx, cy, h = self.geom(keys)
        t = self.t
        X = cx[:, None, None] + 0.5 * h[:, None, None] * t[None, :, None] + 0 * t[None, None, :]
        Y = cy[:, None, None] + 0 * t[None, :, None] + 0.5 * h[:, None, None] * t[None, None, :]
        F = self.fun.f(X, Y)
        c = np.einsum("ai,lij,bj->lab", self.C, F, self.C)
        a, b = np.meshgrid(np.arange(self.K), np.arange(self.K), indexing="ij")
        tail = (a + b) >= self.K - 1
        return np.sqrt((c[:, tail] ** 2).sum(axis=1))

    def fscale(self):
        s = np.linspace(-0.5, 0.5, 801)
        X, Y = np.meshgrid(self.cx0 + self.size * s, self.cy0 + self.size * s, indexing="ij")
        ins = self.domain.inside(X, Y)
        return float(np.abs(self.fun.f(X[ins], Y[ins])).max())


def _children(k):
    l, x, y = k
    return [(l + 1, 2 * x + dx, 2 * y + dy) for dy in (0, 1) for dx in (0, 1)]


def _covering_leaf(leaves, l, x, y):
    """Leaf containing box (l, x, y) if it is at level <= l, else None."""
    while l >= 0:
        if (l, x, y) in leaves:
            return (l, x, y)
        l, x, y = l - 1, x >> 1, y >> 1
    return None


def balance(leaves):
    """Split leaves until adjacent leaves differ by at most one level."""
    leaves = set(leaves)
    by_level = {}
    for k in leaves:
        by_level.setdefault(k[0], set()).add(k)
    lmax = max(by_level)
    for m in range(lmax, 1, -1):
        work = list(by_level.get(m, ()))
        for (l, x, y) in work:
            if (l, x, y) not in leaves:
                continue
            n = 1 << l
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    if dx == 0 and dy == 0:
                        continue
                    px, py = x + dx, y + dy
                    if px < 0 or py < 0 or px >= n or py >= n:
                        continue
                    while True:
                        cov = _covering_leaf(leaves, l, px, py)
                        if cov is None or cov[0] >= l - 1:
                            break
                        leaves.remove(cov)
                        by_level[cov[0]].discard(cov)
                        for ch in _children(cov):
                            leaves.add(ch)
                            by_level.setdefault(ch[0], set()).add(ch)
    return leaves


def _owners(leaves_sorted, kinds):
    """Extension-list owners (closest cut centre; later cut leaf wins ties)."""
    lmax = max(k[0] for k in leaves_sorted)
    idx = {k: i for i, k in enumerate(leaves_sorted)}

    def cen(k):
        l, x, y = k
        return (2 * x + 1) << (lmax - l), (2 * y + 1) << (lmax - l)

    owner = {}
    best = {}
    leafset = set(leaves_sorted)
    for i, k in enumerate(leaves_sorted):
        if kinds[i] != CUT:
            continue
        l, x, y = k
        n = 1 << l
        sx, sy = cen(k)
        cand = set()
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                if dx == 0 and dy == 0:
                    continue
                px, py = x + dx, y + dy
                if px < 0 or py < 0 or px >= n or py >= n:
                    continue
                cov = _covering_leaf(leafset, l, px, py)
                if cov is not None:
                    cand.add(cov)
                else:  # finer leaves inside this colleague position
                    stack = [(l, px, py)]
                    while stack:
                        b = stack.pop()
                        if b in leafset:
                            cand.add(b)
                        else:
                            stack.extend(_children(b))
        for c in cand:
            j = idx[c]
            if kinds[j] != EXTERIOR:
                continue
            cx, cy = cen(c)
            d2 = (cx - sx) ** 2 + (cy - sy) ** 2
            if j not in best or d2 <= best[j]:
                best[j] = d2
                owner[j] = i
    return owner


def build_tree(cfg, stencil_points=None, max_rounds=50):
    """Build the tree described by a workload configuration.

    Returns a dict with int32 arrays level, ix, iy (canonical leaf order),
    int8 kind, the cut-leaf indices and, when ``stencil_points`` (the |X| x 2
    stencil in the Sbar frame) is given, the uint8 interior mask of every cut
    leaf's stencil.
    """
    B = TreeBuilder(cfg["root"], cfg["K"], cfg["domain"], cfg["fun"])
    spec = cfg["tree"]
    if spec["kind"] == "uniform":
        d = spec["depth"]
        leaves = {(d, x, y) for x in range(1 << d) for y in range(1 << d)}
    else:
        tol, maxd, mincut = spec["tol"], spec["max_depth"], spec.get("min_cut_level", 0)
        minlev = spec.get("min_level", 0)
        fs = B.fscale()
        leaves = set()
        front = [(0, 0, 0)]
        while front:
            kinds = B.classify(front)
            tails = B.tails(front)
            nxt = []
            for k, kd, tl in zip(front, kinds, tails):
                split = False
                if k[0] < maxd and kd != EXTERIOR:
                    if tl > tol * fs:
                        split = True
                    if kd == CUT and k[0] < mincut:
                        split = True
                    if k[0] < minlev:
                        split = True
                if split:
                    nxt.extend(_children(k))
                else:
                    leaves.add(k)
            front = nxt
    for _ in range(max_rounds):
        leaves = balance(leaves)
        srt = sorted(leaves, key=lambda k: leaf_order_key(*k))
        kinds = B.classify(srt)
        owner = _owners(srt, kinds)
        bad = [srt[j] for j, i in owner.items() if srt[i][0] > srt[j][0]]
        if not bad:
            break
        for k in bad:
            leaves.discard(k)
            leaves.update(_children(k))
    else:
        raise RuntimeError("extension restriction did not converge")
    keys = np.array(srt, dtype=np.int64)
    out = {"level": keys[:, 0].astype(np.int32), "ix": keys[:, 1].astype(np.int32),
           "iy": keys[:, 2].astype(np.int32), "kind": np.asarray(kinds, dtype=np.int8)}
    out["cut_ids"] = np.nonzero(out["kind"] == CUT)[0]
    cx, cy, h = B.geom(keys)
    out["cx"], out["cy"], out["h"] = cx, cy, h
    if stencil_points is not None:
        P = np.asarray(stencil_points)
        m = np.zeros((out["cut_ids"].size, P.shape[0]), dtype=np.uint8)
        for r, i in enumerate(out["cut_ids"]):
            X = cx[i] + 1.5 * h[i] * P[:, 0]
            Y = cy[i] + 1.5 * h[i] * P[:, 1]
            m[r] = cfg["domain"].inside(X, Y)
        out["mask"] = m
    return out


def sample_inputs(cfg, tree, stencil_points):
    """f on every leaf grid (rows of non-regular leaves are unused by the
    solver) and f at the interior stencil points of every cut leaf (zero at
    exterior points)."""
    K = cfg["K"]
    t = cheb_nodes(K)
    cx, cy, h = tree["cx"], tree["cy"], tree["h"]
    X = (cx[:, None, None] + 0.5 * h[:, None, None] * t[None, :, None] + 0 * t[None, None, :]).reshape(-1, K * K)
    Y = (cy[:, None, None] + 0 * t[None, :, None] + 0.5 * h[:, None, None] * t[None, None, :]).reshape(-1, K * K)
    f_leaf = cfg["fun"].f(X, Y)
    P = np.asarray(stencil_points)
    cut = tree["cut_ids"]
    f_cut = np.zeros((cut.size, P.shape[0]))
    for r, i in enumerate(cut):
        sx = cx[i] + 1.5 * h[i] * P[:, 0]
        sy = cy[i] + 1.5 * h[i] * P[:, 1]
        v = cfg["fun"].f(sx, sy)
        f_cut[r] = np.where(tree["mask"][r] != 0, v, 0.0)
    return f_leaf, f_cut
