"""Quad-tree geometry for the oracle: leaf nodes, checks, masks, lists.

A tree is given by its leaves: level l, integer position (ix, iy) with
0 <= ix, iy < 2^l, inside a root square of side ``size`` centred at
``(cx, cy)`` (Section 4: the root box D and its recursive subdivision).

Everything combinatorial is done in exact integer arithmetic on the finest
dyadic grid, so that distance ties are decided exactly.
"""
import numpy as np

from . import cheb
from . import stencil


class Tree:
    def __init__(self, level, ix, iy, root=(0.0, 0.0, 2.0)):
        self.level = np.asarray(level, dtype=np.int64)
        self.ix = np.asarray(ix, dtype=np.int64)
        self.iy = np.asarray(iy, dtype=np.int64)
        self.cx0, self.cy0, self.size = (float(v) for v in root)
        self.n = self.level.size
        self.lmax = int(self.level.max()) if self.n else 0

    # geometry -----------------------------------------------------------
    def h(self):
        return self.size / (2.0 ** self.level)

    def centers(self):
        h = self.h()
        x = self.cx0 - 0.5 * self.size + (self.ix + 0.5) * h
        y = self.cy0 - 0.5 * self.size + (self.iy + 0.5) * h
        return x, y

    def int_box(self, i):
        """Leaf i as [x0, x1) x [y0, y1) on the grid of spacing size/2^(lmax+1)."""
        s = 1 << (self.lmax + 1 - int(self.level[i]))
        return (int(self.ix[i]) * s, (int(self.ix[i]) + 1) * s,
                int(self.iy[i]) * s, (int(self.iy[i]) + 1) * s)

    def int_center2(self, i):
        """The centre in units of size/2^(lmax+1) (an exact integer pair)."""
        x0, x1, y0, y1 = self.int_box(i)
        return (x0 + x1) // 2, (y0 + y1) // 2

    def leaf_nodes(self, K):
        """World coordinates of every leaf's K x K first-kind grid, shape
        (L, K*K); node (a, b) -> flat a*K + b with a the x index."""
        t = cheb.nodes(K)
        x, y = self.centers()
        h = self.h()
        X = x[:, None, None] + 0.5 * h[:, None, None] * t[None, :, None] + 0.0 * t[None, None, :]
        Y = y[:, None, None] + 0.0 * t[None, :, None] + 0.5 * h[:, None, None] * t[None, None, :]
        return X.reshape(self.n, K * K), Y.reshape(self.n, K * K)

    # checks -------------------------------------------------------------
    def check_partition(self):
        """Leaves are exactly the leaves of a quad-tree over the root: no leaf
        is an ancestor of another and every internal box has all 4 children."""
        leaves = set(zip(self.level.tolist(), self.ix.tolist(), self.iy.tolist()))
        if len(leaves) != self.n:
            return False
        internal = set()
        for (l, x, y) in leaves:
            while l > 0:
                l, x, y = l - 1, x >> 1, y >> 1
                internal.add((l, x, y))
        if leaves & internal:
            return False
        if self.n == 1:
            return (0, 0, 0) in leaves
        for (l, x, y) in internal:
            for dx in (0, 1):
                for dy in (0, 1):
                    c = (l + 1, 2 * x + dx, 2 * y + dy)
                    if c not in leaves and c not in internal:
                        return False
        return True

    def adjacency(self):
        """List of (i, j) pairs of distinct leaves whose closed boxes touch."""
        boxes = [self.int_box(i) for i in range(self.n)]
        pairs = []
        # sweep by x to keep it near-linear for moderate trees
        order = sorted(range(self.n), key=lambda i: boxes[i][0])
        active = []
        for i in order:
            x0, x1, y0, y1 = boxes[i]
            active = [j for j in active if boxes[j][1] >= x0]
            for j in active:
                a0, a1, b0, b1 = boxes[j]
                if a0 <= x1 and x0 <= a1 and b0 <= y1 and y0 <= b1:
                    pairs.append((j, i))
            active.append(i)
        return pairs

    def is_balanced(self):
        for i, j in self.adjacency():
            if abs(int(self.level[i]) - int(self.level[j])) > 1:
                return False
        return True


def cut_masks(tree, cut_ids, domain, K, Kbar=12, deg=10):
    """Interior flags of the stencil points of every cut leaf, shape
    (n_cut, |X|).  Sbar has side 3h and the cut leaf's centre (Section 3.2)."""
    P = stencil.stencil_points(K, Kbar, deg)
    x, y = tree.centers()
    h = tree.h()
    out = np.zeros((len(cut_ids), P.shape[0]), dtype=bool)
    for r, i in enumerate(cut_ids):
        X = x[i] + 1.5 * h[i] * P[:, 0]
        Y = y[i] + 1.5 * h[i] * P[:, 1]
        out[r] = domain.inside(X, Y)
    return out


def stencil_world(tree, i, K, Kbar=12, deg=10):
    P = stencil.stencil_points(K, Kbar, deg)
    x, y = tree.centers()
    h = tree.h()
    return x[i] + 1.5 * h[i] * P[:, 0], y[i] + 1.5 * h[i] * P[:, 1]


def extension_owner(tree, kinds, cut_kind=2, ext_kind=0):
    """Owner cut leaf of every leaf (Section 4, extension lists), or -1.

    A cut leaf owns itself.  An exterior leaf S' belongs to the extension
    list of the cut leaf S whose extension square Sbar overlaps S' with
    positive area and whose centre is closest to the centre of S'; when two
    centres are equally close the one that comes later in the canonical
    order (ascending leaf index) takes precedence.  Distances are compared
    exactly in integers.

    Returns (owner, violations) where violations lists (S', S) pairs in
    which the owner S is finer than S' (the extension restriction forbids a
    coarse neighbour in an extension list).
    """
    kinds = np.asarray(kinds)
    owner = np.full(tree.n, -1, dtype=np.int64)
    cuts = [i for i in range(tree.n) if kinds[i] == cut_kind]
    for i in cuts:
        owner[i] = i
    ext = [j for j in range(tree.n) if kinds[j] == ext_kind]
    best = {}
    ext_boxes = {j: tree.int_box(j) for j in ext}
    ext_c = {j: tree.int_center2(j) for j in ext}
    for i in cuts:  # canonical order
        x0, x1, y0, y1 = tree.int_box(i)
        w = x1 - x0
        bx0, bx1, by0, by1 = x0 - w, x1 + w, y0 - w, y1 + w  # Sbar
        ci = tree.int_center2(i)
        for j in ext:
            a0, a1, b0, b1 = ext_boxes[j]
            if min(a1, bx1) - max(a0, bx0) > 0 and min(b1, by1) - max(b0, by0) > 0:
                cj = ext_c[j]
                d2 = (ci[0] - cj[0]) ** 2 + (ci[1] - cj[1]) ** 2
                if j not in best or d2 <= best[j][0]:
                    best[j] = (d2, i)
    violations = []
    for j, (_, i) in best.items():
        owner[j] = i
        if tree.level[i] > tree.level[j]:
            violations.append((j, i))
    return owner, violations
