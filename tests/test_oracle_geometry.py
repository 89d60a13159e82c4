"""Pins for the oracle's tree checks and extension lists (CPU).

Hand-made trees whose answers are fixed by the definitions of Section 4:
balance (level restriction), exact tiling, the extension list with the
closest-centre rule and the "later cut square wins" tie rule, and the
extension restriction (no coarse neighbour in an extension list).
"""
import numpy as np

from oracle.geometry import Tree, extension_owner, cut_masks
from workloads import Disk


def uniform(depth):
    n = 2 ** depth
    lv, ix, iy = [], [], []
    for a in range(n):
        for b in range(n):
            lv.append(depth), ix.append(a), iy.append(b)
    return lv, ix, iy


def refine(lv, ix, iy, k):
    l, x, y = lv.pop(k), ix.pop(k), iy.pop(k)
    for dx in (0, 1):
        for dy in (0, 1):
            lv.append(l + 1), ix.append(2 * x + dx), iy.append(2 * y + dy)


def test_partition_and_balance():
    lv, ix, iy = uniform(2)
    t = Tree(lv, ix, iy)
    assert t.check_partition() and t.is_balanced()
    # refine the corner leaf (0,0) twice -> level 4 next to level 2: unbalanced
    k = [i for i in range(len(lv)) if (ix[i], iy[i]) == (0, 0)][0]
    refine(lv, ix, iy, k)
    t = Tree(lv, ix, iy)
    assert t.check_partition() and t.is_balanced()
    k = [i for i in range(len(lv)) if (lv[i], ix[i], iy[i]) == (3, 1, 1)][0]
    refine(lv, ix, iy, k)
    t = Tree(lv, ix, iy)
    assert t.check_partition() and not t.is_balanced()
    # a missing leaf breaks the tiling
    t = Tree(lv[:-1], ix[:-1], iy[:-1])
    assert not t.check_partition()


def test_extension_list_closest_centre_and_tie_rule():
    # 4x4 uniform tree; cut leaves at (1,1) and (1,3), exterior leaf (1,2)
    # is equidistant from both centres -> the later cut leaf owns it.
    lv, ix, iy = uniform(2)
    t = Tree(lv, ix, iy)
    kinds = np.ones(t.n, dtype=int)  # regular
    idx = {(ix[i], iy[i]): i for i in range(t.n)}
    c1, c2 = idx[(1, 1)], idx[(1, 3)]
    e = idx[(1, 2)]
    e2 = idx[(0, 0)]      # only in Sbar of (1,1)
    e3 = idx[(3, 3)]      # in no Sbar
    for i in (c1, c2):
        kinds[i] = 2
    for i in (e, e2, e3):
        kinds[i] = 0
    own, viol = extension_owner(t, kinds)
    assert not viol
    assert own[c1] == c1 and own[c2] == c2
    later = max(c1, c2)
    assert own[e] == later
    assert own[e2] == c1
    assert own[e3] == -1
    # regular leaves never belong to a list
    assert all(own[i] == -1 for i in range(t.n) if kinds[i] == 1)
    # strictly closer centre wins regardless of order: (0,2) is closer to (1,3)?
    # centres (1.5,1.5)/(1.5,3.5) vs (0.5,2.5): equal -> later again
    k02 = idx[(0, 2)]
    kinds[k02] = 0
    own, _ = extension_owner(t, kinds)
    assert own[k02] == later
    # (2,0): in Sbar of (1,1) only
    k20 = idx[(2, 0)]
    kinds[k20] = 0
    own, _ = extension_owner(t, kinds)
    assert own[k20] == c1


def test_extension_restriction_violation_detected():
    # level-2 tree with one leaf refined; a fine cut leaf whose Sbar overlaps
    # a coarse exterior neighbour that it is closest to -> violation
    lv, ix, iy = uniform(2)
    k = [i for i in range(len(lv)) if (ix[i], iy[i]) == (1, 1)][0]
    refine(lv, ix, iy, k)
    t = Tree(lv, ix, iy)
    assert t.is_balanced()
    kinds = np.ones(t.n, dtype=int)
    cut = [i for i in range(t.n) if (lv[i], ix[i], iy[i]) == (3, 2, 2)][0]
    coarse = [i for i in range(t.n) if (lv[i], ix[i], iy[i]) == (2, 0, 0)][0]
    kinds[cut] = 2
    kinds[coarse] = 0
    own, viol = extension_owner(t, kinds)
    assert own[coarse] == cut
    assert (coarse, cut) in viol


def test_masks_follow_inside_test():
    lv, ix, iy = uniform(3)
    t = Tree(lv, ix, iy)
    d = Disk(0.6)
    cx, cy = t.centers()
    kinds = d.classify_boxes(cx, cy, t.h())
    cuts = [i for i in range(t.n) if kinds[i] == 2]
    m = cut_masks(t, cuts, d, 8)
    assert m.shape == (len(cuts), 274)
    counts = m.sum(axis=1)
    assert len(cuts) == 20 and counts.min() > 0 and counts.max() < 274
    # a cut leaf's own K x K nodes: interior exactly where |x| < 0.6
    X, Y = t.leaf_nodes(8)
    for r, i in enumerate(cuts):
        assert np.array_equal(m[r, :64], X[i] ** 2 + Y[i] ** 2 < 0.36)
