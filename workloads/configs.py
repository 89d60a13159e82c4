"""Named, seeded workload configurations.

Each configuration fixes the root box, the leaf grid size K, the FMM order p,
the domain, the analytic data f = Laplacian(u) and how the quad-tree is
refined.  Tree *construction* is not done here (it belongs to the host side of
the solver); this module only states the recipe.

* ``disk_uniform3``: root [-1,1]^2, uniform depth 3 (64 leaves), K = 8,
  disk of radius 0.6, u = exp(-((x-0.1)^2 + (y+0.2)^2)/0.05), p = 20.
* ``starfish_adaptive``: starfish r = 0.5 + 0.15 cos(5 theta), u a sum of four
  Gaussians with widths drawn from U[0.01, 0.1] and centres drawn uniformly in
  the domain (seed 1), K = 16, adaptive refinement on Chebyshev tails
  (tolerance 1e-13) with cut leaves at level 8, depth at most 9: 4207 leaves,
  about 1.08e6 leaf nodes; FMM order 24 (the smallest order whose measured
  rel Linf against the oracle is below 1e-11: 8.1e-13).
* ``wedge_adaptive``: [-0.6,0.6]^2 minus the wedge |arg z| < pi/6, same kind
  of data (widths from U[0.005, 0.1], seed 3), K = 16, cut leaves at level 9,
  every non-exterior leaf at level >= 7: 14254 leaves, 3.65e6 leaf nodes;
  FMM order 24.
* ``starfish_batch``: 256 seeded right-hand sides (Gaussian sums of 1-8
  bumps, widths U[0.01, 0.1], seed 4) on one starfish tree of depth 8 (cut
  leaves at level 8), refined on the sum of all of them; K = 16, p = 24.
* small variants used by the tests (``disk_tiny``, ``starfish_small``,
  ``disk_adaptive_small``).
"""
import math

import numpy as np

from .domains import Disk, Starfish, SquareMinusWedge
from .functions import GaussianSum


def _seeded_gaussians(domain, n, wlo, whi, seed, box=0.7):
    rng = np.random.default_rng(seed)
    widths = rng.uniform(wlo, whi, n)
    centers = []
    while len(centers) < n:
        p = rng.uniform(-box, box, 2)
        if domain.inside(p[0], p[1]):
            centers.append(p)
    return GaussianSum(np.array(centers), widths)


def batch_functions(domain, nrhs, seed):
    """Seeded right-hand sides for the batched workload: Gaussian sums of 1-8
    bumps each (widths U[0.01, 0.1], centres uniform in the domain)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nrhs):
        nb = int(rng.integers(1, 9))
        widths = rng.uniform(0.01, 0.1, nb)
        centers = []
        while len(centers) < nb:
            q = rng.uniform(-0.7, 0.7, 2)
            if domain.inside(q[0], q[1]):
                centers.append(q)
        out.append(GaussianSum(np.array(centers), widths, rng.uniform(0.5, 1.5, nb)))
    return out


class _Union:
    """The sum of several right-hand sides (the tree of a batch is refined on
    it, so it resolves every member)."""

    def __init__(self, funs):
        self.funs = funs

    def f(self, x, y):
        return sum(g.f(x, y) for g in self.funs)


def _cfg(name):
    if name == "disk_uniform3":
        dom = Disk(0.6)
        return dict(name=name, root=(0.0, 0.0, 2.0), K=8, p=20, domain=dom,
                    fun=GaussianSum([[0.1, -0.2]], [0.05]),
                    tree=dict(kind="uniform", depth=3), seed=None)
    if name == "disk_tiny":
        dom = Disk(0.6)
        return dict(name=name, root=(0.0, 0.0, 2.0), K=8, p=30, domain=dom,
                    fun=GaussianSum([[0.1, -0.2]], [0.05]),
                    tree=dict(kind="uniform", depth=2), seed=None)
    if name == "disk_adaptive_small":
        dom = Disk(0.55, 0.03, -0.02)
        return dict(name=name, root=(0.0, 0.0, 2.0), K=8, p=40, domain=dom,
                    fun=GaussianSum([[0.15, -0.1], [-0.2, 0.2]], [0.01, 0.05], [1.0, -0.5]),
                    tree=dict(kind="adaptive", tol=1e-6, max_depth=6, min_cut_level=3),
                    seed=None)
    if name == "starfish_small":
        dom = Starfish(0.5, 0.15, 5)
        return dict(name=name, root=(0.0, 0.0, 2.0), K=16, p=40, domain=dom,
                    fun=_seeded_gaussians(dom, 4, 0.01, 0.1, seed=1),
                    tree=dict(kind="adaptive", tol=1e-6, max_depth=6, min_cut_level=4),
                    seed=1)
    if name == "starfish_adaptive":
        dom = Starfish(0.5, 0.15, 5)
        return dict(name=name, root=(0.0, 0.0, 2.0), K=16, p=24, domain=dom,
                    fun=_seeded_gaussians(dom, 4, 0.01, 0.1, seed=1),
                    tree=dict(kind="adaptive", tol=1e-13, max_depth=9, min_cut_level=8),
                    seed=1)
    if name == "wedge_adaptive":
        dom = SquareMinusWedge(0.6, math.pi / 6)
        return dict(name=name, root=(0.0, 0.0, 2.0), K=16, p=24, domain=dom,
                    fun=_seeded_gaussians(dom, 4, 0.005, 0.1, seed=3),
                    tree=dict(kind="adaptive", tol=1e-12, max_depth=10, min_cut_level=9, min_level=7),
                    seed=3)
    if name == "starfish_batch":
        dom = Starfish(0.5, 0.15, 5)
        funs = batch_functions(dom, 256, seed=4)
        return dict(name=name, root=(0.0, 0.0, 2.0), K=16, p=24, domain=dom, fun=_Union(funs), rhs=funs,
                    tree=dict(kind="adaptive", tol=1e-12, max_depth=8, min_cut_level=8), seed=4)
    raise KeyError(name)


CONFIG_NAMES = ("disk_uniform3", "disk_tiny", "disk_adaptive_small", "starfish_small",
                "starfish_adaptive", "wedge_adaptive", "starfish_batch")


def get_config(name):
    return _cfg(name)
