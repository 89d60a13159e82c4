"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only describes *inputs*: planar domains (an inside test and a
box classification rule), analytic right-hand sides f = Laplacian(u) built from
Gaussian bumps, and the named workload configurations with their seeds.  It
holds none of the method's arithmetic (no extension, no quadrature, no
expansions), so both sides of every parity test can draw from it.

The workloads are shaped like the paper's experiments (Section 6): analytic
smooth solutions on planar domains embedded in a square root box, with the
source data sampled on K x K first-kind Chebyshev leaf grids.
"""
from .domains import Disk, Starfish, SquareMinusWedge, Domain  # noqa: F401
from .functions import GaussianSum  # noqa: F401
from .configs import get_config, CONFIG_NAMES  # noqa: F401
