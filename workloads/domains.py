"""Planar domains: inside tests and the cut/regular/exterior box rule.

A leaf box is *regular* when it lies inside the domain, *cut* when the
boundary crosses it and *exterior* otherwise (Section 4, definition of regular
leaf nodes and cut squares).  The paper leaves the intersection test to the
user; here it is part of the input definition:

* the disk uses the exact distance test;
* the other domains sample the closed box on a uniform (m+1) x (m+1) grid
  (corners and edges included) and call the box cut when the samples contain
  both inside and outside points.
"""
import math

import numpy as np

EXTERIOR, REGULAR, CUT = 0, 1, 2


class Domain:
    name = "domain"
    sample_m = 64

    def inside(self, x, y):  # pragma: no cover - interface
        raise NotImplementedError

    def classify_boxes(self, cx, cy, h):
        """Return EXTERIOR/REGULAR/CUT per box (arrays of centres, sides)."""
        cx = np.atleast_1d(np.asarray(cx, dtype=np.float64))
        cy = np.atleast_1d(np.asarray(cy, dtype=np.float64))
        h = np.broadcast_to(np.asarray(h, dtype=np.float64), cx.shape)
        s = np.linspace(-0.5, 0.5, self.sample_m + 1)
        sx, sy = np.meshgrid(s, s, indexing="ij")
        out = np.empty(cx.shape, dtype=np.int8)
        chunk = 256
        for b in range(0, cx.size, chunk):
            e = min(cx.size, b + chunk)
            X = cx[b:e, None, None] + h[b:e, None, None] * sx[None]
            Y = cy[b:e, None, None] + h[b:e, None, None] * sy[None]
            ins = self.inside(X, Y).reshape(e - b, -1)
            a = ins.all(axis=1)
            n = ~ins.any(axis=1)
            k = np.full(e - b, CUT, dtype=np.int8)
            k[a] = REGULAR
            k[n] = EXTERIOR
            out[b:e] = k
        return out


class Disk(Domain):
    """Open disk of radius r about (x0, y0)."""

    def __init__(self, r=0.6, x0=0.0, y0=0.0):
        self.r, self.x0, self.y0 = float(r), float(x0), float(y0)
        self.name = f"disk(r={self.r})"

    def inside(self, x, y):
        x = np.asarray(x, dtype=np.float64) - self.x0
        y = np.asarray(y, dtype=np.float64) - self.y0
        return x * x + y * y < self.r * self.r

    def classify_boxes(self, cx, cy, h):
        cx = np.atleast_1d(np.asarray(cx, dtype=np.float64)) - self.x0
        cy = np.atleast_1d(np.asarray(cy, dtype=np.float64)) - self.y0
        h = np.broadcast_to(np.asarray(h, dtype=np.float64), cx.shape)
        half = 0.5 * h
        # nearest and farthest points of the closed box from the centre
        nx = np.maximum(np.abs(cx) - half, 0.0)
        ny = np.maximum(np.abs(cy) - half, 0.0)
        fx = np.abs(cx) + half
        fy = np.abs(cy) + half
        dmin2 = nx * nx + ny * ny
        dmax2 = fx * fx + fy * fy
        r2 = self.r * self.r
        out = np.full(cx.shape, CUT, dtype=np.int8)
        out[dmax2 < r2] = REGULAR
        out[dmin2 >= r2] = EXTERIOR
        return out


class Starfish(Domain):
    """Star-shaped domain r(theta) = r0 + a cos(m theta) about the origin."""

    def __init__(self, r0=0.5, a=0.15, m=5):
        self.r0, self.a, self.m = float(r0), float(a), int(m)
        self.name = f"starfish(r0={self.r0},a={self.a},m={self.m})"

    def radius(self, theta):
        return self.r0 + self.a * np.cos(self.m * theta)

    def inside(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        th = np.arctan2(y, x)
        return np.hypot(x, y) < self.radius(th)


class SquareMinusWedge(Domain):
    """Square [-s, s]^2 with the wedge |arg z| < alpha removed (apex at 0).

    The removed wedge opens along +x; the domain has corners at the square's
    four vertices, at the apex and where the wedge meets the square.
    """

    def __init__(self, s=0.6, alpha=math.pi / 6):
        self.s, self.alpha = float(s), float(alpha)
        self.name = f"square-wedge(s={self.s},alpha={self.alpha:.6f})"

    def inside(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        sq = (np.abs(x) < self.s) & (np.abs(y) < self.s)
        wedge = (x > 0) & (np.abs(y) <= np.tan(self.alpha) * x)
        origin = (x == 0) & (y == 0)
        return sq & ~wedge & ~origin
