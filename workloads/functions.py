"""Analytic right-hand sides: f = Laplacian(u) for u a sum of Gaussians.

u(x) = sum_k a_k exp(-|x - c_k|^2 / w_k) and
f(x) = sum_k a_k (4 |x - c_k|^2 / w_k^2 - 4 / w_k) exp(-|x - c_k|^2 / w_k).

The paper's experiments use exactly this kind of smooth analytic data (its
interior example contains a narrow Gaussian bump; Section 6.1).
"""
import numpy as np


class GaussianSum:
    def __init__(self, centers, widths, amps=None):
        self.c = np.asarray(centers, dtype=np.float64).reshape(-1, 2)
        self.w = np.asarray(widths, dtype=np.float64).reshape(-1)
        if amps is None:
            amps = np.ones(self.w.shape)
        self.a = np.asarray(amps, dtype=np.float64).reshape(-1)
        assert self.c.shape[0] == self.w.size == self.a.size

    def u(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for (cx, cy), w, a in zip(self.c, self.w, self.a):
            r2 = (x - cx) ** 2 + (y - cy) ** 2
            out += a * np.exp(-r2 / w)
        return out

    def f(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for (cx, cy), w, a in zip(self.c, self.w, self.a):
            r2 = (x - cx) ** 2 + (y - cy) ** 2
            out += a * (4.0 * r2 / (w * w) - 4.0 / w) * np.exp(-r2 / w)
        return out

    def describe(self):
        return {"centers": self.c.tolist(), "widths": self.w.tolist(), "amps": self.a.tolist()}
