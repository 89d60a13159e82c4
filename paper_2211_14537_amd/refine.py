"""Learned refinement for the adaptive quad-tree (host logic; the network is
trained and evaluated by the library's HIP kernels).

The plain criterion (R10, as in tree.py): a box is split while the l2 norm
of its Chebyshev coefficients of total order >= K-1 exceeds tol * max|f|.
The classifier reads the last four coefficient rows of a box that R10
splits (features below) and predicts whether all four of its children will
be split as well; the learned builder then splits such a box two levels at
once, which skips evaluating f and its coefficients on the four children.  R10 is still
applied to every box the builder evaluates, so it remains the fallback (a
wrong "keep" costs nothing but the saving) and the judge: every final leaf
satisfies R10, whatever the network says.  A wrong "refine twice" can only
add leaves (finer than needed).

Training data: boxes split by R10 in plain trees of seeded Gaussian sums
(1-8 bumps, widths log-uniform in [0.005, 0.2]) on the square [-1, 1]^2,
labelled by R10 applied to their children.  Training: FP32, Adam, on the
GPU (vfx_mlp_grad / vfx_mlp_adam); inference: FP16 (vfx_mlp_infer_f16).
"""
import time

import numpy as np

from workloads.functions import GaussianSum

from .tree import _coef_matrix, cheb_nodes

K = 16
NFEAT = 64
ROOT = (0.0, 0.0, 2.0)


def random_function(rng):
    nb = int(rng.integers(1, 9))
    c = rng.uniform(-0.8, 0.8, (nb, 2))
    w = np.exp(rng.uniform(np.log(0.005), np.log(0.2), nb))
    a = rng.choice([-1.0, 1.0], nb) * rng.uniform(0.5, 1.5, nb)
    return GaussianSum(c, w, a)


def fscale(fun, root=ROOT):
    s = np.linspace(-0.5, 0.5, 801)
    X, Y = np.meshgrid(root[0] + root[2] * s, root[1] + root[2] * s, indexing="ij")
    return float(np.abs(fun.f(X, Y)).max())


_C = _coef_matrix(K)
_T = cheb_nodes(K)
_A, _B = np.meshgrid(np.arange(K), np.arange(K), indexing="ij")
_TAIL = (_A + _B) >= K - 1


def coefficients(fun, keys, root=ROOT):
    """16 x 16 first-kind Chebyshev coefficients of f on each box (l, x, y)."""
    keys = np.asarray(keys, dtype=np.int64).reshape(-1, 3)
    h = root[2] / (2.0 ** keys[:, 0])
    cx = root[0] - 0.5 * root[2] + (keys[:, 1] + 0.5) * h
    cy = root[1] - 0.5 * root[2] + (keys[:, 2] + 0.5) * h
    X = cx[:, None, None] + 0.5 * h[:, None, None] * _T[None, :, None] + 0 * _T[None, None, :]
    Y = cy[:, None, None] + 0 * _T[None, :, None] + 0.5 * h[:, None, None] * _T[None, None, :]
    F = fun.f(X, Y)
    return np.einsum("ai,lij,bj->lab", _C, F, _C)


def tail_norm(c):
    return np.sqrt((c[:, _TAIL] ** 2).sum(axis=1))


def features(c, fs):
    """The last four coefficient rows, log10(|c| / max|f|) clipped to
    [-30, 0] and mapped to [-1, 1]: 64 float32 values per box."""
    v = np.log10(np.abs(c[:, K - 4:, :]).reshape(-1, NFEAT) / fs + 1e-300)
    return ((np.clip(v, -30.0, 0.0) + 15.0) / 15.0).astype(np.float32)


def build(fun, tol, max_depth, decide=None, root=ROOT):
    """Adaptive tree by R10; `decide(features) -> bool array` (or None) says
    which split boxes are split two levels at once.  Returns the leaves
    (sorted keys) and counts: evaluated boxes, leaves, two-level jumps."""
    fs = fscale(fun, root)
    front = [(0, 0, 0)]
    leaves, evaluated, jumps = [], 0, 0
    while front:
        keys = np.array(front, dtype=np.int64)
        c = coefficients(fun, keys, root)
        evaluated += len(front)
        split = (tail_norm(c) > tol * fs) & (keys[:, 0] < max_depth)
        two = np.zeros(len(front), dtype=bool)
        if decide is not None and split.any():
            can = split & (keys[:, 0] + 2 <= max_depth)
            if can.any():
                two[can] = decide(features(c[can], fs))
        nxt = []
        for (l, x, y), s, t in zip(front, split, two):
            if not s:
                leaves.append((l, x, y))
                continue
            if t:
                jumps += 1
                nxt.extend((l + 2, 4 * x + i, 4 * y + j) for i in range(4) for j in range(4))
            else:
                nxt.extend((l + 1, 2 * x + i, 2 * y + j) for i in range(2) for j in range(2))
        front = nxt
    return sorted(leaves), {"evaluated": evaluated, "leaves": len(leaves), "jumps": jumps}


def check_leaves(fun, leaves, tol, max_depth, root=ROOT):
    """R10 as judge: True if every leaf passes the tail test (or sits at
    max_depth)."""
    keys = np.array(leaves, dtype=np.int64)
    c = coefficients(fun, keys, root)
    fs = fscale(fun, root)
    return bool(((tail_norm(c) <= tol * fs) | (keys[:, 0] >= max_depth)).all())


def training_data(n_samples, seed, tol=1e-12, max_depth=10):
    """(features, labels) of boxes split by R10 in plain trees of random
    Gaussian sums, labelled by whether R10 splits all four children."""
    rng = np.random.default_rng(seed)
    Xs, ys, n = [], [], 0
    while n < n_samples:
        fun = random_function(rng)
        fs = fscale(fun)
        front = [(0, 0, 0)]
        while front and n < n_samples:
            keys = np.array(front, dtype=np.int64)
            c = coefficients(fun, keys)
            split = (tail_norm(c) > tol * fs) & (keys[:, 0] < max_depth)
            idx = np.nonzero(split & (keys[:, 0] + 1 < max_depth))[0]
            if idx.size:
                kids = np.array([(l + 1, 2 * x + i, 2 * y + j) for (l, x, y) in keys[idx]
                                 for i in range(2) for j in range(2)], dtype=np.int64)
                ck = coefficients(fun, kids)
                ks = (tail_norm(ck) > tol * fs).reshape(-1, 4).all(axis=1)
                Xs.append(features(c[idx], fs))
                ys.append(ks.astype(np.float32))
                n += idx.size
            front = [(l + 1, 2 * x + i, 2 * y + j) for (l, x, y), s in zip(keys.tolist(), split) if s
                     for i in range(2) for j in range(2)]
    X = np.concatenate(Xs)[:n_samples]
    y = np.concatenate(ys)[:n_samples]
    return X, y


def init_params(seed):
    """He-style initial parameters (float32), the layout of vfx_mlp_*."""
    rng = np.random.default_rng(seed)
    D = NFEAT
    parts = [rng.normal(0, np.sqrt(2 / D), D * D), np.zeros(D), rng.normal(0, np.sqrt(2 / D), D * D), np.zeros(D),
             rng.normal(0, np.sqrt(1 / D), D), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def train(X, y, epochs=30, batch=1024, lr=3e-3, seed=0, device="cuda:0", log=None):
    """Adam on the GPU through the library's kernels; returns the float32
    parameters and the per-epoch mean loss."""
    import torch
    from . import vfx
    dev = torch.device(device)
    rng = np.random.default_rng(seed)
    theta = torch.tensor(init_params(seed), device=dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    g = torch.zeros_like(theta)
    Xd = torch.tensor(X, device=dev)
    yd = torch.tensor(y, device=dev)
    work = torch.empty(vfx.mlp_grad_work(batch), dtype=torch.float32, device=dev)
    logits = torch.empty(len(X), dtype=torch.float32, device=dev)
    hist, step = [], 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(len(X)), device=dev)
        for b0 in range(0, len(X) - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            xb = Xd[sel].contiguous()
            yb = yd[sel].contiguous()
            vfx.mlp_grad(theta, xb, yb, g, work)
            step += 1
            vfx.mlp_adam(theta, g, m, v, step, lr=lr)
        vfx.mlp_forward(theta, Xd, logits)
        s = logits.double()
        L = float(torch.mean(torch.clamp(s, min=0) - s * yd.double() + torch.log1p(torch.exp(-s.abs()))))
        hist.append(L)
        if log:
            log(f"epoch {ep}: loss {L:.4f}")
    torch.cuda.synchronize()
    return theta.cpu().numpy(), hist


class Classifier:
    """FP16 inference with the library kernel; decide(features) -> bool."""

    def __init__(self, theta, device="cuda:0", threshold=0.0):
        import torch
        from . import vfx
        self.dev = torch.device(device)
        t32 = torch.tensor(np.asarray(theta, dtype=np.float32), device=self.dev)
        self.th = torch.empty(t32.numel(), dtype=torch.float16, device=self.dev)
        vfx.f32_to_f16(t32, self.th)
        self.threshold = threshold
        self.vfx = vfx

    def logits(self, F):
        import torch
        x32 = torch.tensor(np.asarray(F, dtype=np.float32), device=self.dev)
        xh = torch.empty(x32.shape, dtype=torch.float16, device=self.dev)
        self.vfx.f32_to_f16(x32, xh)
        out = torch.empty(x32.shape[0], dtype=torch.float32, device=self.dev)
        self.vfx.mlp_infer_f16(self.th, xh, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def __call__(self, F):
        return self.logits(F) > self.threshold
