"""Learned refinement: the classifier's HIP kernels against the float64
oracle (forward, gradient, Adam, FP16 inference), training on the GPU, and
the gain of the learned tree builder with the plain criterion as fallback
and judge."""
import numpy as np
import pytest

from gpu_cases import say
from oracle import mlp

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda:0")


def _problem(B, seed):
    rng = np.random.default_rng(seed)
    theta = (mlp.init(seed) + 0.05 * rng.standard_normal(mlp.N_PARAMS)).astype(np.float32)
    X = rng.uniform(-1, 1, (B, 64)).astype(np.float32)
    y = (rng.random(B) < 0.4).astype(np.float32)
    return theta, X, y


@pytest.mark.parametrize("B", [1, 45, 300])
def test_forward_and_gradient_match_oracle(gpu_device, B):
    import torch
    from paper_2211_14537_amd import vfx
    assert vfx.mlp_param_count() == mlp.N_PARAMS
    theta, X, y = _problem(B, 3 + B)
    th, xd, yd = _t(theta), _t(X), _t(y)
    logits = torch.empty(B, dtype=torch.float32, device="cuda:0")
    vfx.mlp_forward(th, xd, logits)
    g = torch.empty_like(th)
    work = torch.empty(vfx.mlp_grad_work(B), dtype=torch.float32, device="cuda:0")
    vfx.mlp_grad(th, xd, yd, g, work)
    torch.cuda.synchronize()
    s_o, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64))
    g_o = mlp.backward(theta.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    es = np.abs(logits.cpu().numpy() - s_o).max() / max(1.0, np.abs(s_o).max())
    eg = np.abs(g.cpu().numpy() - g_o).max() / np.abs(g_o).max()
    say(f"    B={B}: logits rel err {es:.2e}, gradient rel err {eg:.2e}")
    assert es < 2e-5 and eg < 2e-4
    # deterministic: a second gradient is bitwise the same
    g2 = torch.empty_like(th)
    vfx.mlp_grad(th, xd, yd, g2, work)
    torch.cuda.synchronize()
    assert torch.equal(g, g2)


def test_adam_step_matches_oracle(gpu_device):
    import torch
    from paper_2211_14537_amd import vfx
    rng = np.random.default_rng(9)
    n = mlp.N_PARAMS
    theta, grad = rng.standard_normal(n), rng.standard_normal(n) * 1e-2
    m, v = rng.standard_normal(n) * 1e-3, rng.random(n) * 1e-4
    th, gd, md, vd = (_t(a) for a in (theta, grad, m, v))
    vfx.mlp_adam(th, gd, md, vd, 7, lr=1e-3)
    torch.cuda.synchronize()
    th_o, m_o, v_o = mlp.adam_step(theta.astype(np.float32).astype(np.float64), grad.astype(np.float32),
                                   m.astype(np.float32), v.astype(np.float32), 7, lr=1e-3)
    assert np.abs(th.cpu().numpy() - th_o).max() < 1e-6
    assert np.abs(md.cpu().numpy() - m_o).max() < 1e-8


def test_f16_inference_tracks_fp32(gpu_device):
    import torch
    from paper_2211_14537_amd import vfx
    theta, X, _ = _problem(2000, 11)
    th, xd = _t(theta), _t(X)
    l32 = torch.empty(2000, dtype=torch.float32, device="cuda:0")
    vfx.mlp_forward(th, xd, l32)
    thh = torch.empty(th.numel(), dtype=torch.float16, device="cuda:0")
    xh = torch.empty(xd.shape, dtype=torch.float16, device="cuda:0")
    vfx.f32_to_f16(th, thh)
    vfx.f32_to_f16(xd, xh)
    l16 = torch.empty_like(l32)
    vfx.mlp_infer_f16(thh, xh, l16)
    torch.cuda.synchronize()
    a, b = l32.cpu().numpy(), l16.cpu().numpy()
    d = np.abs(a - b).max() / max(1.0, np.abs(a).max())
    agree = np.mean((a > 0) == (b > 0))
    say(f"    FP16 vs FP32 logits: rel {d:.2e}, decisions agree {agree:.4f}")
    assert d < 3e-2 and agree > 0.99


def test_training_and_learned_tree_gain(gpu_device):
    """Train on boxes of plain-criterion trees (GPU, FP32), then build trees
    for unseen functions with FP16 inference: every leaf still passes the
    plain criterion, the builder evaluates fewer boxes, and the leaf count
    stays within 2% of the plain tree's."""
    from paper_2211_14537_amd import refine
    X, y = refine.training_data(12000, 1)
    Xt, yt = refine.training_data(3000, 2)
    theta, hist = refine.train(X, y, epochs=12, batch=1024, lr=3e-3, seed=0)
    clf = refine.Classifier(theta, threshold=1.0)
    acc = float(np.mean((clf.logits(Xt) > 0) == (yt > 0.5)))
    say(f"    training loss {hist[0]:.4f} -> {hist[-1]:.4f}; held-out accuracy {acc:.3f}")
    assert hist[-1] < hist[0] and acc > 0.9
    rng = np.random.default_rng(100)
    ev0 = ev1 = lv0 = lv1 = 0
    for _ in range(6):
        f = refine.random_function(rng)
        L0, s0 = refine.build(f, 1e-12, 10)
        L1, s1 = refine.build(f, 1e-12, 10, decide=clf)
        assert refine.check_leaves(f, L1, 1e-12, 10)
        ev0, ev1 = ev0 + s0["evaluated"], ev1 + s1["evaluated"]
        lv0, lv1 = lv0 + s0["leaves"], lv1 + s1["leaves"]
    say(f"    evaluated boxes: plain {ev0}, learned {ev1}; leaves: plain {lv0}, learned {lv1}")
    assert ev1 < 0.97 * ev0
    assert lv1 <= 1.02 * lv0
