"""The allocation-free net charge (vfx_net_charge_noalloc) against the
allocating entry point (vfx_net_charge): the same kernels over the same
fixed leaf partition, so the results must agree bit for bit.  Two calls in a
row, the second on a smaller plan (fewer leaves, fewer partial-sum blocks)
and fewer right-hand sides, so a stale partial of the first call would show;
then the same call captured in a HIP graph and replayed on changed data; and
the refusals (too many right-hand sides, a plan not yet on the device)."""
import numpy as np
import pytest

from gpu_cases import say, setup

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _both(plan, fe):
    import torch
    nrhs = fe.shape[0] if fe.dim() == 3 else 1
    ref = torch.full((nrhs,), float("nan"), dtype=torch.float64, device="cuda:0")
    out = torch.full((nrhs,), float("nan"), dtype=torch.float64, device="cuda:0")
    plan.net_charge(fe, ref)
    plan.net_charge_noalloc(fe, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_net_charge_matches_allocating_entry_point(gpu_device):
    import torch
    from paper_2211_14537_amd import vfx
    assert vfx.net_charge_noalloc_max_rhs() == 64
    rng = np.random.default_rng(17)
    # first call: 385-leaf tree, three right-hand sides
    a = setup("starfish_small", all_regular=True)
    fa = a["f_leaf"]
    stack = _dev(np.stack([fa, -2.0 * fa + 1.0, rng.standard_normal(fa.shape)]))
    ref, out = _both(a["plan"], stack)
    say(f"    starfish_small, 3 rhs: {out} (allocating {ref})")
    assert np.all(np.isfinite(out)) and np.array_equal(out, ref)
    # second call: a smaller tree (64 leaves, 2 partial-sum blocks), one right-hand side
    b = setup("disk_uniform3", all_regular=True)
    fb = _dev(b["f_leaf"] * 3.0 - 0.5)
    ref_b, out_b = _both(b["plan"], fb)
    say(f"    disk_uniform3, 1 rhs: {out_b} (allocating {ref_b})")
    assert np.all(np.isfinite(out_b)) and np.array_equal(out_b, ref_b)
    # the first plan again, one right-hand side: unaffected by the second call
    ref1, out1 = _both(a["plan"], stack[1])
    assert np.array_equal(out1, ref1) and out1[0] == ref[1]
    # captured in a graph and replayed on changed data
    s = torch.cuda.Stream()
    res = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda:0")
    g = vfx.Graph()
    with torch.cuda.stream(s):
        g.begin(s)
        a["plan"].net_charge_noalloc(stack, res, stream=s)
        g.end(s)
    for rep in range(3):
        stack.mul_(1.5).add_(0.25)
        res.fill_(float("nan"))
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        want = torch.empty(3, dtype=torch.float64, device="cuda:0")
        a["plan"].net_charge(stack, want)
        torch.cuda.synchronize()
        assert np.array_equal(res.cpu().numpy(), want.cpu().numpy()), rep
    g.close()
    say("    graph of the allocation-free call: 3 replays equal to the allocating entry point")


def test_noalloc_net_charge_refusals(gpu_device):
    import torch
    from paper_2211_14537_amd import vfx
    a = setup("disk_uniform3", all_regular=True)
    fe = _dev(a["f_leaf"])
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(vfx.VfxError):
        a["plan"].net_charge_noalloc(fe, out)  # the plan has no device data yet
    a["plan"].net_charge(fe, out)  # uploads
    torch.cuda.synchronize()
    big = fe.unsqueeze(0).expand(65, -1, -1).contiguous()
    out65 = torch.zeros(65, dtype=torch.float64, device="cuda:0")
    with pytest.raises(vfx.VfxError):
        a["plan"].net_charge_noalloc(big, out65)
    torch.cuda.synchronize()
