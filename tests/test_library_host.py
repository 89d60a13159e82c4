"""Host-side checks of the HIP library (CPU only, no kernel launches).

* the shared library loads and exports every function declared in
  include/vfx.h;
* its stencil and interpolation matrix equal the oracle's;
* its near-field tables reproduce the oracle's direct quadrature for all 33
  list-1 configurations;
* its interaction lists partition the source leaves for every target leaf
  (every source reached exactly once, through the near field or exactly one
  far-field path);
* its extension lists equal the oracle's;
* its list-3 (M2P) operands reproduce a point source exactly, and list-3
  boxes sit where those operands assume;
* invalid input is rejected with the documented status codes.
"""
import os
import re

import numpy as np
import pytest

from oracle import cheb, geometry, stencil, volume
from paper_2211_14537_amd import tree as T
from paper_2211_14537_amd import vfx
from workloads import get_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "vfx.h")).read()
    names = set(re.findall(r"^\s*(?:int|const char\*)\s+(vfx_\w+)\s*\(", hdr, flags=re.M))
    assert len(names) >= 15
    L = vfx.lib()
    for nm in sorted(names):
        assert hasattr(L, nm), nm
    assert set(vfx.EXPORTED) == names


@pytest.mark.parametrize("K", [8, 16])
def test_stencil_and_matrix_match_oracle(K):
    ctx = vfx.Context(K, 20)
    P = ctx.stencil_points()
    Po = stencil.stencil_points(K)
    assert P.shape == Po.shape
    assert np.abs(P - Po).max() < 1e-15
    A = ctx.debug_table(1, 0, P.shape[0] * 66).reshape(-1, 66)
    Ao = stencil.interp_matrix(K)
    assert np.abs(A - Ao).max() < 1e-12
    assert np.allclose(ctx.leaf_nodes(), cheb.nodes(K), atol=1e-16, rtol=0)


def _near_geometry(c):
    if c < 9:
        return c // 3 - 1, c % 3 - 1, 1.0
    cells = [(a, b) for a in range(4) for b in range(4) if not (a in (1, 2) and b in (1, 2))]
    a, b = cells[(c - 9) if c < 21 else (c - 21)]
    if c < 21:
        return (2 * a - 3) / 2, (2 * b - 3) / 2, 2.0
    return (2 * a - 3) / 4, (2 * b - 3) / 4, 0.5


@pytest.mark.parametrize("K", [8])
def test_near_tables_match_oracle_quadrature(K):
    n = K * K
    ctx = vfx.Context(K, 20)
    t = cheb.nodes(K)
    tx = (0.5 * t[:, None] + 0 * t[None, :]).ravel()
    ty = (0 * t[:, None] + 0.5 * t[None, :]).ravel()
    rng = np.random.default_rng(0)
    for c in range(33):
        Tc = ctx.debug_table(0, c, n * n).reshape(n, n)
        ox, oy, s = _near_geometry(c)
        f = rng.standard_normal(n)
        vo = volume.potential_boxes(tx, ty, [ox], [oy], [s], volume.leaf_coefficients(f[None], K), K)
        err = np.abs(f @ Tc - 2 * np.pi * vo).max()
        assert err < 2e-14, (c, err)


def _plan_for(name, all_regular=False):
    cfg = get_config(name)
    ctx = vfx.Context(cfg["K"], cfg["p"], root=cfg["root"])
    tr = T.build_tree(cfg, ctx.stencil_points())
    kind = np.ones_like(tr["kind"]) if all_regular else tr["kind"]
    return cfg, ctx, tr, vfx.Plan(ctx, tr["level"], tr["ix"], tr["iy"], kind, None if all_regular else tr["mask"])


@pytest.mark.parametrize("all_regular", [True, False])
@pytest.mark.parametrize("name", ["disk_uniform3", "disk_adaptive_small", "starfish_small"])
def test_lists_partition_sources(name, all_regular):
    """Every source leaf whose extended data can be nonzero is reached from
    every target exactly once (near field, or one far-field path); a leaf
    whose f^e vanishes identically (exterior, outside every extension list)
    is never a list-1/list-4 source nor alone under a list-2/list-3 box."""
    cfg, ctx, tr, plan = _plan_for(name, all_regular=all_regular)
    bx = plan.boxes()
    B = bx["level"].size
    L = tr["level"].size
    key = {(int(bx["level"][b]), int(bx["ix"][b]), int(bx["iy"][b])): b for b in range(B)}
    parent = np.full(B, -1)
    for b in range(B):
        lv = bx["level"][b]
        if lv > 0:
            parent[b] = key[(int(lv) - 1, int(bx["ix"][b]) >> 1, int(bx["iy"][b]) >> 1)]
    kids = {}
    for b in range(B):
        if parent[b] >= 0:
            kids.setdefault(parent[b], []).append(b)

    def leaves_under(b):
        if bx["leaf"][b] >= 0:
            return [int(bx["leaf"][b])]
        out = []
        for c in kids[b]:
            out += leaves_under(c)
        return out

    kind = np.asarray(tr["kind"]) if not all_regular else np.ones(L, dtype=np.int8)
    zero = (kind == 0) & (plan.ext_owner() < 0)
    p1, s1, _ = plan.lists(1)
    p2, s2, _ = plan.lists(2)
    p3, s3, _ = plan.lists(3)
    p4, s4, _ = plan.lists(4)
    leaf_box = {int(bx["leaf"][b]): b for b in range(B) if bx["leaf"][b] >= 0}
    for leaf in range(L):
        got = list(s1[p1[leaf]:p1[leaf + 1]])
        for w in s3[p3[leaf]:p3[leaf + 1]]:
            got += leaves_under(w)
        b = leaf_box[leaf]
        while b >= 0:
            for s in s2[p2[b]:p2[b + 1]]:
                got += leaves_under(s)
            got += list(s4[p4[b]:p4[b + 1]])
            b = parent[b]
        if all_regular:
            assert sorted(got) == list(range(L)), leaf
        else:
            got = np.array(got, dtype=int)
            live = np.flatnonzero(~zero)
            assert np.array_equal(np.sort(got[~zero[got]]), live), leaf
            assert np.unique(got).size == got.size, leaf
    if not all_regular:
        assert not zero[s1].any() and not zero[s4].any()
        for w in list(s2) + list(s3):
            assert not zero[leaves_under(w)].all()


@pytest.mark.parametrize("name", ["disk_uniform3", "disk_adaptive_small", "starfish_small"])
def test_extension_owner_matches_oracle(name):
    cfg, ctx, tr, plan = _plan_for(name)
    ot = geometry.Tree(tr["level"], tr["ix"], tr["iy"], cfg["root"])
    assert ot.check_partition() and ot.is_balanced()
    own, viol = geometry.extension_owner(ot, tr["kind"])
    assert not viol
    assert np.array_equal(plan.ext_owner(), own)
    m = geometry.cut_masks(ot, list(tr["cut_ids"]), cfg["domain"], cfg["K"])
    assert np.array_equal(m, tr["mask"].astype(bool))
    st = plan.stats()
    assert st["n_cut"] == tr["cut_ids"].size
    assert st["pinv_doubles"] == 66 * int(tr["mask"].sum())


def test_status_strings():
    L = vfx.lib()
    for code, name in ((vfx.VFX_OK, b"VFX_OK"), (vfx.VFX_EINVAL, b"VFX_EINVAL"), (vfx.VFX_ETREE, b"VFX_ETREE"),
                       (vfx.VFX_EHIP, b"VFX_EHIP"), (vfx.VFX_ENOMEM, b"VFX_ENOMEM")):
        assert L.vfx_status_string(code).split(b" ")[0] == name
    assert L.vfx_status_string(-99) == b"unknown status"
    with pytest.raises(vfx.VfxError) as e:
        vfx.Plan(vfx.Context(8, 20), [1, 1, 1], [0, 1, 0], [0, 0, 1], [1, 1, 1])
    assert str(e.value).startswith("[-2] VFX_ETREE")


def test_rejects_invalid_input():
    with pytest.raises(vfx.VfxError) as e:
        vfx.Context(1, 20)
    assert e.value.code == vfx.VFX_EINVAL
    with pytest.raises(vfx.VfxError) as e:
        vfx.Context(8, 100)
    assert e.value.code == vfx.VFX_EINVAL
    ctx = vfx.Context(8, 20)
    # leaves that do not tile the root
    with pytest.raises(vfx.VfxError) as e:
        vfx.Plan(ctx, [1, 1, 1], [0, 1, 0], [0, 0, 1], [1, 1, 1])
    assert e.value.code == vfx.VFX_ETREE
    # duplicate leaf
    with pytest.raises(vfx.VfxError) as e:
        vfx.Plan(ctx, [1, 1, 1, 1, 1], [0, 1, 0, 1, 1], [0, 0, 1, 1, 1], [1] * 5)
    assert e.value.code == vfx.VFX_ETREE
    # not level-restricted: level 3 leaves next to a level 1 leaf
    lv, ix, iy = [1, 1, 1], [1, 0, 1], [0, 1, 1]
    for a in range(2):
        for b in range(2):
            if (a, b) == (1, 1):
                for c in range(2):
                    for d in range(2):
                        lv.append(3), ix.append(2 * a + c), iy.append(2 * b + d)
            else:
                lv.append(2), ix.append(a), iy.append(b)
    with pytest.raises(vfx.VfxError) as e:
        vfx.Plan(ctx, lv, ix, iy, [1] * len(lv))
    assert e.value.code == vfx.VFX_ETREE
    # extension restriction: fine cut leaf closest to a coarse exterior leaf
    lv, ix, iy = [], [], []
    for a in range(4):
        for b in range(4):
            if (a, b) == (1, 1):
                for c in range(2):
                    for d in range(2):
                        lv.append(3), ix.append(2 * a + c), iy.append(2 * b + d)
            else:
                lv.append(2), ix.append(a), iy.append(b)
    kind = [1] * len(lv)
    cut = [i for i in range(len(lv)) if (lv[i], ix[i], iy[i]) == (3, 2, 2)][0]
    ext = [i for i in range(len(lv)) if (lv[i], ix[i], iy[i]) == (2, 0, 0)][0]
    kind[cut], kind[ext] = 2, 0
    with pytest.raises(vfx.VfxError) as e:
        vfx.Plan(ctx, lv, ix, iy, kind, np.ones((1, ctx.n_stencil), dtype=np.uint8))
    assert e.value.code == vfx.VFX_ETREE
    assert "extension restriction" in str(e.value)
    # kinds out of range
    with pytest.raises(vfx.VfxError) as e:
        vfx.Plan(ctx, [0], [0], [0], [5])
    assert e.value.code == vfx.VFX_EINVAL
    # misaligned buffers are refused before anything is read (the pointers
    # below are never dereferenced: the check is on their values)
    plan = vfx.Plan(ctx, [0], [0], [0], [1])
    for f_leaf, fe_out, V_out in ((8, 16, 16), (16, 8, 16), (16, 16, 8)):
        rc = vfx.lib().vfx_execute(plan._h, f_leaf, 0, fe_out, V_out, None)
        assert rc == vfx.VFX_EINVAL
        assert "16-byte aligned" in vfx.lib().vfx_last_error().decode()
    # precision modes are 0, 1, 2; the mixed modes need K = 16
    for mode in (-1, 3):
        with pytest.raises(vfx.VfxError):
            plan.set_precision(mode, 0)
    for mode in (1, 2):
        with pytest.raises(vfx.VfxError):
            plan.set_precision(mode, 0)


def test_near_lowrank_factors_match_oracle_quadrature():
    """K = 16 near-field operators in truncated low-rank form: the factors
    reproduce the dense table to the truncation tolerance and, applied to
    random leaf data, the oracle's direct quadrature of the near potential."""
    K, n = 16, 256
    ctx = vfx.Context(K, 24)
    rk = ctx.debug_table(22, 0, 66)
    R, rank = rk[:33].astype(int), rk[33:].astype(int)
    assert R[4] == 0  # the self interaction is full rank and stays dense
    assert (R[np.arange(33) != 4] > 0).all()
    assert ((R % 16) == 0).all() and (R <= 64).all() and (rank <= R).all()
    t = cheb.nodes(K)
    tx = (0.5 * t[:, None] + 0 * t[None, :]).ravel()
    ty = (0 * t[:, None] + 0.5 * t[None, :]).ravel()
    rng = np.random.default_rng(1)
    for c in (0, 1, 9, 10, 21, 22):
        A = ctx.debug_table(0, c, n * n).reshape(n, n)
        W = ctx.debug_table(20, c, n * 64).reshape(n, 64)
        Q = ctx.debug_table(21, c, n * 64).reshape(64, n)
        assert np.abs(W[:, rank[c]:]).max() == 0 and np.abs(Q[rank[c]:]).max() == 0
        assert np.abs(W @ Q - A).max() <= 1e-13 * np.abs(A).max(), c
        ox, oy, s = _near_geometry(c)
        f = rng.standard_normal(n)
        vo = volume.potential_boxes(tx, ty, [ox], [oy], [s], volume.leaf_coefficients(f[None], K), K)
        err = np.abs((f @ W) @ Q - 2 * np.pi * vo).max()
        assert err < 1e-13 * max(1.0, np.abs(2 * np.pi * vo).max()), (c, err)


def test_m2p_tables_reproduce_a_point_source():
    """List-3 M2P operands: applied to the scaled multipole of a unit point
    charge inside the source box (a_0 = 1, a_k = -s^k/k with s the charge's
    offset from the box centre in units of the box side), each of the 20
    slots gives log|z - s| at the target leaf's nodes (z in units of the box
    side) up to the truncation |s/z|^P; the other 16 slots and the padding
    rows are zero."""
    K, p = 16, 24
    n, P = K * K, p + 1
    rows = 64 * ((2 * P + 63) // 64)
    ctx = vfx.Context(K, p)
    t = cheb.nodes(K)
    s = 0.3 - 0.2j
    m = np.zeros(rows)
    m[0] = 1.0
    for k in range(1, P):
        a = -s ** k / k
        m[2 * k], m[2 * k + 1] = a.real, a.imag
    used = 0
    for slot in range(36):
        ox, oy = 2 * (slot // 6) - 5, 2 * (slot % 6) - 5
        T = ctx.debug_table(23, slot, rows * n).reshape(rows, n)
        if max(abs(ox), abs(oy)) != 5:
            assert np.abs(T).max() == 0, slot
            continue
        used += 1
        assert np.abs(T[2 * P:]).max() == 0 and np.abs(T[1]).max() == 0
        z = (t[:, None] - ox / 2) + 1j * (t[None, :] - oy / 2)
        ref = np.log(np.abs(z - s)).ravel()
        assert np.abs(m @ T - ref).max() < 1e-13, slot
    assert used == 20


def test_list3_boxes_are_one_level_finer():
    """Every list-3 box of a level-restricted tree is a child of a colleague
    of the leaf, one level finer and not touching it (the M2P slots assume
    it)."""
    cfg, ctx, tr, plan = _plan_for("starfish_small")
    bx = plan.boxes()
    lv, ix, iy = bx["level"], bx["ix"], bx["iy"]
    ptr, src, _ = plan.lists(3)
    lb, lx, ly = (np.asarray(tr[k]) for k in ("level", "ix", "iy"))
    assert len(src) > 0
    for leaf in range(len(ptr) - 1):
        for w in src[ptr[leaf]:ptr[leaf + 1]]:
            assert lv[w] == lb[leaf] + 1
            ox = (2 * ix[w] + 1) - 2 * (2 * lx[leaf] + 1)
            oy = (2 * iy[w] + 1) - 2 * (2 * ly[leaf] + 1)
            assert max(abs(ox), abs(oy)) == 5


def test_near_symmetry_classes():
    """The target-stationary near field applies one table per symmetry
    class: with g the D4 element the library assigns to configuration c,
    T_c[g(i)][g(j)] must equal the class base's T_b[i][j] (a log-kernel
    integral is invariant under an isometry of target and source), and g
    must carry the base's source offset onto c's.  Checked here with node
    maps and offsets computed independently of the library."""
    ctx = vfx.Context(16, 24)
    info = ctx.debug_table(24, 0, 82)
    cls, g, base, R = info[:33].astype(int), info[33:66].astype(int), info[66:73].astype(int), info[73:80].astype(int)
    assert info[80] == 1.0 and info[81] <= 1e-13
    assert cls[4] == 0 and np.count_nonzero(cls == 0) == 1
    assert all(R[k] in (16, 32, 48, 64) for k in range(1, 7))
    K = 16

    def node_map(code):
        a, b = np.divmod(np.arange(K * K), K)
        A, B = (b, a) if code & 1 else (a, b)
        A = K - 1 - A if code & 2 else A
        B = K - 1 - B if code & 4 else B
        return A * K + B

    def offset(c):  # source centre minus target centre, units of the target side
        if c < 9:
            return np.array([c // 3 - 1, c % 3 - 1], float)
        cells = [(i // 4, i % 4) for i in range(16) if not (i // 4 in (1, 2) and i % 4 in (1, 2))]
        aa, bb = cells[(c - 9) % 12]
        return np.array([2 * aa - 3, 2 * bb - 3], float) / (2.0 if c < 21 else 4.0)

    def apply(code, v):
        x, y = (v[1], v[0]) if code & 1 else (v[0], v[1])
        return np.array([-x if code & 2 else x, -y if code & 4 else y])

    worst = 0.0
    for c in range(33):
        b = base[cls[c]]
        assert np.array_equal(apply(g[c], offset(b)), offset(c)), c
        Tc = ctx.debug_table(0, c, K ** 4).reshape(K * K, K * K)  # [j][i]
        Tb = ctx.debug_table(0, b, K ** 4).reshape(K * K, K * K)
        m = node_map(g[c])
        worst = max(worst, np.abs(Tc[np.ix_(m, m)] - Tb).max() / np.abs(Tb).max())
    assert worst <= 1e-13


@pytest.mark.parametrize("i8", [True, False], ids=["int8", "bf16"])
def test_fixed_point_slices_reconstruct_the_near_tables(i8):
    """The fixed-point slices the mixed-precision kernels multiply: every
    operand row v is 2^e sum_s q_s w_s up to the stated residual, with e
    the exponent of max|v| (max|v| < 2^e) and the slices integers in their
    range (int8: five slices, w_s = 2^(-6-7s), |q_s| <= 64, residual
    2^(e-35); bf16: four slices, w_s = 2^(-8(s+1)), |q_0| <= 256, |q_s| <=
    128, residual 2^(e-33)).  Rebuilt here from that definition and compared
    with the FP64 tables the library applies (W, Q of the low-rank
    operators, and the self table)."""
    ctx = vfx.Context(16, 24)
    n, LM = 256, 64
    ns = 5 if i8 else 4
    w = np.array([2.0 ** (-6 - 7 * s) for s in range(5)] if i8 else [2.0 ** (-8 * (s + 1)) for s in range(4)])
    qmax = np.array([64.0] * 5 if i8 else [256.0, 128.0, 128.0, 128.0])
    resid = 35 if i8 else 33

    def check(rows, slices, exps):
        # rows: m x len, slices: ns x m x len, exps: m
        assert np.array_equal(slices, np.rint(slices))
        assert np.all(np.abs(slices) <= qmax[:, None, None])
        m = np.abs(rows).max(axis=1)
        nz = m > 0
        assert np.all(m[nz] < np.ldexp(1.0, exps[nz].astype(int)))
        assert np.all(m[nz] >= np.ldexp(0.5, exps[nz].astype(int)))
        assert np.all(slices[:, ~nz, :] == 0)
        rebuilt = np.ldexp(np.tensordot(w, slices, axes=(0, 0)), exps.astype(int)[:, None])
        bound = np.ldexp(1.0, exps.astype(int) - resid)[:, None]
        assert np.all(np.abs(rebuilt - rows) <= bound)

    which = 25 if i8 else 27
    rk = ctx.debug_table(22, 0, 66)
    for c in (0, 5, 12, 30):
        if rk[c] == 0:
            continue
        t = ctx.debug_table(which, c, 2 * ns * LM * n + LM + n)
        o = 0
        Ws = t[o:o + ns * LM * n].reshape(ns, LM, n); o += ns * LM * n
        We = t[o:o + LM]; o += LM
        Qs = t[o:o + ns * n * LM].reshape(ns, n, LM); o += ns * n * LM
        Qe = t[o:o + n]
        W = ctx.debug_table(20, c, n * LM).reshape(n, LM).T  # rows a, along j
        Q = ctx.debug_table(21, c, n * LM).reshape(LM, n).T  # rows i, along a
        check(W, Ws, We)
        check(Q, Qs, Qe)
    t = ctx.debug_table(which + 1, 0, ns * n * n + n)
    A = ctx.debug_table(0, 4, n * n).reshape(n, n).T  # self table, row i (target), column j
    check(A, t[:ns * n * n].reshape(ns, n, n), t[ns * n * n:])
