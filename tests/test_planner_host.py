"""Host-side checks of the C ABI library (no GPU): exported symbols, the
quadtree and interaction lists against the definitional oracle, target
association against brute force, expansion orders against the paper's
criterion, and argument validation."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import tree as otree
from paper_1602_05301_amd import inputs, qbx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "qbxfmm.h")).read()
    return sorted(set(re.findall(r"\b(qbx_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = qbx.lib()
    declared = _header_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(qbx.EXPORTS) == declared
    assert L.qbx_abi_version() == 3


def _geometries():
    yield "star7", inputs.star(64, 16, lobes=7)
    yield "ellipse", inputs.ellipse(40, 16, a=1.0, b=0.3, rotation=0.3)
    yield "multi", inputs.concat([inputs.star(24, 16, lobes=3, radius=0.5, center=(-0.9, 0.1)),
                                  inputs.ellipse(30, 16, a=0.6, b=0.2, center=(0.8, -0.4))])
    yield "star5_small", inputs.star(8, 4, lobes=5)


def _far_field_partition_holds(t, lists_of):
    """Sec. 7.2: for a target in leaf b, every source is reached exactly once:
    directly through U(b), by a multipole through W(b), or through the local
    expansion of b, which gathers V(a) (multipoles) and X(a) (sources) over a
    = b and its ancestors.  lists_of(name, box) gives a list as box indices."""
    nb = t["level"].size
    ns = sum(len(t["src"][b]) for b in range(nb) if t["leaf"][b])
    for b in np.flatnonzero(t["leaf"]):
        hit = np.zeros(ns, np.int64)
        for u in lists_of("U", b):
            hit[t["src"][u]] += 1
        for w in lists_of("W", b):
            hit[t["src"][w]] += 1
        a = b
        while a >= 0:
            for v in lists_of("V", a):
                hit[t["src"][v]] += 1
            for x in lists_of("X", a):
                hit[t["src"][x]] += 1
            a = t["parent"][a]
        if not np.all(hit == 1):
            return False
    return True


@pytest.mark.parametrize("level_restrict", [False, True])
@pytest.mark.parametrize("leaf_max", [8, 32, 64])
@pytest.mark.parametrize("name,geom", list(_geometries()))
def test_tree_and_lists_match_definitions(name, geom, leaf_max, level_restrict):
    pl = qbx.Plan(geom, 20.0, 1e-8, geom.sx, geom.sy, np.arange(geom.n),
                  qbx.options(p=8, leaf_max=leaf_max, level_restrict=level_restrict))
    bx = pl.boxes()
    t = otree.build(geom.sx, geom.sy, geom.cx, geom.cy, leaf_max, level_restrict=level_restrict)
    for k in ("level", "ix", "iy", "parent"):
        assert np.array_equal(bx[k], t[k]), k
    assert np.array_equal(bx["leaf"].astype(bool), t["leaf"])
    assert np.array_equal(bx["nsrc"], t["nsrc"]) and np.array_equal(bx["nctr"], t["nctr"])
    L = otree.lists(t)
    csr = {}
    for lname, which in (("U", qbx.LIST_U), ("V", qbx.LIST_V), ("W", qbx.LIST_W), ("X", qbx.LIST_X)):
        s, idx = pl.list(which)
        csr[lname] = (s, idx)
        for b in range(len(s) - 1):
            assert np.array_equal(idx[s[b]:s[b + 1]], L[lname][b]), (lname, b)
    # the planner's lists partition the sources seen from every leaf
    assert _far_field_partition_holds(t, lambda n, b: csr[n][1][csr[n][0][b]:csr[n][0][b + 1]])
    st = pl.stats()
    assert st["n_boxes"] == t["level"].size


@pytest.mark.parametrize("leaf_max", [4, 16])
def test_level_restricted_tree_is_balanced(leaf_max):
    """2:1 balance: touching leaves differ by at most one level, and the
    restricted tree refines the adaptive one (every adaptive box is kept)."""
    g = inputs.concat([inputs.star(16, 16, lobes=5, radius=0.5, center=(-0.6, 0.0)),
                       inputs.ellipse(24, 16, a=0.5, b=0.05, center=(0.55, 0.2), rotation=0.4)])
    free = qbx.Plan(g, 20.0, 1e-8, g.sx, g.sy, np.arange(g.n),
                    qbx.options(p=8, leaf_max=leaf_max, level_restrict=False)).boxes()
    bal = qbx.Plan(g, 20.0, 1e-8, g.sx, g.sy, np.arange(g.n),
                   qbx.options(p=8, leaf_max=leaf_max, level_restrict=True)).boxes()

    def unbalanced_pairs(bx):
        lv, ix, iy = (bx[k].astype(np.int64) for k in ("level", "ix", "iy"))
        lf = np.flatnonzero(bx["leaf"] != 0)
        L = int(lv.max())
        s = np.left_shift(1, L - lv[lf])
        x0, x1, y0, y1 = ix[lf] * s, (ix[lf] + 1) * s, iy[lf] * s, (iy[lf] + 1) * s
        touch = ((x0[:, None] <= x1[None, :]) & (x0[None, :] <= x1[:, None]) &
                 (y0[:, None] <= y1[None, :]) & (y0[None, :] <= y1[:, None]))
        gap = np.abs(lv[lf][:, None] - lv[lf][None, :])
        return int(np.count_nonzero(touch & (gap >= 2)))

    assert unbalanced_pairs(free) > 0, "the test geometry must need balancing"
    assert unbalanced_pairs(bal) == 0
    keys = lambda bx: set(zip(bx["level"].tolist(), bx["ix"].tolist(), bx["iy"].tolist()))
    assert keys(free) < keys(bal)


def test_partition_check_catches_a_wrong_w_list():
    """The partition invariant fails for a plausible mistake in the lists: W
    boxes one level too coarse (their parents instead of themselves)."""
    g = inputs.concat([inputs.star(24, 16, lobes=3, radius=0.5, center=(-0.9, 0.1)),
                       inputs.ellipse(30, 16, a=0.6, b=0.2, center=(0.8, -0.4))])
    t = otree.build(g.sx, g.sy, g.cx, g.cy, 8)
    L = otree.lists(t)
    assert _far_field_partition_holds(t, lambda n, b: L[n][b])
    assert any(len(w) for w in L["W"])
    bad = {k: list(v) for k, v in L.items()}
    bad["W"] = [np.unique(t["parent"][w]) if len(w) else w for w in L["W"]]
    assert not _far_field_partition_holds(t, lambda n, b: bad[n][b])


def test_single_box_tree():
    g = inputs.star(2, 4, lobes=3)
    pl = qbx.Plan(g, 5.0, 1e-8, g.sx, g.sy, np.arange(g.n), qbx.options(p=4, leaf_max=64))
    st = pl.stats()
    assert st["n_boxes"] == 1 and st["n_levels"] == 1
    s, idx = pl.list(qbx.LIST_U)
    assert idx.tolist() == [0]


def test_association_matches_brute_force():
    g = inputs.star(32, 16, lobes=5)
    rng = np.random.default_rng(7)
    # targets scattered near the curve: nodes pushed along the normal by
    # random multiples of the panel length, both sides, plus far points
    j = rng.integers(0, g.n, 3000)
    s = rng.uniform(-0.2, 0.9, j.size) * g.h[j]
    tx = np.concatenate([g.sx[j] + s * g.nx[j], rng.uniform(-3, 3, 200)])
    ty = np.concatenate([g.sy[j] + s * g.ny[j], rng.uniform(-3, 3, 200)])
    ref = oracle.associate(tx, ty, g.cx, g.cy, g.cr, g.sx, g.sy, g.h, 0.05)
    keep = ref != -2
    # targets the brute force marks as failures make the planner fail as a whole
    with pytest.raises(qbx.QbxError) as ei:
        qbx.Plan(g, 10.0, 1e-8, tx, ty, None, qbx.options(p=8))
    assert ei.value.status == qbx.QBX_E_ASSOC and (~keep).any()
    pl = qbx.Plan(g, 10.0, 1e-8, tx[keep], ty[keep], None, qbx.options(p=8))
    assert np.array_equal(pl.association(), ref[keep])


def test_explicit_association_is_kept():
    g = inputs.star(16, 8, lobes=5)
    tc = np.arange(g.n, dtype=np.int32)
    pl = qbx.Plan(g, 10.0, 1e-8, g.sx, g.sy, tc, qbx.options(p=8))
    assert np.array_equal(pl.association(), tc)


def _criterion(omega, R, n):
    """|H_n(3 omega R) J_n(sqrt(2) omega R)| in mpmath (no overflow)."""
    import mpmath
    x, y = 3 * omega * R, np.sqrt(2) * omega * R
    return np.array([float(abs(mpmath.hankel1(int(k), x)) * abs(mpmath.besselj(int(k), y)))
                     for k in np.atleast_1d(n)])


@pytest.mark.parametrize("omega,eps", [(50.0, 1e-10), (10.0, 1e-6), (120.0, 1e-8)])
def test_orders_follow_the_criterion(omega, eps):
    g = inputs.star(256, 16, lobes=7)
    p = 14
    pl = qbx.Plan(g, omega, eps, g.sx, g.sy, np.arange(g.n), qbx.options(p=p))
    P = pl.orders()
    st = pl.stats()
    R0 = st["root_radius"]
    p_add = st["p_add"]
    for lev, Pl in enumerate(P):
        R = R0 / 2 ** lev
        pf = Pl - p_add
        n_hi = np.arange(pf + 1, pf + 60)
        assert np.all(_criterion(omega, R, n_hi) <= eps), lev
        if pf > 1:
            assert _criterion(omega, R, np.array([pf]))[0] > eps, lev


@pytest.mark.parametrize("bad", ["omega", "eps", "p", "normal", "radius", "nan", "tgt_ctr", "fp32_eps"])
def test_invalid_arguments_are_rejected(bad):
    g = inputs.star(8, 8, lobes=3)
    omega, eps, opts, tc = 10.0, 1e-8, qbx.options(p=8), np.arange(g.n)
    if bad == "omega":
        omega = -1.0
    elif bad == "eps":
        eps = 0.5
    elif bad == "p":
        opts = qbx.options(p=41)
    elif bad == "normal":
        g.nx[3] *= 1.1
    elif bad == "radius":
        g.cr[0] = 0.0
    elif bad == "nan":
        g.sx[5] = np.nan
    elif bad == "tgt_ctr":
        tc = tc.copy(); tc[0] = g.n + 5
    elif bad == "fp32_eps":
        eps, opts = 1e-8, qbx.options(p=8, far_fp32=True)   # FP32 far field needs eps >= 1e-6
    with pytest.raises(qbx.QbxError) as ei:
        qbx.Plan(g, omega, eps, g.sx, g.sy, tc, opts)
    assert ei.value.status == qbx.QBX_E_INVAL


def test_fp32_far_field_accepted_at_loose_tolerance():
    g = inputs.star(8, 8, lobes=3)
    pl = qbx.Plan(g, 10.0, 1e-6, g.sx, g.sy, np.arange(g.n), qbx.options(p=8, far_fp32=True))
    assert pl.stats()["n_levels"] >= 1


def test_context_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = qbx.lib().qbx_ctx_create(0, None, ctypes.byref(h))
    assert rc == qbx.QBX_E_DEVICE
