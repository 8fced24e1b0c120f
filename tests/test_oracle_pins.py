"""Pins of the oracle against facts fixed by the paper and by mathematics.

None of these re-type the oracle's formulas: each compares an oracle result
with an independent quantity (scipy / mpmath special functions, direct kernel
sums, closed forms on the circle, Green's identity, brute force on tiny
inputs, hand-built association cases)."""
import mpmath
import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import translations as T
from paper_1602_05301_amd import inputs


# ---------------------------------------------------------------------------
# Bessel / Hankel sequences
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("x", [1e-2, 0.1, 0.7, 2.5, 5.0, 20.0, 100.0])
def test_hankel_seq_vs_scipy(x):
    N = 60
    h = oracle.hankel1_seq(x, N)
    ref = sp.hankel1(np.arange(N + 1), x)
    ok = np.isfinite(ref)
    rel = np.abs(h[ok] - ref[ok]) / np.abs(ref[ok])
    assert rel.max() < 1e-13


@pytest.mark.parametrize("x,n", [(0.3, 7), (3.0, 0), (3.0, 1), (12.5, 17), (40.0, 55)])
def test_hankel_vs_mpmath(x, n):
    ref = complex(mpmath.hankel1(n, x))
    h = oracle.hankel1_seq(x, n)[n]
    assert abs(h - ref) / abs(ref) < 1e-13


@pytest.mark.parametrize("x", [1e-3, 0.2, 1.0, 2.5, 7.0, 30.0, 150.0])
def test_besselj_seq_vs_scipy_and_sum_rule(x):
    N = 80
    j = oracle.besselj_seq(x, N)
    ref = sp.jv(np.arange(N + 1), x)
    assert np.max(np.abs(j - ref)) < 1e-14 * max(1.0, np.max(np.abs(ref))) * 10
    # J_0 + 2 sum_k J_{2k} = 1 (generating function at t = 1); needs N >> x
    if x < 40:
        assert abs(j[0] + 2 * np.sum(j[2::2]) - 1.0) < 1e-13


@pytest.mark.parametrize("x", [0.05, 1.0, 9.0])
def test_wronskian(x):
    # J_{n+1} Y_n - J_n Y_{n+1} = 2/(pi x)
    h = oracle.hankel1_seq(x, 20)
    j = oracle.besselj_seq(x, 20)
    y = h.imag
    w = j[1:] * y[:-1] - j[:-1] * y[1:]
    assert np.max(np.abs(w / (2 / (np.pi * x)) - 1.0)) < 1e-12


# ---------------------------------------------------------------------------
# Graf's addition theorem and the translation operators, each checked by a
# round trip against direct kernel sums.
# ---------------------------------------------------------------------------

def _direct_S(omega, t, s, q):
    return np.sum(q * sp.hankel1(0, omega * np.abs(t - s)))


def _direct_D(omega, t, s, q, nu):
    d = t - s
    r = np.abs(d)
    cosang = (d.real * nu.real + d.imag * nu.imag) / r
    return np.sum(q * omega * sp.hankel1(1, omega * r) * cosang)


def _cluster(rng, centre, radius, n):
    s = centre + radius * (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)) / np.sqrt(2)
    q = inputs.complex_gaussian(rng, n)
    qd = inputs.complex_gaussian(rng, n)
    ang = rng.uniform(0, 2 * np.pi, n)
    return s, q, qd, np.exp(1j * ang)


@pytest.mark.parametrize("omega", [1.0, 10.0, 100.0])
def test_graf_p2l_l2p(omega):
    # H0(omega|x - s|) = sum_{|l|<=P} O_l(s - c) L_l(x - c) for |x-c| <= |s-c|/2
    rng = np.random.default_rng(11)
    c = 0.1 + 0.2j
    for _ in range(5):
        ds = rng.uniform(0.5, 1.0) / omega * 4 * np.exp(1j * rng.uniform(0, 6.3))
        s = c + ds
        x = c + 0.5 * abs(ds) * rng.uniform(0, 1) * np.exp(1j * rng.uniform(0, 6.3))
        P = 40 + int(1.5 * omega * abs(ds))
        g = T.p2l(omega, c, s, 1.0, 0.0, 1.0, P)
        val = T.l2p(omega, g, c, x)
        ref = sp.hankel1(0, omega * abs(x - s))
        assert abs(val - ref) / abs(ref) < 1e-12


@pytest.mark.parametrize("omega", [2.0, 25.0])
def test_p2m_m2m_m2l_l2l_round_trip(omega):
    """Charges and dipoles in a child box -> multipole -> parent multipole ->
    local at a well-separated box -> shifted local -> value, vs direct."""
    rng = np.random.default_rng(5)
    R = 0.5 / omega * 4  # box radius so that omega R = 2
    m_child = 0.0 + 0.0j
    s, q, qd, nu = _cluster(rng, m_child, R, 12)
    P = 60
    a = T.p2m(omega, m_child, s, q, qd, nu, P)
    m_parent = m_child + R * (1 + 1j)
    a2 = T.m2m(omega, a, m_child, m_parent, P)
    c = m_parent + 8 * R + 4j * R
    g = T.m2l(omega, a2, m_parent, c, P)
    c2 = c - 0.5 * R + 0.5j * R
    g2 = T.l2l(omega, g, c, c2, P)
    for x in [c2 + 0.3 * R, c2 - 0.2j * R, c + 0.4 * R * np.exp(2j)]:
        ref = _direct_S(omega, x, s, q) + _direct_D(omega, x, s, qd, nu)
        for val in (T.m2p(omega, a, m_child, x), T.m2p(omega, a2, m_parent, x),
                    T.l2p(omega, g, c, x), T.l2p(omega, g2, c2, x)):
            assert abs(val - ref) / abs(ref) < 1e-11


def test_p2l_dipole_matches_direct():
    omega = 7.0
    rng = np.random.default_rng(3)
    c = 0.3 - 0.1j
    s = c + 1.0 * np.exp(1j * rng.uniform(0, 6.3, 6))
    qd = inputs.complex_gaussian(rng, 6)
    nu = np.exp(1j * rng.uniform(0, 6.3, 6))
    g = T.p2l(omega, c, s, np.zeros(6), qd, nu, 60)
    for x in [c + 0.3, c + 0.25j, c - 0.2 - 0.1j]:
        ref = _direct_D(omega, x, s, qd, nu)
        assert abs(T.l2p(omega, g, c, x) - ref) / abs(ref) < 1e-12


# ---------------------------------------------------------------------------
# Direct QBX against closed forms
# ---------------------------------------------------------------------------

def _oversampled(g_nodes, q_src, n_panels, make):
    """Sources: the same panels with q_src nodes each (exact geometry, no
    interpolation); centres: those of the node discretisation."""
    src = make(n_panels, q_src)
    return src


@pytest.mark.parametrize("n", [0, 3, 7])
def test_circle_closed_forms(n):
    """S[e^{in phi}](x) = (i pi R/2) J_n(wR) H_n(w|x|) e^{in theta} and
    D[e^{in phi}](x) = (i pi R w/2) J_n'(wR) H_n(w|x|) e^{in theta} for |x|>=R;
    on the curve QBX with exterior centres yields the exterior limits."""
    omega, R, p = 10.0, 1.0, 12
    nodes = inputs.circle(64, 16, R)
    src = inputs.circle(64, 64, R)
    phi_s = np.arctan2(src.sy, src.sx)
    sig = np.exp(1j * n * phi_s)[None, :]
    # on-surface targets at the nodes, each with its own centre; plus far targets
    rng = np.random.default_rng(0)
    tx_f, ty_f = inputs.annulus_targets(rng, 40, 1.5, 2.5)
    tx = np.concatenate([nodes.sx, tx_f])
    ty = np.concatenate([nodes.sy, ty_f])
    ctr = np.concatenate([np.arange(nodes.n), -np.ones(40)]).astype(np.int32)
    geom = inputs.Geometry(sx=src.sx, sy=src.sy, w=src.w, nx=src.nx, ny=src.ny, h=src.h,
                           cx=nodes.cx, cy=nodes.cy, cr=nodes.cr, panel=src.panel, q=64)
    uS = oracle.direct_qbx(omega, p, geom, tx, ty, sig, None, tgt_ctr=ctr)[0]
    uD = oracle.direct_qbx(omega, p, geom, tx, ty, None, sig, tgt_ctr=ctr)[0]
    rho = np.hypot(tx, ty)
    th = np.arctan2(ty, tx)
    base = sp.hankel1(n, omega * rho) * np.exp(1j * n * th)
    refS = 1j * np.pi * R / 2 * sp.jv(n, omega * R) * base
    refD = 1j * np.pi * R * omega / 2 * sp.jvp(n, omega * R) * base
    errS = np.linalg.norm(uS - refS) / np.linalg.norm(refS)
    errD = np.linalg.norm(uD - refD) / np.linalg.norm(refD)
    assert errS < 1e-10 and errD < 1e-10, (errS, errD)


def _green_data(geom, omega, x0):
    d = (geom.sx - x0[0]) + 1j * (geom.sy - x0[1])
    r = np.abs(d)
    u = sp.hankel1(0, omega * r)
    dudn = -omega * sp.hankel1(1, omega * r) * (d.real * geom.nx + d.imag * geom.ny) / r
    return u, dudn


@pytest.mark.parametrize("q_src,tol", [(64, 1e-9)])
def test_greens_identity_oversampled(q_src, tol):
    """u = D[u] - S[du/dn] on and off the 5-lobe star for u = H0(w|x - x0|)
    with x0 inside (Sec. 8.1, eq. (greensid)); sources oversampled."""
    omega, p = 10.0, 12
    x0 = (0.1, 0.05)
    nodes = inputs.star(32, 16, lobes=5, amp=0.3)
    src = inputs.star(32, q_src, lobes=5, amp=0.3)
    geom = inputs.Geometry(sx=src.sx, sy=src.sy, w=src.w, nx=src.nx, ny=src.ny, h=src.h,
                           cx=nodes.cx, cy=nodes.cy, cr=nodes.cr, panel=src.panel, q=q_src)
    u_src, dudn = _green_data(src, omega, x0)
    rng = inputs.rng_for(0, inputs.PURPOSE_TARGETS)
    tx_a, ty_a = inputs.annulus_targets(rng, 1024, 1.4, 2.0)
    tx = np.concatenate([nodes.sx, tx_a])
    ty = np.concatenate([nodes.sy, ty_a])
    ctr = np.concatenate([np.arange(nodes.n), -np.ones(tx_a.size)]).astype(np.int32)
    u = oracle.direct_qbx(omega, p, geom, tx, ty, -dudn[None, :], u_src[None, :],
                          tgt_ctr=ctr)[0]
    ref = sp.hankel1(0, omega * np.hypot(tx - x0[0], ty - x0[1]))
    nb = nodes.n
    wts = nodes.w
    eps_b = np.sqrt(np.sum(np.abs(u[:nb] - ref[:nb]) ** 2 * wts) / np.sum(np.abs(ref[:nb]) ** 2 * wts))
    eps_v = np.linalg.norm(u[nb:] - ref[nb:]) / np.linalg.norm(ref[nb:])
    assert eps_b < tol and eps_v < tol, (eps_b, eps_v)


def test_greens_identity_literal_discretisation_floor():
    """Without oversampling (sources = the 16 nodes per panel) the boundary
    error is set by the quadrature floor, ~1e-4 for this curve."""
    omega, p = 10.0, 12
    x0 = (0.1, 0.05)
    g = inputs.star(32, 16, lobes=5, amp=0.3)
    u_src, dudn = _green_data(g, omega, x0)
    u = oracle.direct_qbx(omega, p, g, g.sx, g.sy, -dudn[None, :], u_src[None, :],
                          tgt_ctr=np.arange(g.n, dtype=np.int32))[0]
    ref = u_src
    err = np.sqrt(np.sum(np.abs(u - ref) ** 2 * g.w) / np.sum(np.abs(ref) ** 2 * g.w))
    assert 1e-6 < err < 1e-3


def test_coefficients_match_brute_force_formula_tiny():
    """Tiny case: coefficients from mpmath Hankel functions in a plain loop."""
    omega, p = 3.0, 4
    rng = np.random.default_rng(1)
    sx, sy = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    w = rng.uniform(0.1, 0.2, 3)
    ang = rng.uniform(0, 6.3, 3)
    nx, ny = np.cos(ang), np.sin(ang)
    ss = inputs.complex_gaussian(rng, (1, 3))
    sd = inputs.complex_gaussian(rng, (1, 3))
    cx, cy = np.array([2.0, -1.7]), np.array([0.3, 1.9])
    alpha = oracle.qbx_coefficients(omega, p, sx, sy, w, nx, ny, ss, sd, cx, cy)
    for i in range(2):
        for l in range(-p, p + 1):
            acc = mpmath.mpc(0)
            for j in range(3):
                # S: (i/4) w sigma H_l(w r) e^{i l th};  D: normal derivative in s,
                # taken here by a high-order central difference in mpmath.
                def field(px, py):
                    dx, dy = px - cx[i], py - cy[i]
                    r = mpmath.sqrt(dx * dx + dy * dy)
                    th = mpmath.atan2(dy, dx)
                    return mpmath.hankel1(l, omega * r) * mpmath.exp(1j * l * th)
                qs = 0.25j * w[j] * complex(ss[0, j])
                qd = 0.25j * w[j] * complex(sd[0, j])
                acc += qs * field(mpmath.mpf(sx[j]), mpmath.mpf(sy[j]))
                dn = mpmath.diff(lambda e: field(sx[j] + e * nx[j], sy[j] + e * ny[j]), 0)
                acc += qd * dn
            ref = complex(acc)
            got = alpha[0, l + p, i]
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (i, l, got, ref)


# ---------------------------------------------------------------------------
# Association (Sec. 6.1)
# ---------------------------------------------------------------------------

def test_association_hand_built_cases():
    # two centres of radius 1 at x = 0 and x = 1.5; one source node at (0,-1.2), h = 0.8
    cx = np.array([0.0, 1.5]); cy = np.array([0.0, 0.0]); cr = np.array([1.0, 1.0])
    sx = np.array([0.0]); sy = np.array([-1.2]); sh = np.array([0.8])
    tx = np.array([0.2, 1.3, 0.75, 0.0, 5.0, 1.02, 0.0])
    ty = np.array([0.0, 0.0, 0.0, -1.25, 5.0, 0.0, -1.04])
    got = oracle.associate(tx, ty, cx, cy, cr, sx, sy, sh, eps_assoc=0.05)
    # 0.2 -> centre 0; 1.3 -> centre 1 (nearer); 0.75 is equidistant -> lowest index 0;
    # (0,-1.25) is outside both disks but within h/4 = 0.2 of the node -> fail (-2);
    # (5,5) far -> smooth (-1); (1.02, 0): both eligible, nearer is 1;
    # (0,-1.04): outside disk 0 by 4% (< eps_assoc) -> centre 0
    assert got.tolist() == [0, 1, 0, -2, -1, 1, 0]


def test_association_brute_force_on_star_nodes():
    g = inputs.star(32, 16, lobes=5, amp=0.3)
    got = oracle.associate(g.sx, g.sy, g.cx, g.cy, g.cr, g.sx, g.sy, g.h)
    # every node lies on the boundary of its own centre's disk, so each node gets
    # an eligible centre (its own or a nearer neighbour's)
    assert (got >= 0).all()
    d_own = np.hypot(g.sx - g.cx, g.sy - g.cy)
    d_got = np.hypot(g.sx - g.cx[got], g.sy - g.cy[got])
    assert (d_got <= d_own * (1 + 1e-15)).all()


def test_m2l_quarter_turn_identity():
    """The translation of a V offset turned by r quarter turns equals the
    unturned one with inputs times i^{rk} and outputs times i^{rl} (O_n
    carries e^{in theta}); the library keeps one M2L table per orbit of
    the 40 V offsets on this identity.  Checked with the plain-sum M2L for
    every V offset against its representative (dx > 0, dy >= 0)."""
    from oracle import translations as tr
    omega, P, side = 7.0, 12, 0.3
    rng = np.random.default_rng(11)
    a = rng.standard_normal(2 * P + 1) + 1j * rng.standard_normal(2 * P + 1)
    ipow = np.array([1.0, 1j, -1.0, -1j])
    k = np.arange(-P, P + 1)
    m = 0.37 - 0.21j
    checked = 0
    for dy in range(-3, 4):
        for dx in range(-3, 4):
            if abs(dx) <= 1 and abs(dy) <= 1:
                continue
            # quarter turns back (clockwise) until the first quadrant
            x, y, r = dx, dy, 0
            while not (x > 0 and y >= 0):
                x, y, r = y, -x, r + 1
            assert r < 4
            direct = tr.m2l(omega, a, m, m + side * complex(dx, dy), P)
            turned = ipow[(r * k) % 4] * tr.m2l(omega, ipow[(r * k) % 4] * a, m,
                                                m + side * complex(x, y), P)
            assert np.max(np.abs(direct - turned)) <= 1e-12 * np.max(np.abs(direct)), (dx, dy, r)
            checked += 1
    assert checked == 40


# ---------------------------------------------------------------------------
# The stage-by-stage FMM oracle (Sec. 7.2) against the direct sum
# ---------------------------------------------------------------------------

def _fmm_geometries():
    return {"star": inputs.star(20, 16, lobes=5),
            "ellipse": inputs.ellipse(20, 16, a=1.0, b=0.35, rotation=0.3),
            "two_curves": inputs.concat([
                inputs.star(12, 16, lobes=3, radius=0.5, center=(-0.8, 0.1)),
                inputs.ellipse(12, 16, a=0.6, b=0.25, center=(0.75, -0.3))])}


@pytest.mark.parametrize("p", [8, 12])
@pytest.mark.parametrize("omega", [5.0, 30.0])
@pytest.mark.parametrize("name", ["star", "ellipse", "two_curves"])
def test_fmm_oracle_matches_direct_sum(name, omega, p):
    """oracle.fmm (Stages 1-8 box by box) reproduces the direct QBX sum over
    all sources to eps: the lists and stages only regroup that sum, and
    every translation is truncated at P_l = p_FMM(l) + p_add.  A dropped
    list, a wrong W or X definition, a sign or index slip in any stage
    leaves an O(1) part of the field wrong.  Trees with V lists on two or
    more levels and non-empty W and X lists, plain and level-restricted."""
    from oracle import fmm
    from oracle import tree as otree
    g = _fmm_geometries()[name]
    eps, p_add = 1e-8, 40
    rng = np.random.default_rng([5, int(omega), p])
    ss = inputs.complex_gaussian(rng, (1, g.n))
    sd = inputs.complex_gaussian(rng, (1, g.n))
    tc = np.arange(g.n, dtype=np.int32)
    ref = oracle.direct_qbx(omega, p, g, g.sx, g.sy, ss, sd, tgt_ctr=tc)
    lr = name != "ellipse"
    t = otree.build(g.sx, g.sy, g.cx, g.cy, 32, level_restrict=lr)
    L = otree.lists(t)
    assert len(set(lv for v, lv in zip(L["V"], t["level"]) if len(v))) >= 2
    assert sum(len(w) for w in L["W"]) > 0 and sum(len(x) for x in L["X"]) > 0
    P = fmm.orders(omega, t["R0"], int(t["level"].max()) + 1, eps, p_add)
    u, _ = fmm.qbx_fmm(omega, p, P, g, g.sx, g.sy, tc, ss, sd, 32, level_restrict=lr)
    rel = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    mx = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    assert rel <= eps and mx <= 10 * eps, (rel, mx)


def test_fmm_oracle_error_falls_with_p_add():
    """The FMM error is truncation only: it falls geometrically as the
    orders grow (Sec. 7.1), by orders of magnitude per ten extra terms."""
    from oracle import fmm
    from oracle import tree as otree
    g = _fmm_geometries()["star"]
    omega, p = 5.0, 8
    rng = np.random.default_rng(17)
    ss = inputs.complex_gaussian(rng, (1, g.n))
    tc = np.arange(g.n, dtype=np.int32)
    ref = oracle.direct_qbx(omega, p, g, g.sx, g.sy, ss, None, tgt_ctr=tc)
    t = otree.build(g.sx, g.sy, g.cx, g.cy, 32)
    errs = []
    for p_add in (10, 20, 30):
        P = fmm.orders(omega, t["R0"], int(t["level"].max()) + 1, 1e-8, p_add)
        u, _ = fmm.qbx_fmm(omega, p, P, g, g.sx, g.sy, tc, ss, None, 32)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    assert errs[0] > 100 * errs[1] > 100 * 100 * errs[2], errs


def test_fmm_oracle_without_far_field():
    """A tree of one or two levels has no V list: the FMM oracle is then the
    direct sum itself (U lists cover every source) up to rounding."""
    from oracle import fmm
    from oracle import tree as otree
    g = inputs.star(6, 8, lobes=3)
    omega, p = 8.0, 10
    rng = np.random.default_rng(23)
    ss = inputs.complex_gaussian(rng, (1, g.n))
    sd = inputs.complex_gaussian(rng, (1, g.n))
    tc = np.arange(g.n, dtype=np.int32)
    ref = oracle.direct_qbx(omega, p, g, g.sx, g.sy, ss, sd, tgt_ctr=tc)
    for n_max in (200, 40):
        t = otree.build(g.sx, g.sy, g.cx, g.cy, n_max)
        assert int(t["level"].max()) + 1 == (1 if n_max == 200 else 2)
        P = fmm.orders(omega, t["R0"], int(t["level"].max()) + 1, 1e-10, 20)
        u, _ = fmm.qbx_fmm(omega, p, P, g, g.sx, g.sy, tc, ss, sd, n_max)
        assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("eps", [1e-6, 1e-10, 1e-14])
def test_fmm_order_low_frequency_limit(eps):
    """For omega R -> 0, |H_n(3 omega R) J_n(sqrt2 omega R)| tends to
    (sqrt2/3)^n / (pi n) (leading terms of both series, DLMF 10.7.3 and
    10.7.7), so the order of Sec. 7.1 tends to the last n where that bound
    exceeds eps."""
    from oracle import fmm
    n = np.arange(1, 200)
    lim = (np.sqrt(2.0) / 3.0) ** n / (np.pi * n)
    expect = int(n[lim > eps].max())
    # keep away from a threshold crossing the O(x^2) corrections could move
    assert np.min(np.abs(np.log(lim[expect - 2:expect + 1] / eps))) > 1e-3
    assert fmm.fmm_order(1.0, 1e-4, eps) == expect


def test_fmm_order_grows_with_frequency_and_accuracy():
    """The order is non-decreasing in omega R and in 1/eps, and at high
    frequency exceeds the 3 omega R terms the Hankel factor needs to
    start decaying."""
    from oracle import fmm
    xs = [0.05, 0.5, 2.0, 8.0, 20.0]
    for eps in (1e-6, 1e-10):
        o = [fmm.fmm_order(1.0, x, eps) for x in xs]
        assert all(a <= b for a, b in zip(o, o[1:])), o
        assert o[-1] >= np.sqrt(2) * xs[-1]
    assert fmm.fmm_order(1.0, 2.0, 1e-10) > fmm.fmm_order(1.0, 2.0, 1e-6)
