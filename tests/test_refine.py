"""Panel refinement to Conditions 1-4 (Sec. 5), checked by brute force."""
import numpy as np

from paper_1602_05301_amd import inputs
from paper_1602_05301_amd.refine import refine


def _check(curves, res, omega, tol=0.03):
    """Conditions 1-4 on the refined discretisation, by brute force over 200
    samples per panel (independent of the k-d tree path)."""
    g = res.geom
    hpan = g.h[::g.q]                                   # length of each panel, curves in order
    start = np.cumsum([0] + [e.size - 1 for e in res.edges])
    samp, hs = [], []
    for k, (f, e) in enumerate(zip(curves, res.edges)):
        t = e[:-1, None] + (e[1:, None] - e[:-1, None]) * np.linspace(0, 1, 200)[None, :]
        x, y = f(t, 0)
        samp.append(np.stack([x, y], axis=2))
        h = hpan[start[k]:start[k + 1]]
        hs.append(h)
        assert np.all(h <= 2 * np.roll(h, 1) * (1 + 1e-12)) and np.all(h <= 2 * np.roll(h, -1) * (1 + 1e-12))
        assert omega * h.max() <= 5.0 + 1e-9
    pts = np.concatenate(samp)                          # [panels, 200, 2]
    hp = np.concatenate(hs)
    c = np.stack([g.cx, g.cy], axis=1)
    hk = g.h
    d = np.sqrt(((c[:, None, None, :] - pts[None]) ** 2).sum(axis=3)).min(axis=2)   # [centres, panels]
    assert np.all(d.min(axis=1) >= (1 - tol) * 0.5 * hk), "condition 1"
    assert np.all(d >= (1 - tol) * 0.25 * hp[None, :]), "condition 3"


def test_refine_noop_when_conditions_hold():
    f = inputs._shape("ellipse", 1.0, 1.5, 0.0, (0.0, 0.0))
    e0 = np.linspace(0, 2 * np.pi, 33)
    res = refine([f], omega=2.0, edges=[e0])
    assert res.rounds == 0 and res.bisected == 0
    assert np.array_equal(res.edges[0], e0)


def test_refine_wavelength_only():
    """A circle of radius 1 at omega = 40: only condition 4 acts, so the
    panels double until 40 (2 pi / n) <= 5: n = 64 from 8."""
    circ = lambda t, d: (np.cos(t), np.sin(t)) if d == 0 else (-np.sin(t), np.cos(t))
    res = refine([circ], omega=40.0)
    n = res.edges[0].size - 1
    assert n == 64, n
    _check([circ], res, 40.0)


def test_refine_close_curves():
    """Two ellipses 0.02 apart, coarse panels: conditions 1 and 3 bisect the
    facing panels (and 2 grades them) until every condition holds."""
    f1 = inputs._shape("ellipse", 1.0, 2.0, 0.0, (0.0, 0.0))
    f2 = inputs._shape("ellipse", 1.0, 2.0, 0.0, (2.02, 0.0))
    res = refine([f1, f2], omega=3.0)
    assert res.rounds > 2 and res.bisected > 0
    n1 = res.edges[0].size - 1
    h1 = res.geom.h[::16][:n1]
    assert h1.max() / h1.min() > 8              # graded towards the gap
    _check([f1, f2], res, 3.0)


def _geom_and_panels(curves, edges, q=16):
    from paper_1602_05301_amd import refine as R
    parts, owner = [], []
    for ci, (f, e) in enumerate(zip(curves, edges)):
        out = inputs._panelize(e, q, lambda th, f=f: f(th, 0), lambda th, f=f: f(th, 1))
        parts.append(inputs._finish(*out, q, {}))
        owner.append(np.full(e.size - 1, ci))
    g = inputs.concat(parts)
    return g, R.panels_of(g, np.concatenate(owner))


def _dense(P, k, n=4001):
    t = np.linspace(-1.0, 1.0, n)
    V = np.polynomial.legendre.legvander(t, P.cx.shape[1] - 1)
    return P.cx[k] @ V.T, P.cy[k] @ V.T


def test_legendre_fit_reproduces_polynomials():
    """The interpolant through q Gauss nodes is exact for degree < q: the
    fitted coefficients of a random degree-15 Legendre series are its own."""
    from paper_1602_05301_amd.refine import legendre_fit_matrix
    rng = np.random.default_rng(3)
    c = rng.standard_normal(16)
    x, _ = np.polynomial.legendre.leggauss(16)
    got = legendre_fit_matrix(16) @ np.polynomial.legendre.legval(x, c)
    assert np.allclose(got, c, atol=1e-13)


def test_panel_geometry_against_dense_samples():
    """Centre of mass of a straight panel is its midpoint; every point of a
    curved panel lies in Z_k; exact distances agree with the minimum over
    4001 samples of the panel to within the samples' spacing error, and are
    never larger."""
    from paper_1602_05301_amd.refine import panel_distance
    line = lambda t, d: (np.stack([t, 0.5 * t]) if d == 0 else np.stack([np.ones_like(t), 0.5 * np.ones_like(t)]))
    g, P = _geom_and_panels([line], [np.array([0.0, 2.0])])
    assert np.allclose([P.mx[0], P.my[0]], [1.0, 0.5], atol=1e-13)
    f = inputs._shape("star", 1.0, 5, 0.3, (0.0, 0.0))
    g, P = _geom_and_panels([f], [np.linspace(0.0, 2.0 * np.pi, 13)])
    rng = np.random.default_rng(5)
    for k in range(P.h.size):
        x, y = _dense(P, k)
        assert np.max(np.maximum(np.abs(x - P.mx[k]), np.abs(y - P.my[k]))) <= P.r[k]
    n = 400
    k = rng.integers(0, P.h.size, n)
    px = P.mx[k] + rng.uniform(-1, 1, n) * 2 * P.h[k]
    py = P.my[k] + rng.uniform(-1, 1, n) * 2 * P.h[k]
    d = panel_distance(P, px, py, k)
    for i in range(n):
        x, y = _dense(P, k[i])
        brute = np.sqrt(((x - px[i]) ** 2 + (y - py[i]) ** 2).min())
        assert d[i] <= brute + 1e-12 and d[i] >= brute - 1e-6 * P.h[k[i]], (i, d[i], brute)


def test_adjacency_is_cyclic_per_curve():
    from paper_1602_05301_amd.refine import _adjacent
    g, P = _geom_and_panels([inputs._shape("ellipse", 1.0, 2.0, 0.0, (0.0, 0.0)),
                             inputs._shape("ellipse", 1.0, 2.0, 0.0, (5.0, 0.0))],
                            [np.linspace(0, 2 * np.pi, 7), np.linspace(0, 2 * np.pi, 5)])
    n = np.array([0, 0, 0, 0, 5, 6, 6, 9])
    k = np.array([0, 1, 5, 2, 0, 7, 9, 6])
    assert _adjacent(P, n, k).tolist() == [True, True, True, False, True, True, True, True]
    assert not _adjacent(P, np.array([5]), np.array([6]))      # different curves


def test_conditions_1_3_against_brute_force():
    """Flags of Conditions 1 and 3 on two close ellipses and a star, by the
    area-query candidates and exact distances, equal those of a brute-force
    pass over every (centre, panel) pair with 4001 samples per panel."""
    from paper_1602_05301_amd.refine import _adjacent, conditions_1_3
    curves = [inputs._shape("ellipse", 1.0, 2.0, 0.0, (0.0, 0.0)),
              inputs._shape("ellipse", 1.0, 2.0, 0.0, (2.05, 0.0)),
              inputs._shape("star", 0.6, 5, 0.3, (0.9, 2.9))]
    edges = [np.linspace(0.0, 2.0 * np.pi, 13) for _ in curves]
    g, P = _geom_and_panels(curves, edges)
    f1, f3 = conditions_1_3(P, g.cx, g.cy, g.panel)
    npan, nc = P.h.size, g.cx.size
    D = np.empty((nc, npan))
    for k in range(npan):
        x, y = _dense(P, k)
        D[:, k] = np.sqrt(((g.cx[:, None] - x[None]) ** 2 + (g.cy[:, None] - y[None]) ** 2).min(axis=1))
    cp = g.panel
    own = cp[:, None] == np.arange(npan)[None, :]
    t1 = 0.5 * P.h[cp][:, None]
    b1 = np.zeros(npan, bool)
    b1[cp[((D <= t1) & ~own).any(axis=1)]] = True
    nn, kk = np.meshgrid(cp, np.arange(npan), indexing="ij")
    adj = _adjacent(P, nn.ravel(), kk.ravel()).reshape(nc, npan)
    t3 = 0.25 * P.h[None, :]
    b3 = ((D <= t3) & ~adj).any(axis=0)
    # no pair sits within the samples' error of its threshold
    assert np.min(np.abs(D - t1)[~own]) > 1e-6 * P.h.min()
    assert np.min(np.abs(D - t3)[~adj]) > 1e-6 * P.h.min()
    assert b1.any() and b3.any()
    assert np.array_equal(f1, b1) and np.array_equal(f3, b3)
