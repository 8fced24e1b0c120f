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
