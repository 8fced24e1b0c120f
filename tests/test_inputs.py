"""The seeded input recipes: properties each generator promises."""
import numpy as np

from paper_1602_05301_amd import inputs


def test_multiscale_curves_recipe():
    """64 curves, 570k-630k nodes, every panel within omega h <= 5 and
    h kappa <= c, neighbouring panels within a factor 2 in length, curves
    kept apart (nodes of different curves at least about the 0.5 gap)."""
    from scipy.spatial import cKDTree
    omega = 100.0
    g, c = inputs.multiscale_curves(omega=omega)
    parts = g.meta["parts"]
    assert len(parts) == 64
    assert 570_000 <= g.n <= 630_000
    assert np.max(np.abs(g.sx)) < 10 and np.max(np.abs(g.sy)) < 10
    q = g.q
    h = g.h[::q]
    assert omega * h.max() <= 5.0 + 1e-9
    npan = np.array([pt["n_panels"] for pt in parts])
    assert npan.sum() == h.size
    curve = np.repeat(np.arange(len(parts)), npan * q)
    # 2:1 between neighbours on each closed curve
    start = np.concatenate([[0], np.cumsum(npan)])
    for k in range(len(parts)):
        hk = h[start[k]:start[k + 1]]
        assert np.all(hk <= 2.0 * np.roll(hk, 1) + 1e-12) and np.all(hk <= 2.0 * np.roll(hk, -1) + 1e-12)
    # separation: nodes of two curves at least 0.45 apart (placement keeps
    # 0.5 between 128 sample points per curve)
    pts = [np.stack([g.sx[curve == k], g.sy[curve == k]], axis=1) for k in range(len(parts))]
    lo = np.array([p.min(axis=0) for p in pts])
    hi = np.array([p.max(axis=0) for p in pts])
    trees = [cKDTree(p) for p in pts]
    for a in range(len(parts)):
        for b in range(a + 1, len(parts)):
            if np.any(lo[a] > hi[b] + 0.45) or np.any(lo[b] > hi[a] + 0.45):
                continue
            d, _ = trees[b].query(pts[a], k=1)
            assert d.min() >= 0.45, (a, b, d.min())
    # both kinds, several sizes
    kinds = {pt["kind"] for pt in parts}
    assert kinds == {"star", "ellipse"}
    assert 0.0 < c < 10.0


def test_batched_geometries_recipe():
    """256 curves, node counts in [512, 16384] in whole panels, omega in
    [5, 150], omega times every panel's length at most 5 (Condition 4)."""
    cur = inputs.batched_geometries(256)
    assert len(cur) == 256
    n = np.array([g.n for g, _ in cur])
    assert n.min() >= 512 and n.max() <= 16384 and np.all(n % 16 == 0)
    for g, w in cur:
        assert 5.0 <= w <= 150.0
        assert w * np.max(g.h) <= 5.0 + 1e-9
