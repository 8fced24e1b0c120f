"""Panel refinement to the paper's geometric conditions (Sec. 5).

A discretisation of closed parametric curves into theta-panels of q Gauss
nodes, each node with the QBX centre s + (h/2) n, is refined by bisecting
flagged panels until

  1. every centre c of panel k is at least h_k / 2 from the curve
     (expansion disk undisturbed by sources; eq. dcgam, per panel);
  2. adjacent panels differ in length by at most a factor 2;
  3. every centre is at least h_l / 4 from every source panel l
     (sufficient quadrature resolution from all panels to all centres);
  4. omega h <= 5 for every panel (panel size against the wavelength).

Distances from a centre to a panel are taken to dense samples of the panel
(n_samp points, ends included), found with a k-d tree on the host or, given
a qbx.Context, through area queries on the device (Sec. 5: a geometry whose
sources are the samples and whose centres are the QBX centres, and disk
tests qbx_geom_points_near); `slack` shortens the required distances by the
samples' spacing so that a panel is not flagged for sampling error alone.
Condition 1 flags the centre's own panel; 3 flags the source panel that is
too close (a shorter panel needs less clearance).

The curves are callables f(t, d) returning the d-th theta-derivative
(d = 0, 1) of (x(t), y(t)) for t in [0, 2 pi], counter-clockwise (outward
normal (y', -x') / |gamma'|), as inputs._shape builds them.
"""
from __future__ import annotations

import dataclasses
import types

import numpy as np

from . import inputs


@dataclasses.dataclass
class Refined:
    edges: list            # per curve: theta panel edges
    geom: inputs.Geometry  # q Gauss nodes per panel, centres at h/2
    rounds: int
    bisected: int          # panels bisected in all


def _panel_samples(f, e, n_samp):
    """Points along each panel (n_samp per panel, ends included) and panel lengths."""
    a, b = e[:-1, None], e[1:, None]
    t = a + (b - a) * np.linspace(0.0, 1.0, n_samp)[None, :]
    x, y = f(t, 0)
    xg, wg = np.polynomial.legendre.leggauss(16)
    half = 0.5 * (b - a)
    tg = 0.5 * (a + b) + half * xg[None, :]
    dx, dy = f(tg, 1)
    h = (half[:, 0] * (wg[None, :] * np.hypot(dx, dy)).sum(axis=1))
    return np.stack([x, y], axis=2), h


def _device_near(ctx, pts, c, h_all, pan_of_pt, hk, gapf, omega):
    """Conditions 1 and 3 per query through area queries on the device: for
    each centre, whether a sample lies within gapf h_k / 2; for each sample
    of panel l, whether a centre lies within gapf h_l / 4."""
    import torch
    from . import qbx
    ns, nc = pts.shape[0], c.shape[0]
    # sources = samples (weights and normals are placeholders: only the
    # tree and the points are used), centres = the QBX centres, no targets
    pseudo = types.SimpleNamespace(sx=pts[:, 0], sy=pts[:, 1], w=np.zeros(ns), nx=np.ones(ns),
                                   ny=np.zeros(ns), h=h_all[pan_of_pt], cx=c[:, 0], cy=c[:, 1],
                                   cr=0.5 * hk)
    geo = qbx.Geometry(ctx, pseudo, omega, 1e-6, np.zeros(0), np.zeros(0), None,
                       qbx.options(p=1, direct=True))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(f"cuda:{ctx.device}")
    near1 = geo.points_near("sources", dev(c[:, 0]), dev(c[:, 1]), dev(gapf * 0.5 * hk)).cpu().numpy()
    near3 = geo.points_near("centres", dev(pts[:, 0]), dev(pts[:, 1]),
                            dev(gapf * 0.25 * h_all[pan_of_pt])).cpu().numpy()
    return near1, near3


def flags(curves, edges, omega: float, q: int = 16, n_samp: int = 33, slack: float = 0.02, ctx=None):
    """Panels violating each condition: list over curves of boolean arrays
    (cond1, cond2, cond3, cond4), plus the discretisation.  With ctx (a
    qbx.Context), Conditions 1 and 3 are found through area queries on the
    device instead of a host k-d tree."""
    from scipy.spatial import cKDTree
    parts, samp, hs, owner = [], [], [], []
    for ci, (f, e) in enumerate(zip(curves, edges)):
        out = inputs._panelize(e, q, lambda th: f(th, 0), lambda th: f(th, 1))
        parts.append(inputs._finish(*out, q, dict(n_panels=e.size - 1)))
        pts, h = _panel_samples(f, e, n_samp)
        samp.append(pts)
        hs.append(h)
        owner.append(np.full(e.size - 1, ci))
    geom = inputs.concat(parts)
    h_all = np.concatenate(hs)
    npan = h_all.size
    pts_all = np.concatenate(samp).reshape(-1, 2)
    pan_of_pt = np.repeat(np.arange(npan), n_samp)
    cpan = geom.panel                                  # panel of each centre (global numbering)
    c = np.stack([geom.cx, geom.cy], axis=1)
    hk = h_all[cpan]
    gapf = 1.0 - slack
    c1 = np.zeros(npan, bool)
    c3 = np.zeros(npan, bool)
    if ctx is not None:
        near1, near3 = _device_near(ctx, pts_all, c, h_all, pan_of_pt, hk, gapf, omega)
        c1[cpan[near1]] = True
        c3[pan_of_pt[near3]] = True
    else:
        tree = cKDTree(pts_all)
        # 1: any sample of any panel within h_k/2 of a centre of panel k
        for i, nb in enumerate(tree.query_ball_point(c, gapf * 0.5 * hk)):
            if nb:
                c1[cpan[i]] = True
        # 3: a sample of panel l within h_l/4 of any centre
        rmax = gapf * 0.25 * h_all.max()
        for i, nb in enumerate(tree.query_ball_point(c, rmax)):
            if not nb:
                continue
            nb = np.asarray(nb)
            d = np.hypot(pts_all[nb, 0] - c[i, 0], pts_all[nb, 1] - c[i, 1])
            bad = d <= gapf * 0.25 * h_all[pan_of_pt[nb]]
            c3[pan_of_pt[nb[bad]]] = True
    # 2 and 4, per curve
    out, off = [], 0
    for h in hs:
        n = h.size
        c2 = (h > 2.0 * np.roll(h, 1)) | (h > 2.0 * np.roll(h, -1))
        c4 = omega * h > 5.0
        out.append((c1[off:off + n], c2, c3[off:off + n], c4))
        off += n
    return out, geom


def refine(curves, omega: float, edges=None, q: int = 16, start: int = 8, max_rounds: int = 40,
           n_samp: int = 33, slack: float = 0.02, ctx=None) -> Refined:
    """Bisect flagged panels (conditions 1-4) until none is flagged; with
    ctx, Conditions 1 and 3 are found on the device (see flags)."""
    edges = [np.linspace(0.0, 2.0 * np.pi, start + 1) if edges is None else np.asarray(edges[i], float)
             for i in range(len(curves))]
    total = 0
    for rnd in range(max_rounds):
        fl, geom = flags(curves, edges, omega, q, n_samp, slack, ctx)
        nflag = 0
        new = []
        for e, (a, b, c, d) in zip(edges, fl):
            bad = a | b | c | d
            nflag += int(bad.sum())
            if bad.any():
                mid = 0.5 * (e[:-1] + e[1:])[bad]
                e = np.sort(np.concatenate([e, mid]))
            new.append(e)
        if nflag == 0:
            return Refined(edges, geom, rnd, total)
        total += nflag
        edges = new
    raise RuntimeError("refine: conditions not met after %d rounds" % max_rounds)
