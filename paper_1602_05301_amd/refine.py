"""Panel refinement to the paper's geometric conditions (Sec. 5).

A discretisation of closed parametric curves into theta-panels of q Gauss
nodes, each node with the QBX centre s + (h/2) n, is refined by bisecting
flagged panels until

  1. no panel other than its own comes within h_n / 2 of a centre of panel
     n (the expansion disk holds no sources; flags panel n);
  2. adjacent panels differ in length by at most a factor 2;
  3. no centre of a panel other than k or its two neighbours comes within
     h_k / 4 of panel k (quadrature from panel k resolved at every centre;
     flags panel k);
  4. omega h <= 5 for every panel (panel size against the wavelength).

Conditions 1 and 3 are checked as in Sec. 5.1 and 5.2 of the paper:

  * A panel is the Legendre interpolant of degree q - 1 through its q nodes
    (its parametrisation on [-1, 1]); m_k is its centre of mass (the nodes
    weighted by their quadrature weights), Z_k the smallest l-inf square
    about m_k that holds it (radius r_k), and d(c, panel) the exact distance
    from a point to that curve piece (the closest of 33 samples, refined by
    Newton's method on the squared distance).
  * Condition 1: the panels whose Z_k meets a leaf form the leaf's list
    S(b); each centre queries the square C of radius h_n / 2 about it and
    tests the panels of the leaves it meets.
  * Condition 3: each panel queries the square of radius r_k + h_k / 4
    about m_k (it holds the tube of points within h_k / 4 of the panel) and
    tests the centres of the leaves it meets.

The paper's listing for Condition 3 flags the centre's panel; its text and
figure flag the panel whose quadrature is under-resolved (k), which is what
is done here.  Given a qbx.Context, the tree over the centres and the
panels' centres of mass and the area queries run on the device (qbx
area_query); without one, a host k-d tree in the l-inf norm gives the
candidates.  Both candidate sets hold every (point, panel) pair within the
tested distance, and the exact tests decide, so both give the same flags.

The curves are callables f(t, d) returning the d-th theta-derivative
(d = 0, 1) of (x(t), y(t)) for t in [0, 2 pi], counter-clockwise (outward
normal (y', -x') / |gamma'|), as inputs._shape builds them.
"""
from __future__ import annotations

import dataclasses
import types

import numpy as np

from . import inputs

N_SAMPLE = 33          # samples per panel that start the distance search
N_NEWTON = 8           # Newton steps after them
BOX_MARGIN = 0.01      # Z_k widened by this fraction (it only adds candidates)
CHUNK = 200_000        # (point, panel) pairs per vectorised distance pass


@dataclasses.dataclass
class Refined:
    edges: list            # per curve: theta panel edges
    geom: inputs.Geometry  # q Gauss nodes per panel, centres at h/2
    rounds: int
    bisected: int          # panels bisected in all


@dataclasses.dataclass
class Panels:
    """Each panel's interpolant and the data of the area queries."""
    cx: np.ndarray         # [n, q] Legendre coefficients of x(tau)
    cy: np.ndarray
    mx: np.ndarray         # centres of mass
    my: np.ndarray
    r: np.ndarray          # radius of Z_k
    h: np.ndarray          # panel lengths
    curve: np.ndarray      # owning curve
    index: np.ndarray      # index within the curve
    count: np.ndarray      # panels of the owning curve


def legendre_fit_matrix(q: int) -> np.ndarray:
    """T with c = T f: the Legendre coefficients (degree < q) of the
    interpolant through values f at the q Gauss-Legendre nodes.  Gauss
    quadrature of f P_n is exact for the interpolant's degree."""
    x, w = np.polynomial.legendre.leggauss(q)
    V = np.polynomial.legendre.legvander(x, q - 1)           # V[j, n] = P_n(x_j)
    return ((2.0 * np.arange(q) + 1.0) / 2.0)[:, None] * (V * w[:, None]).T


def panels_of(geom, owner: np.ndarray) -> Panels:
    """Interpolants, centres of mass and Z_k of the panels of `geom` (nodes
    in panel order, q per panel); owner[k] is panel k's curve."""
    q = geom.q
    n = geom.sx.size // q
    T = legendre_fit_matrix(q)
    cx = geom.sx.reshape(n, q) @ T.T
    cy = geom.sy.reshape(n, q) @ T.T
    w = geom.w.reshape(n, q)
    mx = (w * geom.sx.reshape(n, q)).sum(axis=1) / w.sum(axis=1)
    my = (w * geom.sy.reshape(n, q)).sum(axis=1) / w.sum(axis=1)
    V = np.polynomial.legendre.legvander(np.linspace(-1.0, 1.0, 129), q - 1)
    r = np.maximum(np.abs(cx @ V.T - mx[:, None]), np.abs(cy @ V.T - my[:, None])).max(axis=1)
    counts = np.bincount(owner)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    return Panels(cx, cy, mx, my, r * (1.0 + BOX_MARGIN), geom.h[::q].copy(), owner,
                  np.arange(n) - first[owner], counts[owner])


def _rows(C, V):
    return np.einsum("ij,ij->i", C, V)


def panel_distance(P: Panels, px, py, k) -> np.ndarray:
    """Distance from each point (px[i], py[i]) to panel k[i]: the closest
    of N_SAMPLE points of the panel, then Newton's method on the squared
    distance from there (kept only where it comes closer)."""
    out = np.empty(px.size)
    q = P.cx.shape[1]
    ts = np.linspace(-1.0, 1.0, N_SAMPLE)
    Vs = np.polynomial.legendre.legvander(ts, q - 1)
    der = lambda C: np.polynomial.legendre.legder(C, axis=1)
    for a in range(0, px.size, CHUNK):
        b = min(px.size, a + CHUNK)
        kk, x0, y0 = k[a:b], px[a:b], py[a:b]
        CX, CY = P.cx[kk], P.cy[kk]
        d2 = (CX @ Vs.T - x0[:, None]) ** 2 + (CY @ Vs.T - y0[:, None]) ** 2
        j = d2.argmin(axis=1)
        best = d2[np.arange(kk.size), j]
        t = ts[j]
        DX, DY = der(CX), der(CY)
        DDX, DDY = der(DX), der(DY)
        for _ in range(N_NEWTON):
            V = np.polynomial.legendre.legvander(t, q - 1)
            ex, ey = _rows(CX, V) - x0, _rows(CY, V) - y0
            dx, dy = _rows(DX, V[:, :q - 1]), _rows(DY, V[:, :q - 1])
            ddx, ddy = _rows(DDX, V[:, :q - 2]), _rows(DDY, V[:, :q - 2])
            g = ex * dx + ey * dy
            gp = dx * dx + dy * dy + ex * ddx + ey * ddy
            step = np.where(gp > 0.0, g / np.where(gp > 0.0, gp, 1.0), 0.0)
            t = np.clip(t - step, -1.0, 1.0)
        V = np.polynomial.legendre.legvander(t, q - 1)
        dn = (_rows(CX, V) - x0) ** 2 + (_rows(CY, V) - y0) ** 2
        out[a:b] = np.sqrt(np.minimum(best, dn))
    return out


def _expand(a, leaf, item_leaf, n_leaves):
    """Join (a, leaf) pairs with the items filed under each leaf: the
    (a, item) pairs, duplicates removed."""
    order = np.argsort(item_leaf, kind="stable")
    counts = np.bincount(item_leaf, minlength=n_leaves)
    starts = np.concatenate([[0], np.cumsum(counts)])
    reps = counts[leaf]
    tot = int(reps.sum())
    if tot == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    a_rep = np.repeat(a, reps)
    off = np.repeat(starts[leaf] - np.concatenate([[0], np.cumsum(reps)[:-1]]), reps) + np.arange(tot)
    items = order[off]
    key = np.unique(a_rep.astype(np.int64) * (int(item_leaf.size) + 1) + items)
    return key // (item_leaf.size + 1), key % (item_leaf.size + 1)


def _pairs_device(ctx, P: Panels, cxs, cys, hn, leaf_max: int = 32):
    """Candidate pairs by the paper's area-query algorithms on the device:
    (centre, panel) for Condition 1 and (panel, centre) for Condition 3."""
    import torch
    from . import qbx
    npan, nc = P.mx.size, cxs.size
    # the tree holds the panels' centres of mass (as sources) and the centres
    pseudo = types.SimpleNamespace(sx=P.mx, sy=P.my, w=np.zeros(npan), nx=np.ones(npan),
                                   ny=np.zeros(npan), h=P.h, cx=cxs, cy=cys, cr=0.5 * hn)
    geo = qbx.Geometry(ctx, pseudo, 1.0, 1e-6, np.zeros(0), np.zeros(0), None,
                       qbx.options(p=1, direct=True, leaf_max=leaf_max))
    nb = geo.stats()["n_boxes"]
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(f"cuda:{ctx.device}")

    def query(x, y, r):
        start, leaves = geo.area_query(dev(x), dev(y), dev(r))
        start, leaves = start.cpu().numpy(), leaves.cpu().numpy().astype(np.int64)
        return np.repeat(np.arange(x.size), np.diff(start)), leaves

    # Condition 1: S(b) from the squares Z_k, then the squares C about the centres
    k_of, leaf_k = query(P.mx, P.my, P.r)
    i_of, leaf_i = query(cxs, cys, 0.5 * hn)
    # _expand files items by leaf: here the items are the (panel, leaf) pairs
    pi, pk = _expand(i_of, leaf_i, leaf_k, nb)
    pairs1 = (pi, k_of[pk])
    # Condition 3: E(b) from the centres' own leaves, then the squares about m_k
    c_of, leaf_c = query(cxs, cys, np.zeros(nc))
    k3, leaf3 = query(P.mx, P.my, P.r + 0.25 * P.h)
    qk, qc = _expand(k3, leaf3, leaf_c, nb)
    pairs3 = (qk, c_of[qc])
    return _unique(*pairs1), _unique(*pairs3)


def _unique(a, b):
    if a.size == 0:
        return a, b
    m = int(b.max()) + 1
    key = np.unique(a.astype(np.int64) * m + b)
    return key // m, key % m


def _pairs_host(P: Panels, cxs, cys, hn):
    """Candidate pairs from host k-d trees in the l-inf norm: for Condition 1
    every panel whose Z_k meets the square C about a centre, for Condition 3
    every centre in the square of radius r_k + h_k / 4 about m_k."""
    from scipy.spatial import cKDTree
    tm = cKDTree(np.stack([P.mx, P.my], axis=1))
    a, b = [], []
    rmax = float(P.r.max())
    for i, nb in enumerate(tm.query_ball_point(np.stack([cxs, cys], axis=1), 0.5 * hn + rmax, p=np.inf)):
        if nb:
            nb = np.asarray(nb)
            ok = np.maximum(np.abs(P.mx[nb] - cxs[i]), np.abs(P.my[nb] - cys[i])) <= 0.5 * hn[i] + P.r[nb]
            a.append(np.full(int(ok.sum()), i))
            b.append(nb[ok])
    pairs1 = (np.concatenate(a) if a else np.zeros(0, np.int64), np.concatenate(b) if b else np.zeros(0, np.int64))
    tc = cKDTree(np.stack([cxs, cys], axis=1))
    a, b = [], []
    for k, nb in enumerate(tc.query_ball_point(np.stack([P.mx, P.my], axis=1), P.r + 0.25 * P.h, p=np.inf)):
        if nb:
            a.append(np.full(len(nb), k))
            b.append(np.asarray(nb))
    pairs3 = (np.concatenate(a) if a else np.zeros(0, np.int64), np.concatenate(b) if b else np.zeros(0, np.int64))
    return _unique(*pairs1), _unique(*pairs3)


def _adjacent(P: Panels, n, k):
    """Whether panels n and k are the same panel or neighbours on one curve."""
    same = P.curve[n] == P.curve[k]
    d = np.abs(P.index[n] - P.index[k])
    return same & ((d <= 1) | (d == P.count[k] - 1))


def conditions_1_3(P: Panels, cxs, cys, cpan, ctx=None):
    """Panels flagged by Condition 1 (a foreign panel within h_n / 2 of a
    centre of panel n: flags n) and Condition 3 (a centre of a panel that is
    neither k nor its neighbour within h_k / 4 of panel k: flags k)."""
    hn = P.h[cpan]
    (i1, k1), (k3, c3) = (_pairs_device(ctx, P, cxs, cys, hn) if ctx is not None
                          else _pairs_host(P, cxs, cys, hn))
    flag1 = np.zeros(P.h.size, bool)
    flag3 = np.zeros(P.h.size, bool)
    keep = k1 != cpan[i1]
    i1, k1 = i1[keep], k1[keep]
    if i1.size:
        d = panel_distance(P, cxs[i1], cys[i1], k1)
        flag1[cpan[i1[d <= 0.5 * hn[i1]]]] = True
    keep = ~_adjacent(P, cpan[c3], k3)
    k3, c3 = k3[keep], c3[keep]
    if k3.size:
        d = panel_distance(P, cxs[c3], cys[c3], k3)
        flag3[k3[d <= 0.25 * P.h[k3]]] = True
    return flag1, flag3


def flags(curves, edges, omega: float, q: int = 16, ctx=None):
    """Panels violating each condition: list over curves of boolean arrays
    (cond1, cond2, cond3, cond4), plus the discretisation.  With ctx (a
    qbx.Context), the area queries of Conditions 1 and 3 run on the device."""
    parts, owner = [], []
    for ci, (f, e) in enumerate(zip(curves, edges)):
        out = inputs._panelize(e, q, lambda th: f(th, 0), lambda th: f(th, 1))
        parts.append(inputs._finish(*out, q, dict(n_panels=e.size - 1)))
        owner.append(np.full(e.size - 1, ci))
    geom = inputs.concat(parts)
    P = panels_of(geom, np.concatenate(owner))
    c1, c3 = conditions_1_3(P, geom.cx, geom.cy, geom.panel, ctx)
    out, off = [], 0
    for e in edges:
        n = e.size - 1
        h = P.h[off:off + n]
        c2 = (h > 2.0 * np.roll(h, 1)) | (h > 2.0 * np.roll(h, -1))
        c4 = omega * h > 5.0
        out.append((c1[off:off + n], c2, c3[off:off + n], c4))
        off += n
    return out, geom


def refine(curves, omega: float, edges=None, q: int = 16, start: int = 8, max_rounds: int = 40,
           ctx=None) -> Refined:
    """Bisect flagged panels (conditions 1-4) until none is flagged; with
    ctx, the area queries run on the device (see flags)."""
    edges = [np.linspace(0.0, 2.0 * np.pi, start + 1) if edges is None else np.asarray(edges[i], float)
             for i in range(len(curves))]
    total = 0
    for rnd in range(max_rounds):
        fl, geom = flags(curves, edges, omega, q, ctx)
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
