"""Seeded synthetic workloads: curve discretisations, targets and densities.

This module is shared by the oracle's tests, the GPU tests and the benchmark.
It holds none of the method's arithmetic (no kernels, expansions or Bessel
functions): it only produces the inputs that the paper's problem statement
takes, i.e. Gauss-Legendre panel nodes on a closed curve with their arclength
weights, outward unit normals and panel lengths (Sec. 2.2, "Geometry
discretization"), one QBX centre per node at distance h_k/2 along the normal
(Sec. 2.2), targets, and complex densities.

Conventions
-----------
* A curve is traversed counter-clockwise; the outward normal is the unit
  tangent rotated by -90 degrees.
* Panels are equal intervals of the curve parameter theta; each carries q
  Gauss-Legendre nodes in theta.  The weight of node j on panel k is
  w_j^GL * (dtheta/2) * |gamma'(theta_j)|, so that sum_j w_j f(s_j) is the
  composite Gauss rule for the arclength integral.  The panel length h_k is
  the sum of its weights.
* Seeds: ``np.random.default_rng([workload_id, purpose])`` with purpose
  0 = geometry, 1 = targets, 2 = densities.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PURPOSE_GEOMETRY = 0
PURPOSE_TARGETS = 1
PURPOSE_DENSITY = 2


def rng_for(workload_id: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng([int(workload_id), int(purpose)])


@dataclass
class Geometry:
    """Discretised closed curve(s) with one QBX centre per node.

    Arrays are float64 of length n (nodes = sources = centres)."""

    sx: np.ndarray
    sy: np.ndarray
    w: np.ndarray        # arclength quadrature weights w_{j,k}
    nx: np.ndarray
    ny: np.ndarray
    h: np.ndarray        # length of the panel each node belongs to
    cx: np.ndarray       # QBX centre  s + (h/2) n
    cy: np.ndarray
    cr: np.ndarray       # expansion radius h/2
    panel: np.ndarray    # panel index of each node (int64)
    q: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.sx.size)


def _gl(q: int):
    x, wq = np.polynomial.legendre.leggauss(q)
    return x, wq


def _panelize(theta_edges, q, gamma, dgamma):
    """Gauss-Legendre nodes in theta on each interval of ``theta_edges``."""
    x, wq = _gl(q)
    a = theta_edges[:-1][:, None]
    b = theta_edges[1:][:, None]
    half = 0.5 * (b - a)
    th = (0.5 * (a + b) + half * x[None, :]).ravel()
    px, py = gamma(th)
    dx, dy = dgamma(th)
    speed = np.hypot(dx, dy)
    w = (wq[None, :] * half).ravel() * speed
    npan = theta_edges.size - 1
    h = w.reshape(npan, q).sum(axis=1)
    nx = dy / speed
    ny = -dx / speed
    panel = np.repeat(np.arange(npan, dtype=np.int64), q)
    return px, py, w, nx, ny, np.repeat(h, q), panel


def _finish(px, py, w, nx, ny, h, panel, q, meta) -> Geometry:
    r = 0.5 * h
    return Geometry(sx=px, sy=py, w=w, nx=nx, ny=ny, h=h,
                    cx=px + r * nx, cy=py + r * ny, cr=r, panel=panel, q=q,
                    meta=meta)


def star(n_panels: int, q: int = 16, lobes: int = 5, amp: float = 0.3,
         radius: float = 1.0, center=(0.0, 0.0), rotation: float = 0.0) -> Geometry:
    """Star curve r(theta) = radius*(1 + amp*cos(lobes*theta)), equal-theta panels."""
    c0, s0 = np.cos(rotation), np.sin(rotation)

    def gamma(t):
        r = radius * (1.0 + amp * np.cos(lobes * t))
        x, y = r * np.cos(t), r * np.sin(t)
        return center[0] + c0 * x - s0 * y, center[1] + s0 * x + c0 * y

    def dgamma(t):
        r = radius * (1.0 + amp * np.cos(lobes * t))
        dr = -radius * amp * lobes * np.sin(lobes * t)
        x = dr * np.cos(t) - r * np.sin(t)
        y = dr * np.sin(t) + r * np.cos(t)
        return c0 * x - s0 * y, s0 * x + c0 * y

    edges = np.linspace(0.0, 2.0 * np.pi, n_panels + 1)
    out = _panelize(edges, q, gamma, dgamma)
    return _finish(*out, q, dict(kind="star", lobes=lobes, amp=amp, radius=radius,
                                  n_panels=n_panels))


def ellipse(n_panels: int, q: int = 16, a: float = 1.0, b: float = 0.5,
            center=(0.0, 0.0), rotation: float = 0.0) -> Geometry:
    c0, s0 = np.cos(rotation), np.sin(rotation)

    def gamma(t):
        x, y = a * np.cos(t), b * np.sin(t)
        return center[0] + c0 * x - s0 * y, center[1] + s0 * x + c0 * y

    def dgamma(t):
        x, y = -a * np.sin(t), b * np.cos(t)
        return c0 * x - s0 * y, s0 * x + c0 * y

    edges = np.linspace(0.0, 2.0 * np.pi, n_panels + 1)
    out = _panelize(edges, q, gamma, dgamma)
    return _finish(*out, q, dict(kind="ellipse", a=a, b=b, n_panels=n_panels))


def circle(n_panels: int, q: int = 16, radius: float = 1.0) -> Geometry:
    return star(n_panels, q, lobes=1, amp=0.0, radius=radius)


@dataclass
class Points:
    """Sources and centres as the library takes them, without the one
    centre per node pairing of Geometry: sources sx, sy, w, nx, ny, h
    (length n_src), centres cx, cy, cr (length n_ctr)."""

    sx: np.ndarray
    sy: np.ndarray
    w: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    h: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    cr: np.ndarray

    @property
    def n(self) -> int:
        return int(self.sx.size)


def two_sided(geom: Geometry, sources: Geometry | None = None) -> Points:
    """Centres on both sides of the curve: node j's exterior centre
    s_j + (h/2) n_j at index j and its interior centre s_j - (h/2) n_j at
    index n + j.  Binding an on-curve target to one or the other selects the
    exterior or the interior limit (side preference); their average is the
    on-surface value.  `sources` (default: the nodes) may be an oversampled
    grid of the same curve."""
    src = geom if sources is None else sources
    r = 0.5 * geom.h
    return Points(src.sx, src.sy, src.w, src.nx, src.ny, src.h,
                  np.concatenate([geom.sx + r * geom.nx, geom.sx - r * geom.nx]),
                  np.concatenate([geom.sy + r * geom.ny, geom.sy - r * geom.ny]),
                  np.concatenate([r, r]))


def concat(geoms) -> Geometry:
    """Several disjoint curves as one discretisation (panel ids renumbered)."""
    off = 0
    panels = []
    for g in geoms:
        panels.append(g.panel + off)
        off += int(g.panel.max()) + 1
    cat = lambda name: np.concatenate([getattr(g, name) for g in geoms])
    return Geometry(sx=cat("sx"), sy=cat("sy"), w=cat("w"), nx=cat("nx"),
                    ny=cat("ny"), h=cat("h"), cx=cat("cx"), cy=cat("cy"),
                    cr=cat("cr"), panel=np.concatenate(panels), q=geoms[0].q,
                    meta=dict(kind="multi", parts=[g.meta for g in geoms]))


def batched_geometries(n: int = 256, workload_id: int = 3, nodes=(512, 16384),
                       omega=(5.0, 150.0)):
    """Independent curves of uneven size for batched evaluation: even
    indices stars (3-9 lobes, amplitude 0.3), odd indices ellipses (aspect
    ratio uniform in [1, 10]); node counts log-uniform in `nodes`, rounded
    to whole 16-node panels; omega uniform in `omega`.  Each curve is scaled
    by min(1, 5 / (omega h_1)), h_1 its longest panel at unit scale, so that
    omega h <= 5 holds on every panel (Condition 4 of Sec. 5).  Returns a
    list of (Geometry, omega)."""
    rng = rng_for(workload_id, 0)
    out = []
    for i in range(n):
        nn = float(np.exp(rng.uniform(np.log(nodes[0]), np.log(nodes[1]))))
        npan = max(2, int(round(nn / 16)))
        w = float(rng.uniform(*omega))
        if i % 2 == 0:
            lobes = int(rng.integers(3, 10))
            make = lambda sc: star(npan, 16, lobes=lobes, amp=0.3, radius=sc)
        else:
            ar = float(rng.uniform(1.0, 10.0))
            make = lambda sc: ellipse(npan, 16, a=sc, b=sc / ar)
        h1 = float(np.max(make(1.0).h))
        out.append((make(min(1.0, 5.0 / (w * h1))), w))
    return out


def _shape(kind, rad, par, rot, center):
    """Position, first and second theta-derivatives of a star (par = lobes,
    amplitude 0.3, r = rad (1 + 0.3 cos(par t))) or an ellipse (par = aspect
    ratio, semi-axes rad and rad / par), rotated and moved to center."""
    c0, s0 = np.cos(rot), np.sin(rot)

    def place(x, y, shift):
        return (shift * center[0] + c0 * x - s0 * y, shift * center[1] + s0 * x + c0 * y)

    if kind == "star":
        k, a = par, 0.3

        def f(t, d):
            r = rad * (1 + a * np.cos(k * t))
            r1 = -rad * a * k * np.sin(k * t)
            r2 = -rad * a * k * k * np.cos(k * t)
            c, sn = np.cos(t), np.sin(t)
            if d == 0:
                return place(r * c, r * sn, 1.0)
            if d == 1:
                return place(r1 * c - r * sn, r1 * sn + r * c, 0.0)
            return place(r2 * c - 2 * r1 * sn - r * c, r2 * sn + 2 * r1 * c - r * sn, 0.0)
    else:
        A, B = rad, rad / par

        def f(t, d):
            c, sn = np.cos(t), np.sin(t)
            if d == 0:
                return place(A * c, B * sn, 1.0)
            if d == 1:
                return place(-A * sn, B * c, 0.0)
            return place(-A * c, -B * sn, 0.0)
    return f


def _adaptive_edges(f, omega, c_curv, q=16, start=8):
    """Theta panels of one closed curve, bisected until every panel has
    omega h <= 5 and h kappa_max <= c_curv (h its arclength, kappa_max the
    largest curvature at its nodes and ends), then until neighbouring panels
    differ in length by at most a factor 2."""
    x, wq = _gl(q)
    xs = np.concatenate([[-1.0], x, [1.0]])

    def measure(e):
        a, b = e[:-1, None], e[1:, None]
        half = 0.5 * (b - a)
        t = 0.5 * (a + b) + half * xs[None, :]
        dx, dy = f(t, 1)
        ddx, ddy = f(t, 2)
        sp = np.hypot(dx, dy)
        h = (half[:, 0] * (wq[None, :] * sp[:, 1:-1]).sum(axis=1))
        kap = np.abs(dx * ddy - dy * ddx) / sp ** 3
        return h, kap.max(axis=1)

    e = np.linspace(0.0, 2.0 * np.pi, start + 1)
    while True:
        h, km = measure(e)
        split = (omega * h > 5.0) | (h * km > c_curv)
        if not split.any():
            break
        mid = 0.5 * (e[:-1] + e[1:])[split]
        e = np.sort(np.concatenate([e, mid]))
    while True:
        h, _ = measure(e)
        hn = np.roll(h, -1)
        hp = np.roll(h, 1)
        split = (h > 2.0 * hn) | (h > 2.0 * hp)
        if not split.any():
            break
        mid = 0.5 * (e[:-1] + e[1:])[split]
        e = np.sort(np.concatenate([e, mid]))
    return e


def multiscale_curves(n_curves: int = 64, omega: float = 100.0, workload_id: int = 2,
                      nodes=(570_000, 630_000), box: float = 10.0, gap: float = 0.5, q: int = 16,
                      q_fine: int = 0):
    """Many disjoint curves of different sizes and curvatures in
    [-box, box]^2, as one discretisation: half ellipses (aspect ratio uniform
    in [1, 10]), half stars (3-9 lobes, amplitude 0.3), circumradius uniform
    in [0.5, 1.5], random rotation, placed largest first by rejection so that
    each curve stays at least `gap` from the others (distance between 128
    sample points per curve).  Panels are adaptive in theta (_adaptive_edges);
    the curvature bound c is bisected until the total node count lies in
    `nodes`.  Returns (Geometry, c); with q_fine > 0, (Geometry, c, fine)
    where fine has q_fine Gauss nodes on each of the same panels."""
    rng = rng_for(workload_id, 0)
    draws = []
    for i in range(n_curves):
        R = float(rng.uniform(0.5, 1.5))
        if i % 2 == 0:
            draws.append(("star", R / 1.3, int(rng.integers(3, 10)), R))
        else:
            draws.append(("ellipse", R, float(rng.uniform(1.0, 10.0)), R))
    # largest first: later, smaller curves fill the gaps
    draws.sort(key=lambda d: -d[3])
    t = np.linspace(0.0, 2.0 * np.pi, 128, endpoint=False)
    specs, placed = [], []          # placed: (centre, circumradius, sample points)
    for i, (kind, rad, par, R) in enumerate(draws):
        for _ in range(200000):
            rot = float(rng.uniform(0.0, 2.0 * np.pi))
            cen = rng.uniform(-box + R, box - R, size=2)
            close = [q for c2, R2, q in placed if np.hypot(*(cen - c2)) < R + R2 + gap]
            if not close:
                break
            px, py = _shape(kind, rad, par, rot, cen)(t, 0)
            pts = np.stack([px, py], axis=1)
            near = np.concatenate(close)
            if ((pts[:, None, :] - near[None, :, :]) ** 2).sum(axis=2).min() >= gap * gap:
                break
        else:
            raise RuntimeError("multiscale_curves: could not place curve %d" % i)
        px, py = _shape(kind, rad, par, rot, cen)(t, 0)
        placed.append((cen, R, np.stack([px, py], axis=1)))
        specs.append((kind, rad, par, rot, (float(cen[0]), float(cen[1]))))

    def build(c_curv, qq=q):
        parts = []
        for kind, rad, par, rot, cen in specs:
            f = _shape(kind, rad, par, rot, cen)
            e = _adaptive_edges(f, omega, c_curv, q)
            out = _panelize(e, qq, lambda th: f(th, 0), lambda th: f(th, 1))
            parts.append(_finish(*out, qq, dict(kind=kind, rad=rad, par=par, n_panels=e.size - 1)))
        return concat(parts)

    lo, hi = 1e-3, 10.0          # curvature bounds giving too many / too few nodes
    for _ in range(60):
        c = float(np.sqrt(lo * hi))
        g = build(c)
        if g.n > nodes[1]:
            lo = c
        elif g.n < nodes[0]:
            hi = c
        else:
            return (g, c, build(c, q_fine)) if q_fine else (g, c)
    raise RuntimeError("multiscale_curves: node target not reached")


def annulus_targets(rng: np.random.Generator, n: int, r_in: float, r_out: float):
    """Area-uniform points in r_in < |x| < r_out."""
    rho = np.sqrt(rng.uniform(r_in ** 2, r_out ** 2, size=n))
    th = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return rho * np.cos(th), rho * np.sin(th)


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """iid N(0,1) real and imaginary parts."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# The named workloads.
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    geom: Geometry
    omega: float
    p: int
    eps: float
    tx: np.ndarray
    ty: np.ndarray
    tgt_ctr: np.ndarray      # explicit centre per target, -1 = let the library decide
    sigma_s: np.ndarray      # [n_dens][n] complex128
    sigma_d: np.ndarray
    leaf_max: int = 32
    direct: bool = False
    meta: dict = field(default_factory=dict)
    p_add: int = -1          # FMM order increment; -1 = the library's default rule

    @property
    def n_dens(self) -> int:
        return int(self.sigma_s.shape[0])


def direct_star512(n_dens: int = 1, n_annulus: int = 1024) -> Workload:
    """Direct QBX on the 5-lobe star: 32 panels x 16 nodes, p = 12, omega = 10,
    512 on-surface targets (own centre) + area-uniform annulus targets."""
    wid = 0
    g = star(32, 16, lobes=5, amp=0.3)
    tx_a, ty_a = annulus_targets(rng_for(wid, PURPOSE_TARGETS), n_annulus, 1.4, 2.0)
    tx = np.concatenate([g.sx, tx_a])
    ty = np.concatenate([g.sy, ty_a])
    tgt_ctr = np.concatenate([np.arange(g.n, dtype=np.int32),
                              -np.ones(n_annulus, dtype=np.int32)])
    r = rng_for(wid, PURPOSE_DENSITY)
    ss = complex_gaussian(r, (n_dens, g.n))
    sd = complex_gaussian(r, (n_dens, g.n))
    return Workload("direct_star5_512", g, 10.0, 12, 1e-10, tx, ty, tgt_ctr, ss, sd,
                    direct=True)


# The order increment of the 32768-node star at eps = 1e-10, p = 14,
# calibrated as the paper does (Sec. 7.1): the smallest p_add for which the
# FMM stays within eps of direct QBX, checked over all 32768 targets for a
# Gaussian and a plane-wave density (`calibrate_padd sweep`): relative l2
# 1.6e-11, largest error 5.3e-10 of the largest value (within 10 eps).  One
# more order takes the finest levels' n = 2 P + 1 past 128, a ninth MFMA row
# block, for 6% more time.  The library's default rule adds a margin of 4
# (43) for geometries it has not seen.
STAR32K_P_ADD = 39


def fmm_star(n_panels: int = 2048, n_dens: int = 1, omega: float = 50.0,
             eps: float = 1e-10, p: int = 14, lobes: int = 7, leaf_max: int = 32,
             workload_id: int = 1, p_add: int = -1) -> Workload:
    """QBX-FMM on the 7-lobe star with on-surface targets (own centres).
    Defaults: 2048 panels x 16 nodes = 32768 sources = centres = targets."""
    g = star(n_panels, 16, lobes=lobes, amp=0.3)
    r = rng_for(workload_id, PURPOSE_DENSITY)
    ss = complex_gaussian(r, (n_dens, g.n))
    sd = complex_gaussian(r, (n_dens, g.n))
    return Workload(f"fmm_star{lobes}_{g.n}", g, omega, p, eps, g.sx.copy(), g.sy.copy(),
                    np.arange(g.n, dtype=np.int32), ss, sd, leaf_max=leaf_max, p_add=p_add)
