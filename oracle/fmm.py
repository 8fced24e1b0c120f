"""FMM-accelerated Global QBX written out stage by stage, in plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the algorithm "FMM-accelerated QBX" of Sec. 7.2 in the paper's
order, with unscaled expansions and the translation operators of
``oracle.translations`` applied box by box:

  Stage 1  tree (``oracle.tree.build``) and U, V, W, X lists;
  Stage 2  P2M at leaves, M2M upward;
  Stage 3  new: P2QBXL, coefficients at each centre from the sources of U(b);
  Stage 4  M2L over V lists;
  Stage 5  new: M2QBXL, the multipoles of W(b) converted at each centre;
  Stage 6  X-list P2L;
  Stage 7  L2L downward;
  Stage 8  new: L2QBXL, psi_b translated to each centre of b, and the sum of
           the three partial coefficient sets.
Orders: P_l = p_FMM(l) + p_add with p_FMM(l) the smallest P such that
|H_n(3 w R_l) J_n(sqrt(2) w R_l)| <= eps for all n > P (Sec. 7.1), evaluated
here with mpmath.  Multipoles live only on levels >= 2 (no V list exists
above), so Stages 2-7 start at level 2.
Only for small inputs: every translation is a Python-level sum.
"""
from __future__ import annotations

import numpy as np

from . import qbx_eval
from . import translations as T
from .tree import build as build_tree
from .tree import lists as build_lists


def fmm_order(omega, R, eps, nmax_extra=80):
    import mpmath
    x, y = 3 * omega * R, np.sqrt(2) * omega * R
    N = int(x) + nmax_extra
    last = 0
    for n in range(N + 1):
        v = abs(mpmath.hankel1(n, x)) * abs(mpmath.besselj(n, y))
        if v > eps:
            last = n
    return max(last, 1)


def orders(omega, R0, nlev, eps, p_add):
    return [fmm_order(omega, R0 / 2 ** l, eps) + p_add for l in range(nlev)]


def box_centre(t, b):
    side = 2.0 * t["R0"] / 2 ** t["level"][b]
    return complex(-t["R0"] + (t["ix"][b] + 0.5) * side, -t["R0"] + (t["iy"][b] + 0.5) * side)


def qbx_fmm_coefficients(omega, p, P_levels, geom, sigma_s, sigma_d, n_max, level_restrict=False):
    """alpha[d, l+p, i] at every centre, one density at a time."""
    t = build_tree(geom.sx, geom.sy, geom.cx, geom.cy, n_max, level_restrict=level_restrict)
    L = build_lists(t)
    nb = t["level"].size
    lev, par, leaf = t["level"], t["parent"], t["leaf"]
    s = geom.sx + 1j * geom.sy
    c = geom.cx + 1j * geom.cy
    nu = geom.nx + 1j * geom.ny
    m = np.array([box_centre(t, b) for b in range(nb)])
    P = lambda b: P_levels[lev[b]]
    sig_s = np.atleast_2d(sigma_s) if sigma_s is not None else None
    sig_d = np.atleast_2d(sigma_d) if sigma_d is not None else None
    nd = (sig_s if sig_s is not None else sig_d).shape[0]
    alpha = np.zeros((nd, 2 * p + 1, c.size), dtype=np.complex128)
    for d in range(nd):
        qs = 0.25j * geom.w * (sig_s[d] if sig_s is not None else 0.0)
        qd = 0.25j * geom.w * (sig_d[d] if sig_d is not None else 0.0)
        qs = np.broadcast_to(qs, s.shape)
        qd = np.broadcast_to(qd, s.shape)
        # Stage 2
        a = [None] * nb
        for b in sorted(range(nb), key=lambda b: -lev[b]):
            if lev[b] < 2:
                continue
            if leaf[b]:
                j = t["src"][b]
                a[b] = T.p2m(omega, m[b], s[j], qs[j], qd[j], nu[j], P(b)) if j.size else \
                    np.zeros(2 * P(b) + 1, np.complex128)
            else:
                kids = np.flatnonzero(par == b)
                a[b] = sum(T.m2m(omega, a[k], m[k], m[b], P(b)) for k in kids)
        # Stages 4 and 6
        psi = [None] * nb
        for b in range(nb):
            if lev[b] < 2:
                continue
            g = np.zeros(2 * P(b) + 1, np.complex128)
            for v in L["V"][b]:
                g = g + T.m2l(omega, a[v], m[v], m[b], P(b))
            for x in L["X"][b]:
                j = t["src"][x]
                if j.size:
                    g = g + T.p2l(omega, m[b], s[j], qs[j], qd[j], nu[j], P(b))
            psi[b] = g
        # Stage 7 (boxes are ordered by level, parents first)
        for b in range(nb):
            if lev[b] >= 3:
                psi[b] = psi[b] + T.l2l(omega, psi[par[b]], m[par[b]], m[b], P(b))
        # Stages 3, 5, 8 (new)
        for b in range(nb):
            if not leaf[b]:
                continue
            usrc = np.concatenate([t["src"][u] for u in L["U"][b]]) if len(L["U"][b]) else np.zeros(0, int)
            for i in t["ctr"][b]:
                acc = np.zeros(2 * p + 1, np.complex128)
                if usrc.size:
                    acc += T.p2l(omega, c[i], s[usrc], qs[usrc], qd[usrc], nu[usrc], p)
                for w in L["W"][b]:
                    acc += T.m2l(omega, a[w], m[w], c[i], p)
                if lev[b] >= 2:
                    acc += T.l2l(omega, psi[b], m[b], c[i], p)
                alpha[d, :, i] = acc
    return alpha, t


def qbx_fmm(omega, p, P_levels, geom, tx, ty, tgt_ctr, sigma_s, sigma_d, n_max, level_restrict=False):
    """Potentials at targets with explicit centres (on-curve or near targets)."""
    alpha, _ = qbx_fmm_coefficients(omega, p, P_levels, geom, sigma_s, sigma_d, n_max,
                                    level_restrict=level_restrict)
    return qbx_eval(omega, p, geom.cx, geom.cy, alpha, tx, ty, np.asarray(tgt_ctr, np.int32)), alpha
