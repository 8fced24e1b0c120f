"""Adaptive quadtree and FMM interaction lists, built from their definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sec. 4 and Sec. 7.2 ("Complete statement of the fast algorithm"):
* the root b0 is the smallest square centred at the origin holding every
  particle (here sources and QBX centres), enlarged by a relative 1e-12 so
  that no particle sits on its outer edge;
* Stage 1: a box is split into four quadrants while it holds more than
  n_max particles (sources + centres); empty children are dropped;
* colleagues: same-level boxes adjacent to b, b included;
* U(b), b a leaf: all leaves adjacent to b (b included);
* V(b): children of the colleagues of b's parent that are well separated
  from b (for same-level boxes: not adjacent);
* W(b), b a leaf: descendants of b's colleagues whose parent is adjacent to
  b but which are not adjacent to b themselves;
* X(b): all b' with b in W(b').

A particle with coordinate x lies in the level-l box of integer index
floor(u 2^l), u = (x + R0) / (2 R0) evaluated once in double precision.
Two boxes are adjacent when their closed squares intersect and neither
contains the other.  Everything here is brute force over all boxes.

Level restriction (the 2:1 balance the paper's experiments use, Sec. 8 with
its remark on level-restricted trees): the leaves that touch one another
differ by at most one level.  With ``level_restrict`` the adaptive tree is
refined until that holds: while some leaf b touches a box two or more levels
finer than b, b is split into its non-empty quadrants.
"""
from __future__ import annotations

import numpy as np

MAX_LEVEL = 30


def root_radius(*coords) -> float:
    m = 0.0
    for c in coords:
        if c.size:
            m = max(m, float(np.max(np.abs(c))))
    if m == 0.0:
        m = 1.0
    return m * (1.0 + 1e-12)


def build(sx, sy, cx, cy, n_max, level_restrict=False):
    """Returns dict(R0, level, ix, iy, parent, leaf, nsrc, nctr, src, ctr) with
    boxes ordered by (level, Morton order of (ix, iy)); src / ctr hold the
    source and centre indices inside each box."""
    sx, sy, cx, cy = (np.asarray(a, dtype=np.float64) for a in (sx, sy, cx, cy))
    R0 = root_radius(sx, sy, cx, cy)
    px = np.concatenate([sx, cx])
    py = np.concatenate([sy, cy])
    ux = (px + R0) / (2.0 * R0)
    uy = (py + R0) / (2.0 * R0)
    boxes = [(0, 0, 0, -1)]            # (level, ix, iy, parent)
    members = [np.arange(px.size)]
    is_src = np.concatenate([np.ones(sx.size, bool), np.zeros(cx.size, bool)])

    def split(b):
        """Appends the non-empty quadrants of box b; returns their indices."""
        lev, ix, iy, par = boxes[b]
        mem = members[b]
        cl = lev + 1
        jx = np.floor(ux[mem] * 2.0 ** cl).astype(np.int64)
        jy = np.floor(uy[mem] * 2.0 ** cl).astype(np.int64)
        keys = sorted(set(zip(jx.tolist(), jy.tolist())), key=lambda k: _morton(k[0], k[1]))
        out = []
        for kx, ky in keys:
            sel = mem[(jx == kx) & (jy == ky)]
            boxes.append((cl, kx, ky, b))
            members.append(sel)
            out.append(len(boxes) - 1)
        return out

    frontier = [0]
    while frontier:
        nxt = []
        for b in frontier:
            if members[b].size > n_max and boxes[b][0] < MAX_LEVEL:
                nxt += split(b)
        frontier = nxt
    if level_restrict:
        while True:
            parents = set(p for (_, _, _, p) in boxes if p >= 0)
            lev = np.array([bb[0] for bb in boxes])
            x0, y0 = np.array([bb[1] for bb in boxes]), np.array([bb[2] for bb in boxes])
            L = int(lev.max())
            s = np.left_shift(1, L - lev)
            bad = []
            for b in range(len(boxes)):
                if b in parents:
                    continue
                fine = lev >= lev[b] + 2
                touch = ((x0 * s <= (x0[b] + 1) * s[b]) & (x0[b] * s[b] <= (x0 + 1) * s) &
                         (y0 * s <= (y0[b] + 1) * s[b]) & (y0[b] * s[b] <= (y0 + 1) * s))
                if np.any(fine & touch):
                    bad.append(b)
            if not bad:
                break
            for b in bad:
                split(b)
    # renumber by (level, Morton)
    order = sorted(range(len(boxes)), key=lambda b: (boxes[b][0], _morton(boxes[b][1], boxes[b][2])))
    newid = {b: i for i, b in enumerate(order)}
    has_child = set(p for (_, _, _, p) in boxes if p >= 0)
    res = dict(R0=R0)
    res["level"] = np.array([boxes[b][0] for b in order], dtype=np.int64)
    res["ix"] = np.array([boxes[b][1] for b in order], dtype=np.int64)
    res["iy"] = np.array([boxes[b][2] for b in order], dtype=np.int64)
    res["parent"] = np.array([newid[boxes[b][3]] if boxes[b][3] >= 0 else -1 for b in order],
                             dtype=np.int64)
    res["leaf"] = np.array([b not in has_child for b in order], dtype=bool)
    res["nsrc"] = np.array([int(is_src[members[b]].sum()) for b in order], dtype=np.int64)
    res["nctr"] = np.array([int((~is_src[members[b]]).sum()) for b in order], dtype=np.int64)
    ns = sx.size
    res["src"] = [np.sort(members[b][is_src[members[b]]]) for b in order]
    res["ctr"] = [np.sort(members[b][~is_src[members[b]]] - ns) for b in order]
    return res


def _morton(ix, iy):
    k = 0
    for bit in range(MAX_LEVEL + 1):
        k |= ((ix >> bit) & 1) << (2 * bit)
        k |= ((iy >> bit) & 1) << (2 * bit + 1)
    return k


def _bounds(t, b, L):
    s = 1 << (L - t["level"][b])
    return t["ix"][b] * s, (t["ix"][b] + 1) * s, t["iy"][b] * s, (t["iy"][b] + 1) * s


def adjacent_matrix(t):
    """A[a, b] = True when boxes a != b touch and neither contains the other."""
    L = int(t["level"].max())
    s = np.left_shift(1, L - t["level"])
    x0, x1 = t["ix"] * s, (t["ix"] + 1) * s
    y0, y1 = t["iy"] * s, (t["iy"] + 1) * s
    touch = ((x0[:, None] <= x1[None, :]) & (x0[None, :] <= x1[:, None]) &
             (y0[:, None] <= y1[None, :]) & (y0[None, :] <= y1[:, None]))
    contains = ((x0[:, None] <= x0[None, :]) & (x1[None, :] <= x1[:, None]) &
                (y0[:, None] <= y0[None, :]) & (y1[None, :] <= y1[:, None]))
    A = touch & ~contains & ~contains.T
    np.fill_diagonal(A, False)
    return A


def lists(t):
    """U, V, W, X as lists of sorted box-index arrays (one per box)."""
    n = t["level"].size
    A = adjacent_matrix(t)
    lev, ix, iy, par, leaf = t["level"], t["ix"], t["iy"], t["parent"], t["leaf"]
    same = lev[:, None] == lev[None, :]
    coll = same & (np.abs(ix[:, None] - ix[None, :]) <= 1) & (np.abs(iy[:, None] - iy[None, :]) <= 1)
    U, V, W = [], [], []
    for b in range(n):
        if leaf[b]:
            u = np.flatnonzero(leaf & A[b])
            U.append(np.sort(np.append(u, b)))
        else:
            U.append(np.zeros(0, np.int64))
        if par[b] >= 0:
            pc = np.flatnonzero(coll[par[b]])
            kids = np.flatnonzero(np.isin(par, pc))
            V.append(np.sort(kids[~A[b, kids] & (kids != b)]))
        else:
            V.append(np.zeros(0, np.int64))
        if leaf[b]:
            deeper = np.flatnonzero(lev > lev[b])
            sh = lev[deeper] - lev[b]
            ax = ix[deeper] >> sh
            ay = iy[deeper] >> sh
            anc_coll = (np.abs(ax - ix[b]) <= 1) & (np.abs(ay - iy[b]) <= 1)
            cand = deeper[anc_coll]
            ok = A[b, par[cand]] & ~A[b, cand]
            W.append(np.sort(cand[ok]))
        else:
            W.append(np.zeros(0, np.int64))
    X = [[] for _ in range(n)]
    for b in range(n):
        for d in W[b]:
            X[d].append(b)
    X = [np.array(sorted(x), dtype=np.int64) for x in X]
    return dict(U=U, V=V, W=W, X=X)
