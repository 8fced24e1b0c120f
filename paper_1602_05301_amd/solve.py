"""Exterior Dirichlet (sound-soft scattering) solves with GMRES on the QBX-FMM matvec.

The field outside the curve is represented as u = D[sigma] + i omega S[sigma]
(Sec. 8.3, eq. rep).  Its exterior limit on the curve gives the second-kind
equation (1/2) sigma + D* sigma + i omega S* sigma = f (Sec. 1, eq. extdir;
f = -u_inc for scattering, eq. int_eq).  QBX with exterior centres returns
the exterior limit itself, so one evaluation with sigma_S = i omega sigma,
sigma_D = sigma and the nodes as targets (each bound to its own centre)
applies the whole left-hand side; the geometry, its tree and tables stay
resident across the iterations.

GMRES (Saad and Schultz 1986): restarted, Arnoldi with classical
Gram-Schmidt applied twice, Givens rotations, in complex128.  `gmres` keeps
the Krylov basis on the host (the matvec on the GPU); `gmres_device` keeps
it on the device, where the Gram-Schmidt products, the norms and the
interpolation of the density to the source grid run as the library's
kernels, and only the small Hessenberg problem is solved on the host.

    python -m paper_1602_05301_amd.solve [--curves 35] [--nodes 105000]

solves the scattering of a plane wave by a set of separated curves (a
synthetic stand-in for the paper's 35 inclusions, sources oversampled 4x)
with gmres_device and prints one JSON object: iterations, relative
residual, time per iteration, and time per matvec (interpolation to the
source grid and the GPU evaluation).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs


class _Hessenberg:
    """The small least-squares problem of one GMRES cycle: the Hessenberg
    columns as they come, reduced by Givens rotations, and the rotated
    right-hand side whose last entry is the residual norm."""

    def __init__(self, m: int, beta: float):
        self.H = np.zeros((m + 1, m), dtype=np.complex128)
        self.cs = np.zeros(m)                                # rotation [[c, s], [-conj(s), c]]
        self.sn = np.zeros(m, dtype=np.complex128)
        self.g = np.zeros(m + 1, dtype=np.complex128)
        self.g[0] = beta
        self.k = 0

    def add_column(self, h, hn: float) -> float:
        """Column k = (h[0..k], hn); returns the new residual norm."""
        k, H, cs, sn, g = self.k, self.H, self.cs, self.sn, self.g
        H[:k + 1, k] = h
        H[k + 1, k] = hn
        for i in range(k):                                   # earlier rotations
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -np.conj(sn[i]) * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        a, c = H[k, k], H[k + 1, k]                          # new rotation zeroes H[k+1, k]
        den = np.hypot(abs(a), abs(c))
        if den == 0.0:
            cs[k], sn[k] = 1.0, 0.0
        elif a == 0.0:
            cs[k], sn[k] = 0.0, np.conj(c) / abs(c)
        else:
            cs[k], sn[k] = abs(a) / den, (a / abs(a)) * np.conj(c) / den
        H[k, k] = cs[k] * a + sn[k] * c
        H[k + 1, k] = 0.0
        g[k + 1] = -np.conj(sn[k]) * g[k]
        g[k] = cs[k] * g[k]
        self.k = k + 1
        return float(abs(g[k + 1]))

    def solution(self) -> np.ndarray:
        kk = self.k
        return np.linalg.solve(np.triu(self.H[:kk, :kk]), self.g[:kk])


def gmres(matvec, b, tol: float = 1e-10, restart: int = 100, maxiter: int = 1000, x0=None):
    """Solve A x = b for the operator x -> matvec(x) (complex vectors).

    Stops when the relative residual |b - A x| / |b| reaches tol or after
    maxiter Arnoldi steps.  Within a cycle the residual is the one of the
    Hessenberg least-squares problem; at every restart, and before
    returning, it is recomputed from b - A x.  Returns (x, info) with info =
    {"iterations" (Arnoldi steps), "residual" (relative, recomputed),
    "history" (relative residual after each step), "converged"}."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    info = {"iterations": 0, "residual": 0.0, "history": [], "converged": True}
    if bnorm == 0.0:
        return np.zeros(n, dtype=np.complex128), info
    its = 0
    while True:
        r = b - matvec(x) if (its or x0 is not None) else b.copy()
        beta = np.linalg.norm(r)
        info["residual"] = float(beta / bnorm)
        if beta / bnorm <= tol or its >= maxiter:
            info["converged"] = bool(beta / bnorm <= tol)
            break
        m = min(restart, maxiter - its)
        V = np.zeros((m + 1, n), dtype=np.complex128)
        hs = _Hessenberg(m, beta)
        V[0] = r / beta
        for k in range(m):
            w = matvec(V[k])
            its += 1
            # classical Gram-Schmidt applied twice (as accurate as modified
            # Gram-Schmidt, in matrix-vector products)
            Vk = V[:k + 1]
            h1 = Vk.conj() @ w
            w = w - h1 @ Vk
            h2 = Vk.conj() @ w
            w = w - h2 @ Vk
            hn = np.linalg.norm(w)
            if hn > 0.0:
                V[k + 1] = w / hn
            est = hs.add_column(h1 + h2, hn) / bnorm
            info["history"].append(est)
            if est <= tol or its >= maxiter or hn == 0.0:
                break
        kk = hs.k
        x = x + hs.solution() @ V[:kk]
    info["iterations"] = its
    return x, info


def gmres_device(ctx, apply, b, tol: float = 1e-10, restart: int = 100, maxiter: int = 1000):
    """GMRES as `gmres`, with the Krylov basis on the device: the Arnoldi
    step (classical Gram-Schmidt twice, the norm and the normalisation) and
    the update of the solution run as the library's kernels
    (qbx_krylov_dot, qbx_krylov_update, qbx_krylov_normalize) on the
    context's stream; only the Gram-Schmidt coefficients of each step come
    back to the host, where the small Hessenberg problem is rotated and
    solved.  apply(v, out) writes A v into out (device complex128 vectors of
    b's length); b: device complex128 vector.  Returns (x on the device,
    info as in gmres)."""
    import torch
    n = int(b.numel())
    dev = b.device
    c128 = torch.complex128
    x = torch.zeros(n, dtype=c128, device=dev)
    m_max = max(1, min(restart, maxiter))
    V = torch.empty((m_max + 1, n), dtype=c128, device=dev)
    coef = torch.empty(2 * m_max + 3, dtype=c128, device=dev)   # [h1 | h2 | |w|^2] of a step
    one = torch.ones(1, dtype=c128, device=dev)
    info = {"iterations": 0, "residual": 0.0, "history": [], "converged": True}

    def sqnorm(v, out):
        ctx.krylov_dot(v.view(1, n), 1, v, out)
        return float(out.cpu()[0].real)

    nb = coef[:1]
    bnorm = np.sqrt(sqnorm(b, nb))
    if bnorm == 0.0:
        return x, info
    its = 0
    while True:
        r = V[0]
        if its == 0:
            r.copy_(b)
        else:
            apply(x, r)                                     # r = A x, then b - A x
            t = b.clone()
            ctx.krylov_update(r.view(1, n), 1, one, t)
            r.copy_(t)
        beta = np.sqrt(sqnorm(r, nb))
        info["residual"] = float(beta / bnorm)
        if beta / bnorm <= tol or its >= maxiter:
            info["converged"] = bool(beta / bnorm <= tol)
            break
        m = min(m_max, maxiter - its)
        hs = _Hessenberg(m, beta)
        ctx.krylov_normalize(r, nb, r)
        for k in range(m):
            w = V[k + 1]
            apply(V[k], w)
            its += 1
            Vk = V[:k + 1]
            h1, h2, nr = coef[:k + 1], coef[k + 1:2 * k + 2], coef[2 * k + 2:2 * k + 3]
            ctx.krylov_dot(Vk, k + 1, w, h1)
            ctx.krylov_update(Vk, k + 1, h1, w)
            ctx.krylov_dot(Vk, k + 1, w, h2)
            ctx.krylov_update(Vk, k + 1, h2, w)
            ctx.krylov_dot(w.view(1, n), 1, w, nr)
            ctx.krylov_normalize(w, nr, w)
            hv = coef[:2 * k + 3].cpu().numpy()
            hn = float(np.sqrt(max(hv[2 * k + 2].real, 0.0)))
            est = hs.add_column(hv[:k + 1] + hv[k + 1:2 * k + 2], hn) / bnorm
            info["history"].append(est)
            if est <= tol or its >= maxiter or hn == 0.0:
                break
        kk = hs.k
        y = torch.from_numpy(-hs.solution()).to(dev)        # x -= V (-y)
        ctx.krylov_update(V[:kk], kk, y, x)
    info["iterations"] = its
    return x, info


# Source Gauss nodes per panel by density nodes per panel q (rows) and
# tolerance (columns 1e-3, 1e-6, 1e-9, 1e-12), as the paper tabulates them
# (Table 1, found empirically per kernel).
_TABLE1_EPS = (1e-3, 1e-6, 1e-9, 1e-12)
_TABLE1 = {2: (8, 16, 24, 32), 4: (12, 24, 32, 40), 8: (16, 32, 40, 48), 16: (32, 48, 64, 64)}


def source_nodes(q: int, eps: float) -> int:
    """Source nodes per panel for density nodes q and tolerance eps: the
    tabulated value of the first column whose tolerance is at most eps (the
    tightest column for eps below 1e-12)."""
    if q not in _TABLE1:
        raise ValueError("density nodes per panel must be one of %s" % sorted(_TABLE1))
    for col, e in enumerate(_TABLE1_EPS):
        if e <= eps:
            return _TABLE1[q][col]
    return _TABLE1[q][-1]


def gl_interp(q: int, qs: int) -> np.ndarray:
    """[qs, q] matrix taking values at the q Gauss-Legendre nodes of [-1, 1]
    to the polynomial interpolant's values at the qs Gauss-Legendre nodes
    (Lagrange basis in barycentric form)."""
    x = np.polynomial.legendre.leggauss(q)[0]
    y = np.polynomial.legendre.leggauss(qs)[0]
    wb = np.array([1.0 / np.prod(x[j] - np.delete(x, j)) for j in range(q)])
    d = y[:, None] - x[None, :]
    L = wb[None, :] / d
    return L / L.sum(axis=1, keepdims=True)


class Oversampled:
    """Sources on a fine grid (q_s Gauss nodes per panel) with the centres
    of the coarse grid (q nodes per panel, the density nodes), as the paper's
    oversampled QBX takes them (Sec. 3.2, Table 1).  Both grids have the same
    panels in the same order; the density is carried to the fine nodes by
    interpolation within each panel."""

    def __init__(self, coarse, fine):
        assert fine.n % coarse.n == 0 and fine.n // coarse.n == fine.q // coarse.q
        self.sx, self.sy, self.w, self.nx, self.ny, self.h = fine.sx, fine.sy, fine.w, fine.nx, fine.ny, fine.h
        self.cx, self.cy, self.cr = coarse.cx, coarse.cy, coarse.cr
        self.n_panels = coarse.n // coarse.q
        self.L = gl_interp(coarse.q, fine.q)

    def upsample(self, sigma: np.ndarray) -> np.ndarray:
        return (np.asarray(sigma).reshape(self.n_panels, -1) @ self.L.T).ravel()


class CFIE:
    """The operator sigma -> (1/2) sigma + D* sigma + i omega S* sigma on a
    curve, applied by the GPU QBX-FMM (a resident qbx.Geometry whose targets
    are the nodes, each with its own centre).  With `fine` (the same panels,
    more Gauss nodes each) the sources are oversampled: sigma is
    interpolated to the fine nodes before each evaluation."""

    def __init__(self, ctx, geom, omega: float, eps: float, p: int, fine=None, **opt):
        import torch
        from . import qbx
        self.omega = float(omega)
        self.n = geom.n
        self.src = Oversampled(geom, fine) if fine is not None else None
        disc = self.src if self.src is not None else geom
        tc = np.arange(geom.n, dtype=np.int32)
        self.geo = qbx.Geometry(ctx, disc, omega, eps, geom.sx, geom.sy, tc, qbx.options(p=p, **opt))
        ns = fine.n if fine is not None else geom.n
        self.ss = torch.empty((1, ns), dtype=torch.complex128, device="cuda")
        self.sd = torch.empty_like(self.ss)
        self.u = torch.empty((1, geom.n), dtype=torch.complex128, device="cuda")
        self.matvecs = 0
        self.gpu_s = 0.0

    def __call__(self, x: np.ndarray) -> np.ndarray:
        import torch
        t0 = time.perf_counter()
        xs = self.src.upsample(x) if self.src is not None else np.ascontiguousarray(x)
        self.sd.copy_(torch.from_numpy(xs[None]))
        self.ss.copy_(torch.from_numpy((1j * self.omega * xs)[None]))
        self.geo.eval(self.ss, self.sd, u=self.u)
        out = self.u.cpu().numpy()[0]
        self.gpu_s += time.perf_counter() - t0
        self.matvecs += 1
        return out


class CFIEDevice:
    """The operator of CFIE on device vectors: apply(sigma, out) writes
    (1/2) sigma + D* sigma + i omega S* sigma into out.  With `fine`, sigma
    is carried to the fine nodes by qbx_upsample (the Gauss-Lagrange
    matrix of gl_interp, on the device), which also forms i omega sigma;
    without, the same kernel with a 1 x 1 matrix forms it."""

    def __init__(self, ctx, geom, omega: float, eps: float, p: int, fine=None, **opt):
        import torch
        from . import qbx
        self.ctx, self.omega, self.n = ctx, float(omega), geom.n
        disc = Oversampled(geom, fine) if fine is not None else geom
        tc = np.arange(geom.n, dtype=np.int32)
        self.geo = qbx.Geometry(ctx, disc, omega, eps, geom.sx, geom.sy, tc, qbx.options(p=p, **opt))
        if fine is not None:
            self.q, self.qs = geom.q, fine.q
            L = gl_interp(geom.q, fine.q)
        else:
            self.q = self.qs = 1
            L = np.ones((1, 1))
        self.L = torch.from_numpy(np.ascontiguousarray(L, dtype=np.float64)).cuda()
        ns = fine.n if fine is not None else geom.n
        self.ss = torch.empty((1, ns), dtype=torch.complex128, device="cuda")
        self.sd = torch.empty_like(self.ss)
        self.matvecs = 0

    def __call__(self, x, out):
        self.ctx.upsample(self.L, self.q, self.qs, x, alpha=1j * self.omega, ys=self.ss, yd=self.sd)
        self.geo.eval(self.ss, self.sd, u=out.view(1, self.n))
        self.matvecs += 1


def volume_eval(ctx, disc, omega: float, eps: float, p: int, sigma_s, sigma_d, tx, ty,
                leaf_max: int = 32) -> np.ndarray:
    """u = S[sigma_s] + D[sigma_d] at targets anywhere off the curve, every
    part through the FMM.  Targets inside an expansion disk (the
    association rule of Sec. 6.1) take QBX as in qbx_eval.  The others take
    the smooth rule, computed as order-0 expansions centred at the targets
    themselves: a second geometry whose centres are those targets (p = 0,
    each target bound to its own centre), so P2QBXL, M2QBXL and L2QBXL are
    exactly the point FMM's direct sum over near sources, M2P and L2P
    (Sec. 7, with the targets as tree points).  sigma_s, sigma_d: [n_src]
    arrays on disc's sources, either may be None."""
    import torch
    from . import qbx
    tx = np.ascontiguousarray(tx, dtype=float)
    ty = np.ascontiguousarray(ty, dtype=float)
    ns = np.asarray(disc.sx).size
    for a in (sigma_s, sigma_d):
        if a is not None and np.asarray(a).size != ns:
            raise ValueError("densities must have one value per source")
    assoc = qbx.Plan(disc, omega, eps, tx, ty, None, qbx.options(p=p, leaf_max=leaf_max)).association()
    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)[None]).cuda()
    ss, sd = dev(sigma_s), dev(sigma_d)
    u = np.zeros(tx.size, dtype=np.complex128)
    q = np.flatnonzero(assoc >= 0)
    if q.size:
        geo = qbx.Geometry(ctx, disc, omega, eps, tx[q], ty[q], assoc[q].astype(np.int32),
                           qbx.options(p=p, leaf_max=leaf_max))
        u[q] = geo.eval(ss, sd).cpu().numpy()[0]
    v = np.flatnonzero(assoc < 0)
    if v.size:
        pts = inputs.Points(np.asarray(disc.sx), np.asarray(disc.sy), np.asarray(disc.w), np.asarray(disc.nx),
                            np.asarray(disc.ny), np.asarray(disc.h), tx[v], ty[v],
                            np.full(v.size, 1e-300))
        geo = qbx.Geometry(ctx, pts, omega, eps, tx[v], ty[v], np.arange(v.size, dtype=np.int32),
                           qbx.options(p=0, leaf_max=leaf_max))
        u[v] = geo.eval(ss, sd).cpu().numpy()[0]
    return u


def field(ctx, geom, omega: float, eps: float, p: int, sigma: np.ndarray, tx, ty, fine=None,
          both_sides: bool = False, **opt) -> np.ndarray:
    """u = D[sigma] + i omega S[sigma] at off-curve targets (QBX inside the
    expansion disks, the FMM's order-0 expansions elsewhere: volume_eval);
    `fine` as in CFIE.  both_sides: centres on both sides of the curve
    (inputs.two_sided), so that targets close to the curve on its inner side
    are served too."""
    src = Oversampled(geom, fine) if fine is not None else None
    s = src.upsample(sigma) if src is not None else np.ascontiguousarray(sigma)
    if both_sides:
        disc = inputs.two_sided(geom, fine)
    else:
        disc = src if src is not None else geom
    return volume_eval(ctx, disc, omega, eps, p, 1j * omega * s, s, tx, ty, **opt)


def plane_wave(omega: float, x, y, dx: float = -2.0 / np.sqrt(5.0), dy: float = 1.0 / np.sqrt(5.0)):
    """exp(i omega d.x), by default the incident wave of the paper's scattering run (Sec. 8.3)."""
    return np.exp(1j * omega * (dx * np.asarray(x) + dy * np.asarray(y)))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--curves", type=int, default=35)
    ap.add_argument("--nodes", type=int, default=105_000)
    ap.add_argument("--omega", type=float, default=12.43)
    ap.add_argument("--eps", type=float, default=5e-7)
    ap.add_argument("--p", type=int, default=9)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--restart", type=int, default=2000)
    ap.add_argument("--maxiter", type=int, default=2000)
    ap.add_argument("--oversample", type=int, default=0,
                    help="source nodes per density node (0: from Table 1 for eps; 1: none)")
    args = ap.parse_args(argv)
    from . import qbx
    q = 16
    qs = source_nodes(q, args.eps) if args.oversample == 0 else q * args.oversample
    made = inputs.multiscale_curves(n_curves=args.curves, omega=args.omega,
                                    nodes=(int(0.95 * args.nodes), int(1.05 * args.nodes)),
                                    q=q, q_fine=qs if qs > q else 0)
    g, c = made[0], made[1]
    fine = made[2] if len(made) > 2 else None
    import torch
    ctx = qbx.Context(0)
    t0 = time.perf_counter()
    A = CFIEDevice(ctx, g, args.omega, args.eps, args.p, fine=fine)
    setup = time.perf_counter() - t0
    f = torch.from_numpy(-plane_wave(args.omega, g.sx, g.sy)).cuda()
    out = torch.empty_like(f)
    A(f, out)                                            # warm-up (scratch, kernels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        A(f, out)
    torch.cuda.synchronize()
    matvec = (time.perf_counter() - t0) / 10
    A.matvecs = 0
    t0 = time.perf_counter()
    sigma, info = gmres_device(ctx, A, f, tol=args.tol, restart=args.restart, maxiter=args.maxiter)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    A(sigma, out)
    n = int(f.numel())
    r = f.clone()
    ctx.krylov_update(out.view(1, n), 1, torch.ones(1, dtype=torch.complex128, device="cuda"), r)
    nr = torch.empty(2, dtype=torch.complex128, device="cuda")
    ctx.krylov_dot(r.view(1, n), 1, r, nr[:1])
    ctx.krylov_dot(f.view(1, n), 1, f, nr[1:])
    nrh = nr.cpu().numpy().real
    true_res = float(np.sqrt(nrh[0] / nrh[1]))
    its = max(info["iterations"], 1)
    out = {"workload": f"{args.curves} separated curves (multiscale recipe), {g.n} unknowns, "
                       f"{fine.n if fine is not None else g.n} sources, omega {args.omega}, "
                       f"eps {args.eps}, p {args.p}, plane wave, GMRES({args.restart}) to {args.tol}, "
                       "Krylov basis and Gram-Schmidt on the device",
           "unknowns": g.n, "sources": fine.n if fine is not None else g.n, "curvature_bound": c,
           "setup_s": setup,
           "iterations": info["iterations"], "converged": info["converged"],
           "relative_residual": true_res, "wall_s": wall,
           "ms_per_iteration": 1e3 * wall / its, "matvec_ms": 1e3 * matvec,
           "iteration_over_matvec": wall / its / matvec}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
