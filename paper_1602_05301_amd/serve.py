"""Continuous-batching server for layer-potential matvec streams.

A request is one geometry (curve nodes, weights, normals, QBX centres) with
omega, eps, p and a chain of densities, as in one GMRES solve: density k+1 is
released only when matvec k has completed.  The server

* admits arrived requests while the HBM budget allows, building their
  resident geometry (host planning plus upload) on a small thread pool so
  that setup overlaps the GPU work of requests already admitted;
* in every step, takes the next matvec of every admitted request whose
  previous matvec is done and evaluates them together with one
  ``qbx_eval_batch`` call (each FMM stage one launch over all of them);
* frees a request's geometry when its last matvec completes.

Results are bitwise the same as evaluating each request alone (the batch
entry point guarantees it per geometry).  ``fifo`` is the plain per-request
path it is compared with: one request at a time in arrival order, setup then
its matvecs through ``qbx_eval``.

    python -m paper_1602_05301_amd.serve [--requests 24] [--qps-fracs 0.5,0.8,0.95]

prints one JSON object: the FIFO path and the server at several arrival
rates (fractions of the measured closed-loop saturation rate), with
throughput (targets x matvecs per second) and p50/p99 request latency
(last matvec done minus arrival).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import dataclasses
import json
import sys
import time

import numpy as np

from . import inputs


@dataclasses.dataclass
class Request:
    rid: int
    n_panels: int            # 16-node panels of its star curve
    lobes: int
    scale: float             # curve radius
    omega: float
    eps: float
    p: int
    n_matvec: int            # chained matvecs (densities) of the request
    seed: int                # of its densities
    arrival: float = 0.0     # seconds after the start of the run
    # filled in by the server
    outputs: list = dataclasses.field(default_factory=list)
    done: float = 0.0
    _geom: object = None
    _base: np.ndarray = None

    @property
    def n(self) -> int:
        return 16 * self.n_panels

    @property
    def geom(self) -> inputs.Geometry:
        """The discretised curve (made on first use)."""
        if self._geom is None:
            self._geom = inputs.star(self.n_panels, 16, lobes=self.lobes, radius=self.scale)
        return self._geom

    def density(self, k: int) -> np.ndarray:
        """Density k (sigma_s = sigma_d), complex128 [n]: a seeded Gaussian
        vector of the request turned by a phase of k (made on first use, so
        that long request streams need not hold every density)."""
        if self._base is None:
            self._base = inputs.complex_gaussian(inputs.rng_for(self.seed, 100 + self.rid), (self.n,))
        return self._base * np.exp(0.7j * k)

    def release(self):
        """Drops the host copies of the curve and densities."""
        self._geom = None
        self._base = None


def make_requests(n: int, seed: int = 4, nodes=(1024, 32768), omega=(1.0, 200.0),
                  eps_choices=(1e-6, 1e-10), matvecs=(20, 60)) -> list:
    """Seeded stream of star-curve requests: node counts log-uniform (rounded
    to whole 16-node panels), omega uniform, eps from eps_choices, 20-60
    chained densities each (Request.density).  Each curve is scaled so that
    its longest panel stays within omega h <= 5 (Condition 4)."""
    rng = inputs.rng_for(seed, 0)
    reqs = []
    for i in range(n):
        nn = int(np.exp(rng.uniform(np.log(nodes[0]), np.log(nodes[1]))))
        npan = max(8, nn // 16)
        lobes = int(rng.integers(3, 10))
        w = float(rng.uniform(*omega))
        # the longest panel of the unit star with npan equal-theta panels
        h1 = float(np.max(inputs.star(npan, 16, lobes=lobes).h))
        scale = min(1.0, 5.0 / (w * h1))
        eps = float(eps_choices[int(rng.integers(0, len(eps_choices)))])
        p = 9 if eps >= 1e-6 else 14
        k = int(rng.integers(matvecs[0], matvecs[1] + 1))
        reqs.append(Request(i, npan, lobes, scale, w, eps, p, k, seed))
    return reqs


def _options(req: Request):
    """A request's geometry options.  The X-list rows are rebuilt in every
    matvec rather than kept: with one density per matvec, reading the kept
    rows of many large geometries costs more than forming them (closed-loop
    rate on this stream 26.1 against 23.3 requests/s), and they would add
    about 12% to each request's footprint under the HBM budget."""
    from . import qbx
    return qbx.options(p=req.p, far_fp32=req.eps >= 1e-6, keep_x_rows=False)


def _build(ctx, req: Request, plan=None):
    from . import qbx
    g = req.geom
    tc = np.arange(g.n, dtype=np.int32)
    return qbx.Geometry(ctx, g, req.omega, req.eps, g.sx, g.sy, tc, _options(req), plan=plan)


def _plan(req: Request):
    """Host planning of a request and the device memory its geometry will
    hold (qbx_plan_bytes), before anything is allocated."""
    from . import qbx
    g = req.geom
    pl = qbx.Plan(g, req.omega, req.eps, g.sx, g.sy, np.arange(g.n, dtype=np.int32), _options(req))
    req.density(0)                       # the request's densities, made here off the serving thread
    return pl, float(pl.bytes(1))


def _progress(every, done, total, what):
    if every and (done % every == 0 or done == total):
        print(f"serve: {what} {done}/{total} requests done", file=sys.stderr, flush=True)


def fifo(ctx, reqs, keep_outputs: bool = False, progress: int = 0) -> dict:
    """Plain per-request path: setup, then every matvec with qbx_eval, one
    request after another, each request starting at max(arrival, previous done).
    progress > 0: a line on stderr every that many finished requests."""
    import torch
    t0 = time.perf_counter()
    for i, r in enumerate(sorted(reqs, key=lambda r: r.arrival)):
        _progress(progress, i, len(reqs), "fifo")
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        geo = _build(ctx, r)
        s = torch.empty((1, r.n), dtype=torch.complex128, device="cuda")
        u = torch.empty_like(s)
        r.outputs = []
        for k in range(r.n_matvec):
            s.copy_(torch.from_numpy(r.density(k)[None]))
            geo.eval(s, s, u=u)
            if keep_outputs:
                r.outputs.append(u.cpu().numpy()[0])
        torch.cuda.synchronize()
        r.done = time.perf_counter() - t0
        del geo
        r.release()
    return _summary(reqs, time.perf_counter() - t0)


class _Active:
    """An admitted request: its geometry, two device density buffers (the
    next matvec's density is uploaded into one while a step reads the
    other), their pinned host staging, and the output buffer."""

    def __init__(self, req, geo, nbytes):
        import torch
        self.req, self.geo, self.k, self.bytes = req, geo, 0, nbytes
        n = req.n
        self.s = [torch.empty((1, n), dtype=torch.complex128, device="cuda") for _ in range(2)]
        self.h = [torch.empty((1, n), dtype=torch.complex128, pin_memory=True) for _ in range(2)]
        self.up = [None, None]          # event: upload into s[i] done (h[i] free again)
        self.u = torch.empty((1, n), dtype=torch.complex128, device="cuda")

    def upload(self, k, stream):
        """Density k into s[k % 2] on the upload stream."""
        import torch
        i = k % 2
        if self.up[i] is not None:
            self.up[i].synchronize()    # its previous upload has left h[i]
        self.h[i].numpy()[0] = self.req.density(k)
        with torch.cuda.stream(stream):
            self.s[i].copy_(self.h[i], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.up[i] = ev


def serve(ctx, reqs, hbm_budget: float, max_batch: int = 32, setup_threads: int = 4,
          keep_outputs: bool = False, progress: int = 0) -> dict:
    """Continuous batching (see the module docstring).  Arrived requests are
    planned on the host (tree, lists, orders) and their device footprint is
    taken from the plan (qbx_plan_bytes), so admission never allocates
    beyond the budget.  Admitted requests get their geometry made from the
    plan on the thread pool.  One step (the next matvec of up to max_batch
    admitted requests, one qbx_eval_batch) is in flight at a time, as the
    chained matvecs require; while it runs, the next densities are uploaded
    on a second stream and the host plans and admits, and completion is
    polled through an event instead of synchronising the device."""
    import torch
    comp = torch.cuda.Stream(device=ctx.device)
    upl = torch.cuda.Stream(device=ctx.device)
    ctx.set_stream(comp)
    pending = sorted(reqs, key=lambda r: r.arrival)
    planning: dict = {}                   # future -> request
    planned: list = []                    # (request, plan, bytes), in arrival order
    building: dict = {}                   # future -> (request, bytes)
    active: list = []
    used = 0.0
    pool = cf.ThreadPoolExecutor(max_workers=setup_threads)
    step, step_ev = None, None
    t0 = time.perf_counter()
    finished = 0
    try:
        while finished < len(reqs):
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending.pop(0)
                planning[pool.submit(_plan, r)] = r
            for fut in [f for f in planning if f.done()]:
                r = planning.pop(fut)
                pl, nb = fut.result()
                planned.append((r, pl, nb))
            planned.sort(key=lambda x: x[0].arrival)
            # admission by the planned footprint, in arrival order
            while planned and (used + planned[0][2] <= hbm_budget or not (active or building or step)):
                r, pl, nb = planned.pop(0)
                used += nb
                building[pool.submit(_build, ctx, r, pl)] = (r, nb)
            for fut in [f for f in building if f.done()]:
                r, nb = building.pop(fut)
                a = _Active(r, fut.result(), nb)
                a.upload(0, upl)
                active.append(a)
            if step is not None:
                if not step_ev.query():
                    time.sleep(2e-5)
                    continue
                t = time.perf_counter() - t0
                keep = []
                for a in step:
                    if keep_outputs:
                        a.req.outputs.append(a.u.cpu().numpy()[0])
                    a.k += 1
                    if a.k == a.req.n_matvec:
                        a.req.done = t
                        used -= a.bytes
                        finished += 1
                        a.geo = None             # frees the resident geometry
                        a.req.release()
                        _progress(progress, finished, len(reqs), "served")
                    else:
                        keep.append(a)
                # round robin: the requests just served go behind those that waited
                active = active[len(step):] + keep
                step = None
                continue
            if not active:
                waits = list(planning) + list(building)
                if waits:
                    cf.wait(waits, timeout=0.002, return_when=cf.FIRST_COMPLETED)
                elif pending:
                    time.sleep(max(0.0, min(0.002, pending[0].arrival - (time.perf_counter() - t0))))
                continue
            # issue one step: the next matvec of up to max_batch requests
            step = active[:max_batch]
            for a in step:
                comp.wait_event(a.up[a.k % 2])
            ctx.eval_batch([a.geo for a in step], [a.s[a.k % 2] for a in step],
                           [a.s[a.k % 2] for a in step], [a.u for a in step])
            step_ev = torch.cuda.Event()
            step_ev.record(comp)
            # the next densities go up while the step runs
            for a in step:
                if a.k + 1 < a.req.n_matvec:
                    a.upload(a.k + 1, upl)
    finally:
        pool.shutdown()
        torch.cuda.synchronize()
        ctx.set_stream(torch.cuda.current_stream(ctx.device))
    return _summary(reqs, time.perf_counter() - t0)


def _summary(reqs, wall: float) -> dict:
    lat = np.array([r.done - r.arrival for r in reqs])
    work = sum(r.n * r.n_matvec for r in reqs)
    return {"requests": len(reqs), "matvecs": sum(r.n_matvec for r in reqs),
            "wall_s": wall, "targets_x_matvecs_per_s": work / wall,
            "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}}


def measured(run: dict, reqs, skip: int) -> dict:
    """A run's figures over the requests after the first `skip` (warm-up):
    latency percentiles of those, throughput over the span from the first
    of them arriving to the last finishing."""
    rest = sorted(reqs, key=lambda r: r.arrival)[skip:]
    if not rest:
        return run
    span = max(r.done for r in rest) - min(r.arrival for r in rest)
    lat = np.array([r.done - r.arrival for r in rest])
    work = sum(r.n * r.n_matvec for r in rest)
    return {"requests": len(rest), "warmup_requests": skip, "matvecs": sum(r.n_matvec for r in rest),
            "span_s": span, "targets_x_matvecs_per_s": work / span,
            "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}}


def batch_vs_sequential(ctx, n_geom: int = 16, rounds: int = 10, max_nodes: int = 16384) -> dict:
    """One matvec on each of n_geom resident geometries (uneven sizes, omega,
    eps; 4 densities each): qbx_eval_batch against qbx_eval one after another."""
    import torch
    reqs = make_requests(n_geom, seed=11, nodes=(512, max_nodes), matvecs=(4, 4))
    geos = [_build(ctx, r) for r in reqs]
    s = [torch.from_numpy(np.stack([r.density(k) for k in range(4)])).cuda() for r in reqs]
    u = [torch.empty_like(x) for x in s]
    for g, x, y in zip(geos, s, u):                  # warm-up (scratch, tiles)
        g.eval(x, x, u=y)
    ctx.eval_batch(geos, s, s, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        for g, x, y in zip(geos, s, u):
            g.eval(x, x, u=y)
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) / rounds
    t0 = time.perf_counter()
    for _ in range(rounds):
        ctx.eval_batch(geos, s, s, u)
    torch.cuda.synchronize()
    bat = (time.perf_counter() - t0) / rounds
    work = sum(r.n * 4 for r in reqs)
    return {"geometries": n_geom, "densities_each": 4, "nodes": [r.n for r in reqs],
            "sequential_ms": seq * 1e3, "batched_ms": bat * 1e3,
            "batched_targets_x_densities_per_s": work / bat}


def batched_p_add(p: int, eps: float) -> int:
    """The order increment of the batched workload: 12 above the library's
    default rule, which some of its small high-frequency curves need to stay
    within eps at every target."""
    from . import qbx
    tiny = inputs.star(4, 4, lobes=3)
    return qbx.Plan(tiny, 1.0, eps, tiny.sx, tiny.sy, np.arange(tiny.n, dtype=np.int32),
                    qbx.options(p=p)).stats()["p_add"] + 12


def batched_workload(ctx, n_geom: int = 256, eps: float = 1e-10, n_dens: int = 4, rounds: int = 3,
                     setup_threads: int = 8) -> dict:
    """The batched workload: n_geom independent star and ellipse curves of
    512-16384 nodes (inputs.batched_geometries), n_dens seeded Gaussian
    densities each, all geometries resident.  Times one qbx_eval_batch over
    all of them against qbx_eval on each in turn (the plain per-request
    path), both with inputs already in HBM.  eps >= 1e-6 runs the FP32 far
    field (p = 9), else FP64 throughout (p = 14)."""
    import torch
    from . import qbx
    far32 = eps >= 1e-6
    p = 9 if far32 else 14
    p_add = batched_p_add(p, eps)
    curves = inputs.batched_geometries(n_geom)
    dr = inputs.rng_for(3, inputs.PURPOSE_DENSITY)
    dens = [inputs.complex_gaussian(dr, (n_dens, g.n)) for g, _ in curves]

    def build(item):
        g, w = item
        return qbx.Geometry(ctx, g, w, eps, g.sx, g.sy, np.arange(g.n, dtype=np.int32),
                            qbx.options(p=p, p_add=p_add, far_fp32=far32))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=setup_threads) as pool:
        geos = list(pool.map(build, curves))
    setup = time.perf_counter() - t0
    s = [torch.from_numpy(d).cuda() for d in dens]
    u = [torch.empty_like(x) for x in s]
    ub = [torch.empty_like(x) for x in s]
    for g, x, y in zip(geos, s, u):                  # warm-up: scratch, tiles, kernels
        g.eval(x, x, u=y)
    ctx.eval_batch(geos, s, s, ub)
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(u, ub))
    t0 = time.perf_counter()
    for _ in range(rounds):
        for g, x, y in zip(geos, s, u):
            g.eval(x, x, u=y)
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) / rounds
    t0 = time.perf_counter()
    for _ in range(rounds):
        ctx.eval_batch(geos, s, s, ub)
    torch.cuda.synchronize()
    bat = (time.perf_counter() - t0) / rounds
    work = sum(g.n * n_dens for g, _ in curves)
    nodes = np.array([g.n for g, _ in curves])
    return {"geometries": n_geom, "densities_each": n_dens, "eps": eps, "far_fp32": far32, "p": p, "p_add": p_add,
            "nodes_total": int(nodes.sum()), "nodes_min": int(nodes.min()), "nodes_max": int(nodes.max()),
            "setup_s": setup, "batched_ms": bat * 1e3, "one_by_one_ms": seq * 1e3,
            "batched_targets_x_densities_per_s": work / bat,
            "one_by_one_targets_x_densities_per_s": work / seq,
            "batched_equals_alone": bool(same)}


def _poisson(reqs, qps: float, seed: int = 7):
    rng = np.random.default_rng(seed)
    t = 0.0
    for r in reqs:
        t += rng.exponential(1.0 / qps)
        r.arrival = t


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=24, help="measured requests per arrival rate")
    ap.add_argument("--warmup-requests", type=int, default=0,
                    help="requests served first at each rate and left out of its figures")
    ap.add_argument("--max-nodes", type=int, default=32768)
    ap.add_argument("--qps-fracs", default="0.5,0.8,0.95")
    ap.add_argument("--fifo-frac", type=float, default=0.8)
    ap.add_argument("--hbm-gib", type=float, default=64.0)
    ap.add_argument("--batched", action="store_true",
                    help="only the batched workload (256 geometries, 4 densities, eps 1e-10 and 1e-6)")
    args = ap.parse_args(argv)
    import torch
    from . import qbx
    ctx = qbx.Context(0)
    if args.batched:
        out = {"batched": [batched_workload(ctx, eps=e) for e in (1e-10, 1e-6)]}
        print(json.dumps(out), flush=True)
        return 0
    budget = args.hbm_gib * 2 ** 30
    nw, n = args.warmup_requests, args.requests
    stream = lambda: make_requests(nw + n, nodes=(1024, args.max_nodes))
    # warm-up: library, kernels, one small request each way
    w = make_requests(2, seed=99, nodes=(1024, 2048), matvecs=(2, 2))
    fifo(ctx, w)
    serve(ctx, make_requests(2, seed=99, nodes=(1024, 2048), matvecs=(2, 2)), budget)
    reqs = stream()
    for r in reqs:
        r.arrival = 0.0
    closed = serve(ctx, reqs, budget, progress=100)    # all at once: saturation rate
    sat_qps = (nw + n) / closed["wall_s"]
    print(f"serve: saturation {sat_qps:.2f} requests/s", file=sys.stderr, flush=True)
    out = {"workload": f"{n} measured star requests after {nw} warm-up ones, 1024-{args.max_nodes} nodes "
                       "log-uniform, omega U[1,200], eps in {1e-6 (FP32 far field), 1e-10}, 20-60 chained "
                       "matvecs, Poisson arrivals",
           "saturation_qps": sat_qps, "closed_loop": closed, "served": {}}
    reqs = stream()
    _poisson(reqs, args.fifo_frac * sat_qps)
    out[f"fifo_at_{args.fifo_frac}"] = measured(fifo(ctx, reqs, progress=100), reqs, nw)
    print("serve: fifo done", file=sys.stderr, flush=True)
    for f in [float(x) for x in args.qps_fracs.split(",")]:
        reqs = stream()
        _poisson(reqs, f * sat_qps)
        out["served"][str(f)] = measured(serve(ctx, reqs, budget, progress=100), reqs, nw)
        print(f"serve: {f} x saturation done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
