"""Calibrate the FMM order increment p_add of FMM-accelerated QBX.

The paper sets P_l = p_FMM(l) + p_add and finds p_add numerically as the
smallest increment for which the FMM-accelerated evaluation keeps the error
of the layer potential below the requested tolerance (Sec. 7.1, its table of
p_add for p = 2, 4, 6, 8).  This script repeats that procedure on the GPU,
with the library's direct mode (coefficients summed over all sources) as
the reference.

    python -m paper_1602_05301_amd.calibrate_padd bisect [--ps ...] [--eps ...]
        small stars (4096, 2048 and 8192 nodes), every (p, eps): the smallest
        p_add with relative l2 error <= eps / 4, by bisection;
    python -m paper_1602_05301_amd.calibrate_padd sweep [--workloads ...]
        workloads of the benchmark's sizes, each at a list of p_add, plain
        and level-restricted trees: relative l2 and max error against the
        direct sum, the orders P_l and the evaluation time.

  sweep workloads:
    star32k     7-lobe star, 2048 panels x 16 = 32768 nodes, omega 50,
                eps 1e-10, p 14, leaves of 32; Gaussian densities and a
                smooth one (a plane wave of frequency omega on the curve)
    multiscale  the 64-curve set (606k nodes), omega 100, eps 1e-8, p 12,
                leaves of 64; the reference on 2048 sampled centres
    batched     8 curves of the 256-curve batched set (spread over its
                sizes), eps 1e-10 / p 14 and eps 1e-6 / p 9
    star4k      7-lobe star, 256 panels, omega 50, eps 1e-10, p 14
    python -m paper_1602_05301_amd.calibrate_padd batched_all
        every curve of the 256-curve batched set at both tolerances.

Prints one JSON object per measurement.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _emit(out, rec):
    line = json.dumps(rec)
    print(line, flush=True)
    if out:
        out.write(line + "\n")
        out.flush()


def bisect(args, out):
    import torch

    from . import inputs, qbx
    ps = [int(v) for v in args.ps.split(",")]
    epss = [float(v) for v in args.eps.split(",")]
    geoms = [("star7_256_w50", inputs.star(256, 16, lobes=7), 50.0),
             ("star5_128_w10", inputs.star(128, 16, lobes=5), 10.0),
             ("star7_512_w120", inputs.star(512, 16, lobes=7), 120.0)]
    ctx = qbx.Context(0)
    for name, g, omega in geoms:
        rng = inputs.rng_for(7, inputs.PURPOSE_DENSITY)
        ss = torch.from_numpy(inputs.complex_gaussian(rng, (1, g.n))).cuda()
        sd = torch.from_numpy(inputs.complex_gaussian(rng, (1, g.n))).cuda()
        tc = np.arange(g.n, dtype=np.int32)
        for p in ps:
            ref_geo = qbx.Geometry(ctx, g, omega, 1e-12, g.sx, g.sy, tc,
                                   qbx.options(p=p, direct=True))
            ref = ref_geo.eval(ss, sd).cpu().numpy()
            del ref_geo
            lo_prev = 0
            for eps in epss:
                cache = {}

                def err(pa):
                    if pa not in cache:
                        geo = qbx.Geometry(ctx, g, omega, eps, g.sx, g.sy, tc,
                                           qbx.options(p=p, p_add=pa, leaf_max=32,
                                                       level_restrict=args.level_restrict))
                        cache[pa] = _rel(geo.eval(ss, sd).cpu().numpy(), ref)
                    return cache[pa]

                lo, hi = lo_prev, max(lo_prev + 8, 16)
                while err(hi) > eps / 4 and hi < 160:
                    lo, hi = hi, hi + 16
                while hi - lo > 1:
                    mid = (lo + hi) // 2
                    if err(mid) <= eps / 4:
                        hi = mid
                    else:
                        lo = mid
                pa = hi if err(hi) <= eps / 4 else None
                if err(lo) <= eps / 4:
                    pa = lo
                _emit(out, dict(geom=name, omega=omega, n=g.n, p=p, eps=eps, p_add=pa,
                                err=cache.get(pa), evals=len(cache),
                                level_restrict=int(args.level_restrict), t=time.time()))
                if pa is not None:
                    lo_prev = max(0, pa - 4)


class _Case:
    """One workload of the sweep: a discretisation, its targets (each bound
    to a centre), densities and the direct reference on a subset of them."""

    def __init__(self, name, g, omega, eps, p, leaf_max, dens, sample=None):
        self.name, self.g, self.omega, self.eps, self.p, self.leaf_max = name, g, omega, eps, p, leaf_max
        self.dens = dens            # list of (label, sigma_s, sigma_d), host [1, n] arrays
        self.sample = sample        # centre (= on-curve target) indices of the reference


def _plane_wave(g, omega):
    return np.exp(1j * omega * (-2.0 * g.sx + 1.0 * g.sy) / np.sqrt(5.0))[None, :]


def _cases(names):
    from . import inputs
    out = []
    if "star32k" in names or "star4k" in names:
        for nm, npan in (("star32k", 2048), ("star4k", 256)):
            if nm not in names:
                continue
            g = inputs.star(npan, 16, lobes=7)
            r = inputs.rng_for(1, inputs.PURPOSE_DENSITY)
            dens = [("gauss", inputs.complex_gaussian(r, (1, g.n)), inputs.complex_gaussian(r, (1, g.n))),
                    ("plane", 1j * 50.0 * _plane_wave(g, 50.0), _plane_wave(g, 50.0))]
            out.append(_Case(nm, g, 50.0, 1e-10, 14, 32, dens))
    if "multiscale" in names:
        g, _c = inputs.multiscale_curves()
        r = inputs.rng_for(2, inputs.PURPOSE_DENSITY)
        dens = [("gauss", inputs.complex_gaussian(r, (1, g.n)), inputs.complex_gaussian(r, (1, g.n))),
                ("plane", 1j * 100.0 * _plane_wave(g, 100.0), _plane_wave(g, 100.0))]
        sample = np.sort(inputs.rng_for(2, inputs.PURPOSE_TARGETS).choice(g.n, 2048, replace=False))
        out.append(_Case("multiscale", g, 100.0, 1e-8, 12, 64, dens, sample))
    if "batched" in names:
        geoms = inputs.batched_geometries()
        order = np.argsort([gg.n for gg, _ in geoms])
        pick = order[np.linspace(0, len(order) - 1, 8).astype(int)]
        for eps, p in ((1e-10, 14), (1e-6, 9)):
            for i in pick:
                g, omega = geoms[int(i)]
                r = inputs.rng_for(3, inputs.PURPOSE_DENSITY)
                dens = [("gauss", inputs.complex_gaussian(r, (1, g.n)), inputs.complex_gaussian(r, (1, g.n)))]
                out.append(_Case(f"batched{int(i)}_eps{eps:g}", g, omega, eps, p, 32, dens))
    return out


def sweep(args, out):
    import torch

    from . import inputs, qbx
    ctx = qbx.Context(0)
    padds = [int(v) for v in args.p_adds.split(",")]
    for case in _cases(args.workloads.split(",")):
        g = case.g
        tc = np.arange(g.n, dtype=np.int32)
        if case.sample is None:
            ref_pts = inputs.Points(g.sx, g.sy, g.w, g.nx, g.ny, g.h, g.cx, g.cy, g.cr)
            sel = tc
        else:
            sel = case.sample
            ref_pts = inputs.Points(g.sx, g.sy, g.w, g.nx, g.ny, g.h, g.cx[sel], g.cy[sel], g.cr[sel])
        t0 = time.perf_counter()
        ref_geo = qbx.Geometry(ctx, ref_pts, case.omega, case.eps, g.sx[sel], g.sy[sel],
                               np.arange(sel.size, dtype=np.int32), qbx.options(p=case.p, direct=True))
        dev = [(lab, torch.from_numpy(np.ascontiguousarray(s)).cuda(),
                torch.from_numpy(np.ascontiguousarray(d)).cuda()) for lab, s, d in case.dens]
        refs = {lab: ref_geo.eval(s, d).cpu().numpy()[0] for lab, s, d in dev}
        del ref_geo
        _emit(out, dict(workload=case.name, n=g.n, omega=case.omega, eps=case.eps, p=case.p,
                        reference="direct", ref_targets=int(sel.size),
                        ref_s=round(time.perf_counter() - t0, 2)))
        for lr in (1, 0):
            for pa in padds:
                t0 = time.perf_counter()
                geo = qbx.Geometry(ctx, g, case.omega, case.eps, g.sx, g.sy, tc,
                                   qbx.options(p=case.p, p_add=pa, leaf_max=case.leaf_max,
                                               level_restrict=bool(lr),
                                               far_fp32=case.eps >= 1e-6))
                setup = time.perf_counter() - t0
                st = geo.stats()
                rec = dict(workload=case.name, n=g.n, omega=case.omega, eps=case.eps, p=case.p,
                           level_restrict=lr, p_add=pa, n_boxes=st["n_boxes"], n_levels=st["n_levels"],
                           setup_s=round(setup, 2))
                u = None
                for lab, s, d in dev:
                    u = geo.eval(s, d, u=u)
                    got = u.cpu().numpy()[0][sel]
                    rec[f"rel_{lab}"] = _rel(got, refs[lab])
                    rec[f"max_{lab}"] = _maxrel(got, refs[lab])
                lab, s, d = dev[0]
                for _ in range(2):
                    geo.eval(s, d, u=u)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    geo.eval(s, d, u=u)
                torch.cuda.synchronize()
                rec["ms"] = round(1e3 * (time.perf_counter() - t0) / 5, 4)
                _emit(out, rec)
                del geo


def batched_all(args, out):
    """Every curve of the 256-curve batched set at eps 1e-10 (p 14, FP64) and
    1e-6 (p 9, FP32 far field), each at a list of p_add: relative l2 and
    largest error against the direct sum over every node, with the curve's
    size, omega and panel lengths."""
    import torch

    from . import inputs, qbx
    ctx = qbx.Context(0)
    curves = inputs.batched_geometries()
    for eps, p, padds in ((1e-10, 14, [int(v) for v in args.p_adds.split(",")]),
                          (1e-6, 9, [int(v) for v in args.p_adds_loose.split(",")])):
        for i, (g, omega) in enumerate(curves):
            tc = np.arange(g.n, dtype=np.int32)
            r = inputs.rng_for(3, inputs.PURPOSE_DENSITY)
            ss = torch.from_numpy(inputs.complex_gaussian(r, (1, g.n))).cuda()
            sd = torch.from_numpy(inputs.complex_gaussian(r, (1, g.n))).cuda()
            ref = qbx.Geometry(ctx, g, omega, eps, g.sx, g.sy, tc,
                               qbx.options(p=p, direct=True)).eval(ss, sd).cpu().numpy()[0]
            rec = dict(index=i, n=g.n, omega=omega, eps=eps, p=p, omega_h_max=float(omega * g.h.max()),
                       omega_h_min=float(omega * g.h.min()))
            for pa in padds:
                geo = qbx.Geometry(ctx, g, omega, eps, g.sx, g.sy, tc,
                                   qbx.options(p=p, p_add=pa, far_fp32=eps >= 1e-6))
                got = geo.eval(ss, sd).cpu().numpy()[0]
                rec[f"rel_{pa}"] = _rel(got, ref)
                rec[f"max_{pa}"] = _maxrel(got, ref)
                del geo
            _emit(out, rec)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["bisect", "sweep", "batched_all"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--ps", default="4,6,8,10,12,14,16,20")
    ap.add_argument("--eps", default="1e-4,1e-6,1e-8,1e-10,1e-12")
    ap.add_argument("--level-restrict", type=int, default=1)
    ap.add_argument("--workloads", default="star32k,star4k,batched,multiscale")
    ap.add_argument("--p-adds", default="12,16,20,24,28,32,36,40")
    ap.add_argument("--p-adds-loose", default="17,21,25,29")
    args = ap.parse_args(argv)
    out = open(args.out, "a") if args.out else None
    if args.mode == "bisect":
        bisect(args, out)
    elif args.mode == "batched_all":
        batched_all(args, out)
    else:
        sweep(args, out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
