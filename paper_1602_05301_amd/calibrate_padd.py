"""Calibrate the FMM order increment p_add of FMM-accelerated QBX.

The paper sets P_l = p_FMM(l) + p_add and finds p_add numerically as the
smallest increment for which the FMM-accelerated evaluation keeps the error
of the layer potential below the requested tolerance (Sec. 7.1, its table of
p_add for p = 2, 4, 6, 8).  This script repeats that procedure on the GPU
for the orders and tolerances the library serves: for each (p, eps) it
evaluates S + D with seeded Gaussian densities on star curves in direct mode
(the reference) and in FMM mode, and bisects for the smallest p_add whose
relative l2 error against the direct evaluation is at most eps / 4.

    python -m paper_1602_05301_amd.calibrate_padd [--quick] [--out FILE]

Prints one JSON object per (p, eps) with the p_add found per geometry and
their maximum.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def main(argv=None):
    import torch

    from . import inputs, qbx

    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--ps", default="4,6,8,10,12,14,16,20")
    ap.add_argument("--eps", default="1e-4,1e-6,1e-8,1e-10,1e-12")
    args = ap.parse_args(argv)
    ps = [int(v) for v in args.ps.split(",")]
    epss = [float(v) for v in args.eps.split(",")]
    geoms = [("star7_256_w50", inputs.star(256, 16, lobes=7), 50.0),
             ("star5_128_w10", inputs.star(128, 16, lobes=5), 10.0),
             ("star7_512_w120", inputs.star(512, 16, lobes=7), 120.0)]
    if args.quick:
        geoms = geoms[:1]
    ctx = qbx.Context(0)
    out = open(args.out, "w") if args.out else None
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
                                           qbx.options(p=p, p_add=pa, leaf_max=32))
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
                rec = dict(geom=name, omega=omega, n=g.n, p=p, eps=eps, p_add=pa,
                           err=cache.get(pa), evals=len(cache), t=time.time())
                print(json.dumps(rec), flush=True)
                if out:
                    out.write(json.dumps(rec) + "\n")
                    out.flush()
                if pa is not None:
                    lo_prev = max(0, pa - 4)
    return 0


if __name__ == "__main__":
    sys.exit(main())
