"""qbx_eval_noalloc (evaluation from the static per-device buffers, no
allocation) against qbx_eval, through the C ABI: two calls in a row, the
second on a smaller input, each bitwise equal to qbx_eval's result; device
memory unchanged by the call; a geometry too large for the static buffers
is rejected before anything runs."""
import numpy as np
import pytest
import torch

from paper_1602_05301_amd import inputs, qbx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return qbx.Context(0)


def _dens(n, nd, seed):
    r = np.random.default_rng(seed)
    s = torch.from_numpy(inputs.complex_gaussian(r, (nd, n))).cuda()
    d = torch.from_numpy(inputs.complex_gaussian(r, (nd, n))).cuda()
    return s, d


def test_noalloc_matches_eval_twice_then_smaller(ctx):
    # a small FMM geometry with off-curve targets (QBX and the order-0
    # geometry of the smooth-rule targets): warms the kernels up
    gs = inputs.star(64, 16, lobes=5)
    rng = np.random.default_rng(3)
    tx_a, ty_a = inputs.annulus_targets(rng, 300, 1.4, 2.0)
    tx = np.concatenate([gs.sx, tx_a])
    ty = np.concatenate([gs.sy, ty_a])
    tc = np.concatenate([np.arange(gs.n, dtype=np.int32), -np.ones(tx_a.size, dtype=np.int32)])
    small = qbx.Geometry(ctx, gs, 15.0, 1e-10, tx, ty, tc, qbx.options(p=12))
    ss_s, sd_s = _dens(gs.n, 1, 5)
    u_warm = torch.empty((1, tx.size), dtype=torch.complex128, device="cuda")
    small.eval_noalloc(ss_s, sd_s, u_warm)
    torch.cuda.synchronize()

    # first call: the 32768-node star, 2 densities (one chunk of 2 or two of 1)
    wl = inputs.fmm_star(n_dens=2)
    g = wl.geom
    big = qbx.Geometry(ctx, g, wl.omega, wl.eps, wl.tx, wl.ty, wl.tgt_ctr, qbx.options(p=wl.p))
    ss, sd = torch.from_numpy(wl.sigma_s).cuda(), torch.from_numpy(wl.sigma_d).cuda()
    u_na = torch.full((2, g.n), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    big.eval_noalloc(ss, sd, u_na)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(0)[0]
    print(f"device free bytes before / after qbx_eval_noalloc: {free0} / {free1}", flush=True)
    assert free1 == free0
    u_ref = big.eval(ss, sd)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(0)[0] < free1       # qbx_eval allocates the geometry's scratch
    assert torch.equal(u_na, u_ref)

    # second call, smaller input: the small geometry, one density, coefficients too
    u2 = torch.full((1, tx.size), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    c2 = torch.full((1, 25, gs.n), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    small.eval_noalloc(ss_s, sd_s, u2, coef=c2)
    u2_ref, c2_ref = small.eval(ss_s, sd_s, coef=True)
    torch.cuda.synchronize()
    assert torch.equal(u2, u2_ref)
    assert torch.equal(c2, c2_ref)
    assert torch.equal(u_warm, u2_ref)


def test_noalloc_direct_mode(ctx):
    wl = inputs.direct_star512(n_dens=3)
    g = wl.geom
    geo = qbx.Geometry(ctx, g, wl.omega, wl.eps, wl.tx, wl.ty, wl.tgt_ctr, qbx.options(p=wl.p, direct=True))
    ss, sd = torch.from_numpy(wl.sigma_s).cuda(), torch.from_numpy(wl.sigma_d).cuda()
    u = torch.empty((3, wl.tx.size), dtype=torch.complex128, device="cuda")
    geo.eval_noalloc(ss, sd, u)
    ref = geo.eval(ss, sd)
    torch.cuda.synchronize()
    assert torch.equal(u, ref)


def test_noalloc_rejects_oversized_geometry(ctx):
    g = inputs.star(8192, 16, lobes=7)         # 131072 nodes: buffers beyond the static array
    geo = qbx.Geometry(ctx, g, 50.0, 1e-10, g.sx, g.sy, np.arange(g.n, dtype=np.int32), qbx.options(p=14))
    s = torch.zeros((1, g.n), dtype=torch.complex128, device="cuda")
    u = torch.zeros((1, g.n), dtype=torch.complex128, device="cuda")
    with pytest.raises(qbx.QbxError) as ei:
        geo.eval_noalloc(s, None, u)
    assert ei.value.status == qbx.QBX_E_UNSUPPORTED
    assert "static array" in str(ei.value)
