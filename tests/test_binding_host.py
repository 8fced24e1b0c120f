"""The Python binding checks every buffer before the library sees a raw
pointer (no GPU): wrong dtype, layout, size or device raise ValueError, and
no library call is made.  Host tensors are refused everywhere except by
eval, whose library call stages host arrays itself."""
import numpy as np
import pytest
import torch

from paper_1602_05301_amd import qbx


class _NoCalls:
    def __getattr__(self, name):
        raise AssertionError(f"library call {name} made with an invalid buffer")


class _Ctx:
    device = 0
    _h = None


def _fake_geometry(ctx, n_src=10, n_ctr=10, n_tgt=7, p=3):
    g = qbx.Geometry.__new__(qbx.Geometry)
    g._h, g.ctx, g.n_src, g.n_ctr, g.n_tgt, g.p = None, ctx, n_src, n_ctr, n_tgt, p
    return g


@pytest.fixture
def no_lib(monkeypatch):
    monkeypatch.setattr(qbx, "lib", lambda: _NoCalls())


def c128(*shape):
    return torch.zeros(shape, dtype=torch.complex128)


@pytest.mark.parametrize("case", ["dtype", "numel", "rows", "noncontig", "none",
                                  "u_numel", "u_dtype", "coef_numel", "too_many"])
def test_eval_rejects_bad_buffers(no_lib, case):
    g = _fake_geometry(_Ctx())
    ss, sd, u, coef = c128(2, 10), c128(2, 10), None, None
    if case == "dtype":
        ss = torch.zeros((2, 10), dtype=torch.complex64)
    elif case == "numel":
        ss = c128(2, 11)
    elif case == "rows":
        sd = c128(3, 10)
    elif case == "noncontig":
        ss = c128(10, 2).t()
    elif case == "none":
        ss = sd = None
    elif case == "u_numel":
        u = c128(2, 8)
    elif case == "u_dtype":
        u = torch.zeros((2, 7), dtype=torch.float64)
    elif case == "coef_numel":
        coef = c128(2, 7, 9)
    elif case == "too_many":
        ss = sd = c128(65, 10)
    with pytest.raises(ValueError):
        g.eval(ss, sd, u=u, coef=coef)


def test_eval_noalloc_rejects_host_tensors(no_lib):
    # every shape right, but host tensors: the static-buffer path takes
    # device memory only
    g = _fake_geometry(_Ctx())
    with pytest.raises(ValueError):
        g.eval_noalloc(c128(2, 10), c128(2, 10), c128(2, 7))


@pytest.mark.parametrize("case", ["count", "foreign", "rows", "u_numel", "dtype", "cpu"])
def test_eval_batch_rejects_bad_buffers(no_lib, case):
    ctx = qbx.Context.__new__(qbx.Context)
    ctx._h, ctx.device = None, 0
    g1, g2 = _fake_geometry(ctx, 10, 10, 7), _fake_geometry(ctx, 5, 5, 4)
    geoms, ss, sd, us = [g1, g2], [c128(1, 10), c128(2, 5)], [None, c128(2, 5)], [c128(1, 7), c128(2, 4)]
    if case == "count":
        us = us[:1]
    elif case == "foreign":
        geoms[1] = _fake_geometry(_Ctx(), 5, 5, 4)
    elif case == "rows":
        sd[1] = c128(1, 5)
    elif case == "u_numel":
        us[0] = c128(1, 8)
    elif case == "dtype":
        ss[1] = torch.zeros((2, 5), dtype=torch.complex64)
    with pytest.raises(ValueError):
        ctx.eval_batch(geoms, ss, sd, us)
