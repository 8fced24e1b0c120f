"""Oracle for FMM-accelerated Global QBX (2D Helmholtz S and D potentials).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this package; the product
library and its Python binding never import it.  It shares no code with the
GPU path.

Contents
--------
* ``qbx_oracle.c`` (built into ``libqbxoracle.so`` with gcc): the direct
  O(N_s N_c) QBX coefficient sum, the truncated J-expansion evaluation, the
  smooth Gauss rule and brute-force target association.  See the header of
  that file for the formulas and the passages they follow.
* ``direct_qbx``: the whole direct pipeline (association, coefficients,
  evaluation), i.e. what the FMM-accelerated path must reproduce to the
  requested tolerance.
* ``translations``: the FMM translation operators written out as plain sums
  (P2M, M2M, M2L, L2L, P2L, M2P, L2P and their double-layer source terms).
* ``tree``: the adaptive quadtree and the U, V, W, X interaction lists built
  straight from their definitions (Sec. 7.2, "Complete statement").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qbx_oracle.c")
_LIB = os.path.join(_HERE, "libqbxoracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O3 for any x86-64 with AVX2, OpenMP
    over centres).  The library travels with the repository, so it is built
    for a portable instruction set, not for the machine that builds it."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC,
               "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def use_native_build(workdir: str) -> str:
    """Rebuilds the oracle with -O3 -march=native for the host it runs on,
    in workdir, and makes this process use that copy (for timing it as a
    CPU baseline).  Returns the library path."""
    global _lib
    out = os.path.join(workdir, "libqbxoracle_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC,
           "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    _lib = None
    _load(out)
    return out


def lib():
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _load(_LIB)
    return _lib


def _load(path):
    global _lib
    if _lib is None:
        L = ctypes.CDLL(path)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.oracle_hankel1_seq.argtypes = [dbl, i32, _dp]
        L.oracle_besselj_seq.argtypes = [dbl, i32, _dp]
        L.oracle_qbx_coefficients.argtypes = [dbl, i32, i64, _dp, _dp, _dp, _dp, _dp,
                                              i32, _dp, _dp, i64, _dp, _dp, _dp, i32]
        L.oracle_qbx_eval.argtypes = [dbl, i32, i64, _dp, _dp, i32, _dp, i64, _dp, _dp,
                                      _ip, _dp, i32]
        L.oracle_smooth.argtypes = [dbl, i64, _dp, _dp, _dp, _dp, _dp, i32, _dp, _dp,
                                    i64, _dp, _dp, _ip, _dp, i32]
        L.oracle_associate.argtypes = [i64, _dp, _dp, i64, _dp, _dp, _dp, i64, _dp, _dp,
                                       _dp, dbl, _ip, i32]
        L.oracle_associate.restype = ctypes.c_int64
        _lib = L
    return _lib


def default_threads() -> int:
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _c(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data_as(_dp)


# ---------------------------------------------------------------------------
# Bessel sequences
# ---------------------------------------------------------------------------

def hankel1_seq(x: float, nmax: int) -> np.ndarray:
    """H_n^{(1)}(x), n = 0..nmax (C library J0,J1,Y0,Y1 + upward recurrence)."""
    out = np.empty(nmax + 1, dtype=np.complex128)
    rc = lib().oracle_hankel1_seq(float(x), int(nmax), out.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("hankel1_seq needs x > 0")
    return out


def besselj_seq(x: float, nmax: int) -> np.ndarray:
    """J_n(x), n = 0..nmax (C library jn)."""
    out = np.empty(nmax + 1, dtype=np.float64)
    lib().oracle_besselj_seq(float(x), int(nmax), out.ctypes.data_as(_dp))
    return out


# ---------------------------------------------------------------------------
# Direct QBX pieces
# ---------------------------------------------------------------------------

def qbx_coefficients(omega, p, sx, sy, w, nx, ny, sigma_s, sigma_d, cx, cy,
                     nthreads=None):
    """alpha[d, l+p, i]: QBX local coefficients at every centre from ALL sources."""
    sx, psx = _d(sx); sy, psy = _d(sy); w, pw = _d(w); nx, pnx = _d(nx); ny, pny = _d(ny)
    cx, pcx = _d(cx); cy, pcy = _d(cy)
    ref = sigma_s if sigma_s is not None else sigma_d
    ref = np.atleast_2d(ref)
    nd = ref.shape[0]
    ss, pss = _c(None if sigma_s is None else np.atleast_2d(sigma_s))
    sd, psd = _c(None if sigma_d is None else np.atleast_2d(sigma_d))
    alpha = np.zeros((nd, 2 * p + 1, cx.size), dtype=np.complex128)
    rc = lib().oracle_qbx_coefficients(float(omega), int(p), sx.size, psx, psy, pw, pnx, pny,
                                       nd, pss, psd, cx.size, pcx, pcy,
                                       alpha.ctypes.data_as(_dp),
                                       nthreads or default_threads())
    if rc != 0:
        raise ValueError("a source coincides with a QBX centre")
    return alpha


def qbx_eval(omega, p, cx, cy, alpha, tx, ty, ctr, nthreads=None, out=None):
    cx, pcx = _d(cx); cy, pcy = _d(cy); tx, ptx = _d(tx); ty, pty = _d(ty)
    alpha = np.ascontiguousarray(alpha, dtype=np.complex128)
    nd = alpha.shape[0]
    ctr = np.ascontiguousarray(ctr, dtype=np.int32)
    u = out if out is not None else np.zeros((nd, tx.size), dtype=np.complex128)
    lib().oracle_qbx_eval(float(omega), int(p), cx.size, pcx, pcy, nd,
                          alpha.ctypes.data_as(_dp), tx.size, ptx, pty,
                          ctr.ctypes.data_as(_ip), u.ctypes.data_as(_dp),
                          nthreads or default_threads())
    return u


def smooth(omega, sx, sy, w, nx, ny, sigma_s, sigma_d, tx, ty, ctr=None,
           nthreads=None, out=None):
    sx, psx = _d(sx); sy, psy = _d(sy); w, pw = _d(w); nx, pnx = _d(nx); ny, pny = _d(ny)
    tx, ptx = _d(tx); ty, pty = _d(ty)
    ref = np.atleast_2d(sigma_s if sigma_s is not None else sigma_d)
    nd = ref.shape[0]
    ss, pss = _c(None if sigma_s is None else np.atleast_2d(sigma_s))
    sd, psd = _c(None if sigma_d is None else np.atleast_2d(sigma_d))
    u = out if out is not None else np.zeros((nd, tx.size), dtype=np.complex128)
    if ctr is not None:
        ctr = np.ascontiguousarray(ctr, dtype=np.int32)
    rc = lib().oracle_smooth(float(omega), sx.size, psx, psy, pw, pnx, pny, nd, pss, psd,
                             tx.size, ptx, pty,
                             None if ctr is None else ctr.ctypes.data_as(_ip),
                             u.ctypes.data_as(_dp), nthreads or default_threads())
    if rc != 0:
        raise ValueError("a smooth-rule target coincides with a source")
    return u


def associate(tx, ty, cx, cy, cr, sx, sy, sh, eps_assoc=0.05, nthreads=None):
    """Brute-force target association: centre index, -1 (smooth rule) or -2 (fail)."""
    tx, ptx = _d(tx); ty, pty = _d(ty); cx, pcx = _d(cx); cy, pcy = _d(cy)
    cr, pcr = _d(cr); sx, psx = _d(sx); sy, psy = _d(sy); sh, psh = _d(sh)
    out = np.empty(tx.size, dtype=np.int32)
    lib().oracle_associate(tx.size, ptx, pty, cx.size, pcx, pcy, pcr, sx.size, psx, psy,
                           psh, float(eps_assoc), out.ctypes.data_as(_ip),
                           nthreads or default_threads())
    return out


def direct_qbx(omega, p, geom, tx, ty, sigma_s, sigma_d, tgt_ctr=None, eps_assoc=0.05,
               nthreads=None, return_coef=False):
    """The whole direct Global-QBX evaluation u = S[sigma_s] + D[sigma_d].

    tgt_ctr: explicit centre per target (-1 entries are associated by the
    brute-force rule); None associates every target."""
    tx = np.asarray(tx, dtype=np.float64)
    ty = np.asarray(ty, dtype=np.float64)
    if tgt_ctr is None:
        ctr = associate(tx, ty, geom.cx, geom.cy, geom.cr, geom.sx, geom.sy, geom.h,
                        eps_assoc, nthreads)
    else:
        ctr = np.asarray(tgt_ctr, dtype=np.int32).copy()
        free = ctr < 0
        if free.any():
            ctr[free] = associate(tx[free], ty[free], geom.cx, geom.cy, geom.cr, geom.sx,
                                  geom.sy, geom.h, eps_assoc, nthreads)
    if (ctr == -2).any():
        raise RuntimeError("target association failed for %d targets" % int((ctr == -2).sum()))
    alpha = qbx_coefficients(omega, p, geom.sx, geom.sy, geom.w, geom.nx, geom.ny,
                             sigma_s, sigma_d, geom.cx, geom.cy, nthreads)
    u = qbx_eval(omega, p, geom.cx, geom.cy, alpha, tx, ty, ctr, nthreads)
    if (ctr == -1).any():
        smooth(omega, geom.sx, geom.sy, geom.w, geom.nx, geom.ny, sigma_s, sigma_d, tx, ty,
               ctr, nthreads, out=u)
    if return_coef:
        return u, alpha, ctr
    return u
