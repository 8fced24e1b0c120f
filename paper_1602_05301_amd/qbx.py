"""Python binding of ``libqbxfmm.so`` (ctypes; argument marshalling only).

Every numerical step runs in the library: the host planner (C++) and the
gfx950 kernels.  PyTorch only provides device memory and the stream.  The
binding fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqbxfmm.so")

QBX_OK, QBX_E_INVAL, QBX_E_NOMEM, QBX_E_DEVICE, QBX_E_ASSOC, QBX_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
LIST_U, LIST_V, LIST_W, LIST_X = 0, 1, 2, 3
_STATUS = {0: "OK", -1: "INVAL", -2: "NOMEM", -3: "DEVICE", -4: "ASSOC", -5: "UNSUPPORTED", -6: "BUSY"}

# Every symbol declared in include/qbxfmm.h.
EXPORTS = [
    "qbx_abi_version", "qbx_last_error", "qbx_options_default",
    "qbx_ctx_create", "qbx_ctx_set_stream", "qbx_ctx_destroy",
    "qbx_plan_create", "qbx_plan_destroy", "qbx_plan_stats", "qbx_plan_boxes",
    "qbx_plan_list", "qbx_plan_orders", "qbx_plan_association",
    "qbx_geom_create", "qbx_geom_from_plan", "qbx_geom_destroy", "qbx_geom_stats",
    "qbx_geom_association", "qbx_geom_bytes", "qbx_geom_profile", "qbx_geom_graph", "qbx_geom_stage_times",
    "qbx_geom_work",
    "qbx_eval_batch", "qbx_geom_autotune",
    "qbx_eval", "qbx_geom_area_query", "qbx_geom_associate", "qbx_geom_points_near",
    "qbx_eval_noalloc", "qbx_plan_bytes",
    "qbx_krylov_dot", "qbx_krylov_update", "qbx_krylov_normalize", "qbx_upsample",
    "qbx_ctx_last_error",
]

STAGES = ["charges", "p2m", "m2m", "m2l", "p2l_x", "l2l", "p2qbxl", "m2qbxl", "l2qbxl",
          "eval", "smooth", "direct", "coef_out"]


class QbxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qbxfmm {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("p_add", ctypes.c_int32), ("leaf_max", ctypes.c_int32),
                ("direct", ctypes.c_int32), ("far_fp32", ctypes.c_int32),
                ("w_direct", ctypes.c_int32), ("level_restrict", ctypes.c_int32),
                ("keep_x_rows", ctypes.c_int32), ("eps_assoc", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("n_ctr", ctypes.c_int64), ("n_tgt", ctypes.c_int64),
                ("n_levels", ctypes.c_int32), ("n_boxes", ctypes.c_int32),
                ("n_leaves", ctypes.c_int32), ("p", ctypes.c_int32), ("p_add", ctypes.c_int32),
                ("n_u_pairs", ctypes.c_int64), ("n_v_pairs", ctypes.c_int64),
                ("n_w_pairs", ctypes.c_int64), ("n_x_pairs", ctypes.c_int64),
                ("n_p2qbxl_pairs", ctypes.c_int64), ("n_m2qbxl_pairs", ctypes.c_int64),
                ("n_x_src_pairs", ctypes.c_int64), ("n_smooth_targets", ctypes.c_int64),
                ("root_radius", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                          "(or python -m paper_1602_05301_amd.build) first")
    # Load PyTorch's HIP runtime first: the library's libamdhip64.so.7
    # dependency then binds to that already-loaded copy, so the process holds
    # a single HIP runtime shared by torch tensors, streams and our kernels.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.qbx_abi_version.restype = i32
    L.qbx_last_error.restype = ctypes.c_char_p
    L.qbx_ctx_last_error.restype = ctypes.c_char_p
    L.qbx_ctx_last_error.argtypes = [_vp]
    L.qbx_options_default.argtypes = [ctypes.POINTER(Options)]
    L.qbx_ctx_create.argtypes = [i32, _vp, ctypes.POINTER(_vp)]
    L.qbx_ctx_set_stream.argtypes = [_vp, _vp]
    L.qbx_ctx_destroy.argtypes = [_vp]
    geom_args = [dbl, dbl, ctypes.POINTER(Options), i64, _dp, _dp, _dp, _dp, _dp, _dp,
                 i64, _dp, _dp, _dp, i64, _dp, _dp, _ip]
    L.qbx_plan_create.argtypes = geom_args + [ctypes.POINTER(_vp)]
    L.qbx_plan_destroy.argtypes = [_vp]
    L.qbx_plan_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
    L.qbx_plan_boxes.argtypes = [_vp] + [_ip] * 7
    L.qbx_plan_list.argtypes = [_vp, i32, _ip, _ip]
    L.qbx_plan_orders.argtypes = [_vp, _ip]
    L.qbx_plan_association.argtypes = [_vp, _ip]
    L.qbx_geom_create.argtypes = [_vp] + geom_args + [ctypes.POINTER(_vp)]
    L.qbx_geom_from_plan.argtypes = [_vp, _vp, ctypes.POINTER(_vp)]
    L.qbx_geom_destroy.argtypes = [_vp]
    L.qbx_geom_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
    L.qbx_geom_association.argtypes = [_vp, _ip]
    L.qbx_geom_bytes.argtypes = [_vp, i32]
    L.qbx_plan_bytes.argtypes = [_vp, i32]
    L.qbx_krylov_dot.argtypes = [_vp, i64, i32, _vp, i64, _vp, _vp]
    L.qbx_krylov_update.argtypes = [_vp, i64, i32, _vp, i64, _vp, _vp]
    L.qbx_krylov_normalize.argtypes = [_vp, i64, _vp, _vp, _vp]
    L.qbx_upsample.argtypes = [_vp, i64, i32, i32, _vp, dbl, dbl, _vp, _vp, _vp]
    L.qbx_geom_profile.argtypes = [_vp, i32]
    L.qbx_geom_graph.argtypes = [_vp, i32]
    L.qbx_geom_autotune.argtypes = [_vp, i32, ctypes.POINTER(i32)]
    L.qbx_eval_batch.argtypes = [_vp, i32, ctypes.POINTER(_vp), ctypes.POINTER(i32),
                                 ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]
    L.qbx_geom_stage_times.argtypes = [_vp, _dp, ctypes.POINTER(ctypes.c_int64), i32]
    L.qbx_geom_work.argtypes = [_vp, i32, _dp]
    L.qbx_eval.argtypes = [_vp, i32, _vp, _vp, _vp, _vp]
    L.qbx_eval_noalloc.argtypes = [_vp, i32, _vp, _vp, _vp, _vp]
    L.qbx_geom_area_query.argtypes = [_vp, i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(i64)]
    L.qbx_geom_associate.argtypes = [_vp, i64, _vp, _vp, _vp, ctypes.POINTER(i64)]
    L.qbx_geom_points_near.argtypes = [_vp, i32, i64, _vp, _vp, _vp, _vp]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("qbx_abi_version", "qbx_last_error", "qbx_ctx_last_error", "qbx_options_default",
                        "qbx_geom_bytes", "qbx_plan_bytes"):
            f.restype = st
    L.qbx_geom_bytes.restype = ctypes.c_size_t
    L.qbx_plan_bytes.restype = ctypes.c_size_t
    _lib = L
    return L


def _check(status):
    if status != QBX_OK:
        raise QbxError(status, lib().qbx_last_error().decode())


def options(p=12, p_add=-1, leaf_max=32, direct=False, eps_assoc=0.05, w_direct=-1,
            far_fp32=False, level_restrict=True, keep_x_rows=True) -> Options:
    o = Options()
    lib().qbx_options_default(ctypes.byref(o))
    o.p, o.p_add, o.leaf_max, o.direct, o.eps_assoc = int(p), int(p_add), int(leaf_max), int(bool(direct)), float(eps_assoc)
    o.w_direct = int(w_direct)
    o.far_fp32 = int(bool(far_fp32))
    o.level_restrict = int(bool(level_restrict))
    o.keep_x_rows = int(bool(keep_x_rows))
    return o


def _need_c128(t, numel, what, device=None, host_ok=False):
    """Checks a buffer the library reads or writes through a raw pointer:
    complex128, contiguous, numel elements, on the context's CUDA device (or,
    with host_ok, in host memory, which qbx_eval stages itself).  Raises
    ValueError before any library call."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what} must be a torch tensor")
    if t.dtype != torch.complex128:
        raise ValueError(f"{what} must be complex128, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{what} must hold {numel} elements, got {t.numel()}")
    if not t.is_cuda:
        if host_ok and t.device.type == "cpu":
            return
        raise ValueError(f"{what} must be a CUDA tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what} is on cuda:{t.device.index}, the context on cuda:{device}")


def _n_dens(sigma_s, sigma_d, n_src, what):
    """Density count of a (sigma_s, sigma_d) pair; both must agree."""
    if sigma_s is None and sigma_d is None:
        raise ValueError(f"{what}: at least one of sigma_s, sigma_d is needed")
    nds = set()
    for s in (sigma_s, sigma_d):
        if s is not None:
            if s.dim() not in (1, 2) or (s.dim() == 2 and s.shape[1] != n_src) or \
                    (s.dim() == 1 and s.shape[0] != n_src):
                raise ValueError(f"{what}: densities must be [n_dens, {n_src}] or [{n_src}]")
            nds.add(int(s.shape[0]) if s.dim() == 2 else 1)
    if len(nds) != 1:
        raise ValueError(f"{what}: sigma_s and sigma_d must have the same number of densities")
    nd = nds.pop()
    if not 1 <= nd <= 64:
        raise ValueError(f"{what}: 1 to 64 densities per call, got {nd}")
    return nd


def _arr(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _geom_args(geom, tx, ty, tgt_ctr):
    arrs = [_arr(getattr(geom, n)) for n in ("sx", "sy", "w", "nx", "ny", "h", "cx", "cy", "cr")]
    tx, ty = _arr(tx), _arr(ty)
    tc = None if tgt_ctr is None else _arr(tgt_ctr, np.int32)
    keep = arrs + [tx, ty] + ([tc] if tc is not None else [])
    ptr = lambda a: a.ctypes.data_as(_dp)
    ns, nc = arrs[0].size, arrs[6].size
    args = [ns] + [ptr(a) for a in arrs[:6]] + [nc] + [ptr(a) for a in arrs[6:]] + \
           [tx.size, ptr(tx), ptr(ty), None if tc is None else tc.ctypes.data_as(_ip)]
    return args, keep


class Plan:
    """Host-only planning: tree, lists, orders, association."""

    def __init__(self, geom, omega, eps, tx, ty, tgt_ctr=None, opts: Options | None = None):
        opts = opts or options()
        args, self._keep = _geom_args(geom, tx, ty, tgt_ctr)
        h = _vp()
        _check(lib().qbx_plan_create(float(omega), float(eps), ctypes.byref(opts), *args, ctypes.byref(h)))
        self._h = h
        self._lib = lib()

    def __del__(self):
        # the library handle taken at construction: at interpreter exit the
        # module's globals may already be gone
        L = getattr(self, "_lib", None)
        if getattr(self, "_h", None) and L is not None:
            L.qbx_plan_destroy(self._h)
            self._h = None

    def stats(self) -> dict:
        s = Stats()
        _check(lib().qbx_plan_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def boxes(self) -> dict:
        nb = self.stats()["n_boxes"]
        out = {k: np.empty(nb, dtype=np.int32) for k in ("level", "ix", "iy", "parent", "leaf", "nsrc", "nctr")}
        _check(lib().qbx_plan_boxes(self._h, *[out[k].ctypes.data_as(_ip) for k in
                                              ("level", "ix", "iy", "parent", "leaf", "nsrc", "nctr")]))
        return out

    def list(self, which: int):
        nb = self.stats()["n_boxes"]
        start = np.empty(nb + 1, dtype=np.int32)
        _check(lib().qbx_plan_list(self._h, which, start.ctypes.data_as(_ip), None))
        idx = np.empty(max(int(start[-1]), 1), dtype=np.int32)
        _check(lib().qbx_plan_list(self._h, which, start.ctypes.data_as(_ip), idx.ctypes.data_as(_ip)))
        return start, idx[: start[-1]]

    def orders(self) -> np.ndarray:
        P = np.empty(self.stats()["n_levels"], dtype=np.int32)
        _check(lib().qbx_plan_orders(self._h, P.ctypes.data_as(_ip)))
        return P

    def association(self) -> np.ndarray:
        out = np.empty(max(self.stats()["n_tgt"], 1), dtype=np.int32)
        _check(lib().qbx_plan_association(self._h, out.ctypes.data_as(_ip)))
        return out[: self.stats()["n_tgt"]]

    def bytes(self, n_dens: int = 1) -> int:
        """Device memory the geometry made from this plan would hold once
        evaluated (qbx_plan_bytes), computed on the host."""
        return int(lib().qbx_plan_bytes(self._h, int(n_dens)))


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = _vp()
        _check(lib().qbx_ctx_create(int(device), _vp(stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._lib = lib()
        self.device = device
        self.stream = stream

    def __del__(self):
        # the library handle taken at construction: at interpreter exit the
        # module's globals may already be gone
        L = getattr(self, "_lib", None)
        if getattr(self, "_h", None) and L is not None:
            L.qbx_ctx_destroy(self._h)
            self._h = None

    def last_error(self) -> str:
        """Message of the last failed call on this context (qbx_ctx_last_error)."""
        return lib().qbx_ctx_last_error(self._h).decode()

    def set_stream(self, stream):
        """Later work of this context goes to `stream` (a torch CUDA stream)."""
        _check(lib().qbx_ctx_set_stream(self._h, _vp(stream.cuda_stream)))
        self.stream = stream

    # ---- GMRES building blocks (qbx_krylov_*, qbx_upsample) ----
    @staticmethod
    def _basis(V, k, n):
        import torch
        if not isinstance(V, torch.Tensor) or V.dtype != torch.complex128 or not V.is_cuda or V.dim() != 2:
            raise ValueError("V must be a 2-D complex128 CUDA tensor of Krylov vectors (rows)")
        if V.stride(1) != 1 or V.shape[0] < k or V.shape[1] < n:
            raise ValueError("V must hold k rows of n contiguous entries")
        return V.stride(0)

    def krylov_dot(self, V, k, w, h):
        """h[i] = sum_j conj(V[i, j]) w[j] for i < k (qbx_krylov_dot)."""
        n = int(w.numel())
        ld = self._basis(V, k, n)
        _need_c128(w, n, "w", self.device)
        _need_c128(h, int(h.numel()), "h", self.device)
        if h.numel() < k:
            raise ValueError("h needs k entries")
        _check(lib().qbx_krylov_dot(self._h, n, int(k), _vp(V.data_ptr()), ld, _vp(w.data_ptr()),
                                    _vp(h.data_ptr())))

    def krylov_update(self, V, k, h, w):
        """w[j] -= sum_i h[i] V[i, j] for i < k (qbx_krylov_update)."""
        n = int(w.numel())
        ld = self._basis(V, k, n)
        _need_c128(w, n, "w", self.device)
        _need_c128(h, int(h.numel()), "h", self.device)
        if h.numel() < k:
            raise ValueError("h needs k entries")
        _check(lib().qbx_krylov_update(self._h, n, int(k), _vp(V.data_ptr()), ld, _vp(h.data_ptr()),
                                       _vp(w.data_ptr())))

    def krylov_normalize(self, w, nrm2, v):
        """v = w / sqrt(Re nrm2[0]) (qbx_krylov_normalize)."""
        n = int(w.numel())
        _need_c128(w, n, "w", self.device)
        _need_c128(v, n, "v", self.device)
        _need_c128(nrm2, int(nrm2.numel()), "nrm2", self.device)
        _check(lib().qbx_krylov_normalize(self._h, n, _vp(w.data_ptr()), _vp(nrm2.data_ptr()),
                                          _vp(v.data_ptr())))

    def upsample(self, L, q, qs, x, alpha=1.0, ys=None, yd=None):
        """Panel densities from q to qs Gauss nodes (qbx_upsample): yd = L x per
        panel, ys = alpha yd.  L: float64 CUDA tensor [qs, q]."""
        import torch
        n_panels = int(x.numel()) // q
        if L.dtype != torch.float64 or not L.is_cuda or not L.is_contiguous() or tuple(L.shape) != (qs, q):
            raise ValueError("L must be a contiguous float64 CUDA tensor [qs, q]")
        _need_c128(x, n_panels * q, "x", self.device)
        for t, nm in ((ys, "ys"), (yd, "yd")):
            if t is not None:
                _need_c128(t, n_panels * qs, nm, self.device)
        ptr = lambda t: None if t is None else _vp(t.data_ptr())
        a = complex(alpha)
        _check(lib().qbx_upsample(self._h, n_panels, int(q), int(qs), _vp(L.data_ptr()), a.real, a.imag,
                                  _vp(x.data_ptr()), ptr(ys), ptr(yd)))

    def eval_batch(self, geoms, sigmas_s, sigmas_d, us):
        """One evaluation per geometry, every stage one launch over all of them (qbx_eval_batch).
        sigmas_s[i] / sigmas_d[i]: [n_dens_i, n_src_i] complex128 CUDA tensors or
        None; us[i]: [n_dens_i, n_tgt_i] outputs."""
        n = len(geoms)
        if not (len(sigmas_s) == len(sigmas_d) == len(us) == n):
            raise ValueError("eval_batch: one sigma_s, sigma_d and u entry per geometry")
        nds = []
        for i, (g, s, d, u) in enumerate(zip(geoms, sigmas_s, sigmas_d, us)):
            if not isinstance(g, Geometry) or g.ctx is not self:
                raise ValueError(f"eval_batch: geometry {i} does not belong to this context")
            nd = _n_dens(s, d, g.n_src, f"eval_batch[{i}]")
            for t, nm in ((s, "sigma_s"), (d, "sigma_d")):
                if t is not None:
                    _need_c128(t, nd * g.n_src, f"eval_batch[{i}] {nm}", self.device)
            _need_c128(u, nd * g.n_tgt, f"eval_batch[{i}] u", self.device)
            nds.append(nd)
        ptr = lambda t: None if t is None else t.data_ptr()
        G = (_vp * n)(*[g._h for g in geoms])
        ND = (ctypes.c_int32 * n)(*nds)
        S = (_vp * n)(*[ptr(s) for s in sigmas_s])
        D = (_vp * n)(*[ptr(d) for d in sigmas_d])
        U = (_vp * n)(*[u.data_ptr() for u in us])
        _check(lib().qbx_eval_batch(self._h, n, G, ND, S, D, U))
        return us


class Geometry:
    """A device-resident geometry (tree, lists, translation tables)."""

    def __init__(self, ctx: Context, geom, omega, eps, tx, ty, tgt_ctr=None,
                 opts: Options | None = None, plan: "Plan | None" = None):
        """From the arrays (qbx_geom_create), or from a host plan made with
        the same arrays and options (qbx_geom_from_plan)."""
        self.opts = opts or options()
        h = _vp()
        if plan is not None:
            _check(lib().qbx_geom_from_plan(ctx._h, plan._h, ctypes.byref(h)))
        else:
            args, keep = _geom_args(geom, tx, ty, tgt_ctr)
            _check(lib().qbx_geom_create(ctx._h, float(omega), float(eps), ctypes.byref(self.opts),
                                         *args, ctypes.byref(h)))
        self._h = h
        self._lib = lib()
        self.ctx = ctx
        self.n_src = int(np.asarray(geom.sx).size)
        self.n_ctr = int(np.asarray(geom.cx).size)
        self.n_tgt = int(np.asarray(tx).size)
        self.p = int(self.opts.p)

    def __del__(self):
        # the library handle taken at construction: at interpreter exit the
        # module's globals may already be gone
        L = getattr(self, "_lib", None)
        if getattr(self, "_h", None) and L is not None:
            L.qbx_geom_destroy(self._h)
            self._h = None

    def stats(self) -> dict:
        s = Stats()
        _check(lib().qbx_geom_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def bytes(self, n_dens: int = 1) -> int:
        """Device memory held once n_dens densities have been evaluated
        (resident part plus evaluation scratch), qbx_geom_bytes."""
        return int(lib().qbx_geom_bytes(self._h, int(n_dens)))

    def association(self) -> np.ndarray:
        out = np.empty(max(self.n_tgt, 1), dtype=np.int32)
        _check(lib().qbx_geom_association(self._h, out.ctypes.data_as(_ip)))
        return out[: self.n_tgt]

    def profile(self, enable: bool = True):
        _check(lib().qbx_geom_profile(self._h, int(bool(enable))))

    def area_query(self, qx, qy, qr):
        """Leaves (plan box numbering) meeting the squares |x - (qx, qy)|_inf <= qr,
        qbx_geom_area_query.  qx, qy, qr: float64 CUDA tensors of one length.
        Returns (start int64[n + 1], leaves int32[start[n]]) on the device."""
        import torch
        n = int(qx.numel())
        for t in (qx, qy, qr):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
                raise ValueError("queries must be contiguous float64 CUDA tensors of one length")
        start = torch.empty(n + 1, dtype=torch.int64, device=qx.device)
        total = ctypes.c_int64(0)
        ptr = lambda t: _vp(t.data_ptr())
        _check(lib().qbx_geom_area_query(self._h, n, ptr(qx), ptr(qy), ptr(qr), ptr(start), None,
                                         ctypes.byref(total)))
        leaves = torch.empty(max(total.value, 1), dtype=torch.int32, device=qx.device)
        _check(lib().qbx_geom_area_query(self._h, n, ptr(qx), ptr(qy), ptr(qr), ptr(start), ptr(leaves),
                                         None))
        return start, leaves[: total.value]

    def points_near(self, which: str, qx, qy, qr):
        """Per query disk |x - (qx, qy)| <= qr: whether one of the geometry's
        sources (which="sources") or centres (which="centres") lies in it,
        found through area queries on the device, qbx_geom_points_near.
        qx, qy, qr: float64 CUDA tensors.  Returns a bool CUDA tensor."""
        import torch
        w = {"sources": 0, "centres": 1}[which]
        n = int(qx.numel())
        for t in (qx, qy, qr):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
                raise ValueError("queries must be contiguous float64 CUDA tensors of one length")
        hit = torch.empty(max(n, 1), dtype=torch.int32, device=qx.device)
        _check(lib().qbx_geom_points_near(self._h, w, n, _vp(qx.data_ptr()), _vp(qy.data_ptr()),
                                          _vp(qr.data_ptr()), _vp(hit.data_ptr())))
        return hit[:n] != 0

    def associate(self, tx, ty):
        """Centre (user numbering) or -1 per target by the planner's rule,
        computed on the device through area queries, qbx_geom_associate.
        tx, ty: float64 CUDA tensors.  Returns (tgt_ctr int32 tensor, number of
        targets in Gamma_near without an eligible centre)."""
        import torch
        n = int(tx.numel())
        for t in (tx, ty):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
                raise ValueError("targets must be contiguous float64 CUDA tensors of one length")
        out = torch.empty(max(n, 1), dtype=torch.int32, device=tx.device)
        nf = ctypes.c_int64(0)
        _check(lib().qbx_geom_associate(self._h, n, _vp(tx.data_ptr()), _vp(ty.data_ptr()),
                                        _vp(out.data_ptr()), ctypes.byref(nf)))
        return out[:n], int(nf.value)

    def autotune(self, n_dens: int = 1) -> int:
        """Pick the fastest M2L configuration on this geometry; returns the
        waves per tile chosen (0 = direct-load kernel)."""
        c = ctypes.c_int32(-1)
        _check(lib().qbx_geom_autotune(self._h, int(n_dens), ctypes.byref(c)))
        return int(c.value)

    def graph(self, enable: bool = True):
        """Replay evaluations from captured HIP graphs (keyed by the buffers)."""
        _check(lib().qbx_geom_graph(self._h, int(bool(enable))))

    def stage_times(self, reset: bool = True) -> dict:
        ms = np.zeros(len(STAGES))
        n = np.zeros(len(STAGES), dtype=np.int64)
        _check(lib().qbx_geom_stage_times(self._h, ms.ctypes.data_as(_dp),
                                          n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          int(bool(reset))))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}

    def work(self, n_dens: int = 1) -> dict:
        f = np.zeros(len(STAGES))
        _check(lib().qbx_geom_work(self._h, int(n_dens), f.ctypes.data_as(_dp)))
        return {s: float(f[i]) for i, s in enumerate(STAGES)}

    def eval_noalloc(self, sigma_s, sigma_d, u, coef=None):
        """As eval, through qbx_eval_noalloc: the library allocates nothing
        (its evaluation buffers are a static array per device).  u (and coef,
        if given) must be preallocated complex128 CUDA tensors."""
        nd = _n_dens(sigma_s, sigma_d, self.n_src, "eval_noalloc")
        for t, nm in ((sigma_s, "sigma_s"), (sigma_d, "sigma_d")):
            if t is not None:
                _need_c128(t, nd * self.n_src, nm, self.ctx.device)
        _need_c128(u, nd * self.n_tgt, "u", self.ctx.device)
        if coef is not None:
            _need_c128(coef, nd * (2 * self.p + 1) * self.n_ctr, "coef", self.ctx.device)
        ptr = lambda t: None if t is None else _vp(t.data_ptr())
        _check(lib().qbx_eval_noalloc(self._h, nd, ptr(sigma_s), ptr(sigma_d), ptr(u), ptr(coef)))
        return u

    def eval(self, sigma_s, sigma_d, u=None, coef=None):
        """u[d, m] = S[sigma_s[d]](t_m) + D[sigma_d[d]](t_m); complex128
        tensors on the context's device, or CPU tensors (qbx_eval copies
        those through device buffers and returns once u is filled)."""
        import torch
        nd = _n_dens(sigma_s, sigma_d, self.n_src, "eval")
        dev = (sigma_s if sigma_s is not None else sigma_d).device
        for t, nm in ((sigma_s, "sigma_s"), (sigma_d, "sigma_d")):
            if t is not None:
                _need_c128(t, nd * self.n_src, nm, self.ctx.device, host_ok=True)
        if u is None:
            u = torch.empty((nd, self.n_tgt), dtype=torch.complex128, device=dev)
        _need_c128(u, nd * self.n_tgt, "u", self.ctx.device, host_ok=True)
        if coef is True:
            coef = torch.empty((nd, 2 * self.p + 1, self.n_ctr), dtype=torch.complex128, device=dev)
        if coef is not None and coef is not False:
            _need_c128(coef, nd * (2 * self.p + 1) * self.n_ctr, "coef", self.ctx.device, host_ok=True)
        ptr = lambda t: None if t is None else _vp(t.data_ptr())
        _check(lib().qbx_eval(self._h, nd, ptr(sigma_s), ptr(sigma_d), ptr(u),
                              ptr(coef) if coef is not None and coef is not False else None))
        return (u, coef) if coef is not None and coef is not False else u
