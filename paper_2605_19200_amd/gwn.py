"""Python binding of the C ABI in ``include/gwn.h`` (argument marshalling only).

Functions keep the C names (``gwn_build2d``, ``gwn_query``, ...).  Device
buffers are torch tensors on a ROCm device; only their data pointers and the
HIP stream handle cross the boundary.  Every step of the query path runs in
the HIP library ``libgwn.so``; if it is missing this module raises at import
time of the library (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgwn.so")

GWN_OK, GWN_EINVAL, GWN_ENOMEM, GWN_EHIP, GWN_EUNSUPPORTED, GWN_EOVERFLOW = range(6)
GWN_FP64, GWN_MIXED = 0, 1
COUNTER_NAMES = ["nodes", "far", "leaves", "leaf_fast", "pieces", "angles", "reclass", "overflow"]
GWN_NCOUNTERS = len(COUNTER_NAMES)
(GWN_I_SUMMARY, GWN_I_LEAVES, GWN_I_NODES, GWN_I_MOMENTS, GWN_I_UNCENTERED, GWN_I_COMPLEX, GWN_I_MULTIPOLE,
 GWN_I_FARBETA, GWN_I_LEAF_TRIMS) = range(9)

EXPORTED = ["gwn_default_params", "gwn_build2d", "gwn_build3d", "gwn_nurbs2d_extract", "gwn_nurbs3d_extract",
            "gwn_set_params",
            "gwn_get_params", "gwn_query", "gwn_query_noalloc", "gwn_query_scratch_bytes",
            "gwn_query_batch", "gwn_query_counters", "gwn_model_bytes", "gwn_inspect", "gwn_profile",
            "gwn_profile_kernel", "gwn_free", "gwn_last_error"]
GWN_K_QUERY2D, GWN_K_TRAV3D, GWN_K_NEAR3D = 0, 1, 2
GWN_NOALLOC_SCRATCH_BYTES = 96 << 20


class GwnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gwn status {status}: {msg}")
        self.status = status


class gwn_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("beta_mixed", ctypes.c_double), ("taylor_order", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reclass_band", ctypes.c_double), ("max_diag_frac", ctypes.c_double),
                ("eps_on", ctypes.c_double), ("gl_nodes", ctypes.c_int32), ("device", ctypes.c_int32),
                ("near_ratio", ctypes.c_double), ("eps_q", ctypes.c_double), ("leaf_far", ctypes.c_int32),
                ("wave_accept", ctypes.c_int32), ("far_tol", ctypes.c_double)]


class gwn_curves2d(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int64), ("degree", ctypes.c_void_p), ("cp_offset", ctypes.c_void_p),
                ("cp_xy", ctypes.c_void_p), ("cp_w", ctypes.c_void_p)]


class gwn_nurbs2d(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int64), ("degree", ctypes.c_void_p), ("cp_offset", ctypes.c_void_p),
                ("cp_xy", ctypes.c_void_p), ("cp_w", ctypes.c_void_p), ("knot_offset", ctypes.c_void_p),
                ("knots", ctypes.c_void_p)]


class gwn_nurbs3d(ctypes.Structure):
    _fields_ = [("n_surfaces", ctypes.c_int64)] + [(f, ctypes.c_void_p) for f in (
        "degree_u", "degree_v", "n_u", "n_v", "cp_offset", "cp_xyz", "cp_w", "knot_u_offset", "knots_u",
        "knot_v_offset", "knots_v", "trim_offset", "trim_degree", "trim_cp_offset", "trim_cp_uv", "trim_cp_w",
        "trim_knot_offset", "trim_knots")]


class gwn_patches3d(ctypes.Structure):
    _fields_ = [("n_patches", ctypes.c_int64), ("cp_xyz", ctypes.c_void_p), ("cp_w", ctypes.c_void_p),
                ("trim_offset", ctypes.c_void_p), ("trim_degree", ctypes.c_void_p),
                ("trim_cp_offset", ctypes.c_void_p), ("trim_cp_uv", ctypes.c_void_p), ("trim_cp_w", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() "
                               "(or python paper_2605_19200_amd/build.py)")
        # PyTorch carries its own HIP runtime; it has to be loaded before the
        # library's, or torch finds no GPU once the library has initialised
        # the device (the binding hands the library torch's device memory)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.gwn_default_params.argtypes = [ctypes.POINTER(gwn_params)]
        L.gwn_default_params.restype = None
        for name, args in [
            ("gwn_build2d", [ctypes.POINTER(gwn_curves2d), ctypes.POINTER(gwn_params), ctypes.POINTER(vp)]),
            ("gwn_build3d", [ctypes.POINTER(gwn_patches3d), ctypes.POINTER(gwn_params), ctypes.POINTER(vp)]),
            ("gwn_nurbs2d_extract", [ctypes.POINTER(gwn_nurbs2d), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                     vp, vp, vp, vp]),
            ("gwn_nurbs3d_extract", [ctypes.POINTER(gwn_nurbs3d), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                     ctypes.POINTER(i64), vp, vp, vp, vp, vp, vp, vp]),
            ("gwn_set_params", [vp, ctypes.POINTER(gwn_params)]),
            ("gwn_get_params", [vp, ctypes.POINTER(gwn_params)]),
            ("gwn_query", [vp, vp, i64, vp, vp, vp]),
            ("gwn_query_noalloc", [vp, vp, i64, vp, vp, vp]),
            ("gwn_query_scratch_bytes", [vp, i64, i32, ctypes.POINTER(i64)]),
            ("gwn_query_batch", [i32, vp, vp, vp, vp, vp, vp]),
            ("gwn_query_counters", [vp, vp, i64, vp, vp]),
            ("gwn_model_bytes", [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
            ("gwn_inspect", [vp, i32, vp, i64, ctypes.POINTER(i64)]),
            ("gwn_free", [vp]),
            ("gwn_profile", [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
            ("gwn_profile_kernel", [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.gwn_last_error.argtypes = []
        L.gwn_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != GWN_OK:
        raise GwnError(status, lib().gwn_last_error().decode(errors="replace"))


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def gwn_default_params(**overrides) -> gwn_params:
    p = gwn_params()
    lib().gwn_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


# dimension and device of every handle built here, for argument checks
_handles: dict = {}


def _handle_key(h):
    return h.value if isinstance(h, ctypes.c_void_p) else int(h)


def _handle_info(h):
    """(dim, device) of a handle."""
    if h is None or _handle_key(h) in (None, 0):
        raise ValueError("NULL handle")
    info = _handles.get(_handle_key(h))
    if info is None:
        p = gwn_params()
        _check(lib().gwn_get_params(h, ctypes.byref(p)))
        summ = np.empty(8)
        cnt = ctypes.c_int64()
        _check(lib().gwn_inspect(h, GWN_I_SUMMARY, _p(summ), 1, ctypes.byref(cnt)))
        info = (int(summ[0]), int(p.device))
        _handles[_handle_key(h)] = info
    return info


def _register(h, dim, params):
    dev = params.device if params is not None else 0
    _handles[_handle_key(h)] = (dim, int(dev))


def gwn_build2d(curves, params: gwn_params | None = None):
    """Build a 2D model from a ``workloads.Curves2D``; returns the handle."""
    deg, off = _np(curves.degree, np.int32), _np(curves.cp_offset, np.int64)
    xy, w = _np(curves.cp_xy, np.float64), _np(curves.cp_w, np.float64)
    c = gwn_curves2d(curves.n, _p(deg), _p(off), _p(xy), _p(w))
    h = ctypes.c_void_p()
    _check(lib().gwn_build2d(ctypes.byref(c), ctypes.byref(params) if params else None, ctypes.byref(h)))
    _register(h, 2, params)
    return h


def gwn_build3d(patches, params: gwn_params | None = None):
    """Build a 3D model from a ``workloads.Patches3D``; returns the handle."""
    arrs = [_np(patches.cp_xyz, np.float64), _np(patches.cp_w, np.float64), _np(patches.trim_offset, np.int64),
            _np(patches.trim_degree, np.int32), _np(patches.trim_cp_offset, np.int64),
            _np(patches.trim_cp_uv, np.float64), _np(patches.trim_cp_w, np.float64)]
    c = gwn_patches3d(patches.n, *[_p(a) for a in arrs])
    h = ctypes.c_void_p()
    _check(lib().gwn_build3d(ctypes.byref(c), ctypes.byref(params) if params else None, ctypes.byref(h)))
    _register(h, 3, params)
    return h


def gwn_nurbs2d_extract(nurbs):
    """Bezier segments of a ``workloads.Nurbs2D`` as a ``workloads.Curves2D``
    (two calls of the C entry point: sizes, then the arrays)."""
    from .workloads import Curves2D
    arrs = [_np(nurbs.degree, np.int32), _np(nurbs.cp_offset, np.int64), _np(nurbs.cp_xy, np.float64),
            _np(nurbs.cp_w, np.float64), _np(nurbs.knot_offset, np.int64), _np(nurbs.knots, np.float64)]
    c = gwn_nurbs2d(nurbs.n, *[_p(a) for a in arrs])
    ns, npt = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().gwn_nurbs2d_extract(ctypes.byref(c), ctypes.byref(ns), ctypes.byref(npt), None, None, None, None))
    if ns.value == 0:
        return Curves2D.from_list([])
    deg = np.zeros(ns.value, np.int32)
    off = np.zeros(ns.value + 1, np.int64)
    xy = np.zeros((npt.value, 2), np.float64)
    w = np.zeros(npt.value, np.float64)
    _check(lib().gwn_nurbs2d_extract(ctypes.byref(c), ctypes.byref(ns), ctypes.byref(npt), _p(deg), _p(off),
                                     _p(xy), _p(w)))
    return Curves2D(deg, off, xy, w)


def gwn_nurbs3d_extract(nurbs):
    """Rational bicubic Bezier patches of a ``workloads.Nurbs3D`` as a
    ``workloads.Patches3D`` (two calls of the C entry point: sizes, then the
    arrays)."""
    from .workloads import Patches3D
    t = nurbs.trims
    arrs = [_np(nurbs.degree_u, np.int32), _np(nurbs.degree_v, np.int32), _np(nurbs.n_u, np.int32),
            _np(nurbs.n_v, np.int32), _np(nurbs.cp_offset, np.int64), _np(nurbs.cp_xyz, np.float64),
            _np(nurbs.cp_w, np.float64), _np(nurbs.knot_u_offset, np.int64), _np(nurbs.knots_u, np.float64),
            _np(nurbs.knot_v_offset, np.int64), _np(nurbs.knots_v, np.float64), _np(nurbs.trim_offset, np.int64),
            _np(t.degree, np.int32), _np(t.cp_offset, np.int64), _np(t.cp_xy, np.float64), _np(t.cp_w, np.float64),
            _np(t.knot_offset, np.int64), _np(t.knots, np.float64)]
    c = gwn_nurbs3d(nurbs.n, *[_p(a) for a in arrs])
    n, nt, nc = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    cnt = [ctypes.byref(n), ctypes.byref(nt), ctypes.byref(nc)]
    _check(lib().gwn_nurbs3d_extract(ctypes.byref(c), *cnt, None, None, None, None, None, None, None))
    if n.value == 0:
        return Patches3D.from_list([])
    out = [np.zeros((n.value, 16, 3)), np.zeros((n.value, 16)), np.zeros(n.value + 1, np.int64),
           np.zeros(nt.value, np.int32), np.zeros(nt.value + 1, np.int64), np.zeros((nc.value, 2)),
           np.zeros(nc.value)]
    _check(lib().gwn_nurbs3d_extract(ctypes.byref(c), *cnt, *[_p(a) for a in out]))
    return Patches3D(*out)


def gwn_set_params(h, params: gwn_params):
    _check(lib().gwn_set_params(h, ctypes.byref(params)))


def gwn_get_params(h) -> gwn_params:
    p = gwn_params()
    _check(lib().gwn_get_params(h, ctypes.byref(p)))
    return p


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check_layout(name, t, dtype, shape):
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _check_device(name, t, device):
    import torch
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU, got {t.device}")
    if device < 0:
        raise ValueError("host-only handle cannot be queried")
    idx = t.device.index if t.device.index is not None else torch.cuda.current_device()
    if idx != device:
        raise ValueError(f"{name} is on cuda:{idx}, the model on cuda:{device}")


def _check_tensors(device, specs):
    """The kernels read and write raw device pointers: refuse anything but
    contiguous tensors of the expected dtype and shape on the model's device
    (ValueError before any launch).  specs: (name, tensor, dtype, shape)."""
    for name, t, dt, shape in specs:
        _check_layout(name, t, dt, shape)
    for name, t, _, _ in specs:
        _check_device(name, t, device)


def _check_query_args(dim, device, points, out_gwn, out_inside, n=None):
    import torch
    if not isinstance(points, torch.Tensor) or points.ndim != 2:
        raise ValueError(f"points must be a [n, {dim}] tensor")
    n = points.shape[0] if n is None else n
    specs = [("points", points, torch.float64, (n, dim)), ("out_gwn", out_gwn, torch.float64, (n,))]
    if out_inside is not None:
        specs.append(("out_inside", out_inside, torch.uint8, (n,)))
    _check_tensors(device, specs)


def _query_call(fn, h, points, out_gwn, out_inside, stream):
    dim, device = _handle_info(h)
    _check_query_args(dim, device, points, out_gwn, out_inside)
    n = points.shape[0]
    _check(fn(h, ctypes.c_void_p(points.data_ptr()), n, ctypes.c_void_p(out_gwn.data_ptr()),
              ctypes.c_void_p(out_inside.data_ptr()) if out_inside is not None else None, _stream_ptr(stream)))


def gwn_query(h, points, out_gwn, out_inside=None, stream=None):
    """points: device float64 tensor [n, dim]; out_gwn: device float64 [n];
    out_inside: device uint8 [n] or None.  Asynchronous on `stream`."""
    _query_call(lib().gwn_query, h, points, out_gwn, out_inside, stream)


def gwn_query_noalloc(h, points, out_gwn, out_inside=None, stream=None):
    """As gwn_query, with the launch's scratch in the library's fixed
    per-GPU array (no device allocation; calls overlapping on one GPU race)."""
    _query_call(lib().gwn_query_noalloc, h, points, out_gwn, out_inside, stream)


def gwn_query_scratch_bytes(h, n: int, n_seg: int = 1) -> int:
    """Device scratch bytes of one query call over n rows in n_seg segments."""
    b = ctypes.c_int64()
    _check(lib().gwn_query_scratch_bytes(h, int(n), int(n_seg), ctypes.byref(b)))
    return b.value


def gwn_query_batch(models, seg_offset, points, out_gwn, out_inside=None, stream=None):
    """models: list of handles (one per segment); seg_offset: host int64
    [n_seg + 1]; points/out_*: device tensors covering all segments."""
    import torch
    n_seg = len(models)
    off = _np(seg_offset, np.int64)
    if off.ndim != 1 or off.size != n_seg + 1:
        raise ValueError(f"seg_offset must hold n_seg + 1 = {n_seg + 1} entries, got {off.size}")
    if n_seg:
        if off[0] != 0 or np.any(np.diff(off) < 0):
            raise ValueError("seg_offset must start at 0 and be non-decreasing")
        infos = [_handle_info(m) for m in models]
        dims, devs = {d for d, _ in infos}, {v for _, v in infos}
        if len(dims) != 1 or len(devs) != 1:
            raise ValueError("all models of a batch must share one dimension and one device")
        (dim,), (device,) = dims, devs
        if not isinstance(points, torch.Tensor) or points.ndim != 2:
            raise ValueError(f"points must be a [n, {dim}] tensor")
        _check_query_args(dim, device, points, out_gwn, out_inside, n=int(off[-1]))
    arr = (ctypes.c_void_p * max(n_seg, 1))(*[m.value if isinstance(m, ctypes.c_void_p) else m for m in models])
    _check(lib().gwn_query_batch(n_seg, ctypes.cast(arr, ctypes.c_void_p), _p(off),
                                 ctypes.c_void_p(points.data_ptr()), ctypes.c_void_p(out_gwn.data_ptr()),
                                 ctypes.c_void_p(out_inside.data_ptr()) if out_inside is not None else None,
                                 _stream_ptr(stream)))


def gwn_query_counters(h, points, counters, stream=None):
    """counters: device int64 tensor [GWN_NCOUNTERS] (overwritten)."""
    import torch
    dim, device = _handle_info(h)
    if not isinstance(points, torch.Tensor) or points.ndim != 2:
        raise ValueError(f"points must be a [n, {dim}] tensor")
    _check_tensors(device, [("points", points, torch.float64, (points.shape[0], dim)),
                            ("counters", counters, torch.int64, (GWN_NCOUNTERS,))])
    _check(lib().gwn_query_counters(h, ctypes.c_void_p(points.data_ptr()), points.shape[0],
                                    ctypes.c_void_p(counters.data_ptr()), _stream_ptr(stream)))


def gwn_model_bytes(h):
    r, q = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().gwn_model_bytes(h, ctypes.byref(r), ctypes.byref(q)))
    return r.value, q.value


_WIDTH = {GWN_I_SUMMARY: lambda d: 8, GWN_I_LEAVES: lambda d: 13 if d == 2 else 65, GWN_I_NODES: lambda d: 13,
          GWN_I_MOMENTS: lambda d: d + d * d + d ** 3, GWN_I_UNCENTERED: lambda d: d + d * d + d ** 3,
          GWN_I_COMPLEX: lambda d: 34, GWN_I_MULTIPOLE: lambda d: 72, GWN_I_FARBETA: lambda d: 1,
          GWN_I_LEAF_TRIMS: lambda d: 10}


def gwn_inspect(h, what: int) -> np.ndarray:
    cnt = ctypes.c_int64()
    _check(lib().gwn_inspect(h, GWN_I_SUMMARY, None, 0, ctypes.byref(cnt)))
    summ = np.empty(8)
    _check(lib().gwn_inspect(h, GWN_I_SUMMARY, _p(summ), 1, ctypes.byref(cnt)))
    dim = int(summ[0])
    _check(lib().gwn_inspect(h, what, None, 0, ctypes.byref(cnt)))
    width = _WIDTH[what](dim)
    out = np.empty((cnt.value, width))
    if cnt.value:
        _check(lib().gwn_inspect(h, what, _p(out), cnt.value, ctypes.byref(cnt)))
    return out


def gwn_profile(enable: bool):
    """Start (True) or stop (False) query-kernel event timing; stopping
    returns (total_ms, launches)."""
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    _check(lib().gwn_profile(1 if enable else 0, ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def gwn_profile_kernel(kernel: int):
    """(total_ms, launches) of one kernel (GWN_K_*) in the set collected by
    the last gwn_profile(False)."""
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    _check(lib().gwn_profile_kernel(int(kernel), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def gwn_free(h):
    if h is not None:
        _handles.pop(_handle_key(h), None)
        _check(lib().gwn_free(h))


def gwn_last_error() -> str:
    return lib().gwn_last_error().decode(errors="replace")


class Model:
    """Owning wrapper of a handle with a torch-facing ``query``."""

    def __init__(self, geometry, params: gwn_params | None = None, **overrides):
        self.params = params if params is not None else gwn_default_params()
        for k, v in overrides.items():
            setattr(self.params, k, v)
        if hasattr(geometry, "cp_xyz"):
            self.dim = 3
            self.h = gwn_build3d(geometry, self.params)
        else:
            self.dim = 2
            self.h = gwn_build2d(geometry, self.params)

    def set(self, **kw):
        p = gwn_get_params(self.h)
        for k, v in kw.items():
            setattr(p, k, v)
        gwn_set_params(self.h, p)
        self.params = p

    def query(self, points, out=None, inside=None, stream=None):
        import torch
        if not isinstance(points, torch.Tensor) or points.ndim != 2:
            raise ValueError(f"points must be a [n, {self.dim}] tensor")
        n = points.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=points.device)
        if inside is None:
            inside = torch.empty(n, dtype=torch.uint8, device=points.device)
        gwn_query(self.h, points, out, inside, stream)
        return out, inside

    def counters(self, points, stream=None):
        import torch
        c = torch.zeros(GWN_NCOUNTERS, dtype=torch.int64, device=points.device)
        gwn_query_counters(self.h, points, c, stream)
        return dict(zip(COUNTER_NAMES, c.cpu().tolist()))

    def bytes(self):
        return gwn_model_bytes(self.h)

    def inspect(self, what):
        return gwn_inspect(self.h, what)

    def close(self):
        if self.h is not None:
            gwn_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
