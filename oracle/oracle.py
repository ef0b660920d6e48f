"""ctypes front end of the CPU oracle (``gwn_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the engine.  ``build()`` compiles the
C source with gcc; nothing here is shared with the GPU engine.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gwn_oracle.c")
LIB = os.path.join(HERE, "_gwn_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", LIB, SRC, "-lm"]
        subprocess.check_call(cmd)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        L.oracle_gwn2d.argtypes = [ctypes.c_int64, p, p, p, p, ctypes.c_int64, p, p, ctypes.c_double, ctypes.c_int]
        L.oracle_gwn2d.restype = ctypes.c_int
        L.oracle_gwn3d.argtypes = [ctypes.c_int64, p, p, p, p, p, p, p, ctypes.c_int64, p, p,
                                   ctypes.c_double, ctypes.c_int]
        L.oracle_gwn3d.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_last_unconverged.restype = ctypes.c_longlong
        L.oracle_last_errbound.restype = ctypes.c_double
        L.oracle_gl_nodes.argtypes = [p, p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class OracleUnconverged(RuntimeError):
    """The adaptive quadrature accepted a panel at a work limit with its
    error estimate above the tolerance: the value is not trustworthy."""


#: quadrature panels accepted unconverged (at a work limit, with an error
#: estimate above the tolerance) by the last gwn2d / gwn3d call
last_unconverged = 0
#: largest per-query bound, in units of w, on the error of those panels
last_errbound = 0.0
#: strict calls raise when a query's bound exceeds this (the tightest pins
#: compare at 1e-11 and above; the parity bar is 1e-6)
STRICT_ERRBOUND = 1e-12


def _converged(strict):
    global last_unconverged, last_errbound
    last_unconverged = int(lib().oracle_last_unconverged())
    last_errbound = float(lib().oracle_last_errbound())
    if strict and last_errbound > STRICT_ERRBOUND:
        raise OracleUnconverged(f"{last_unconverged} quadrature panel(s) accepted at a work limit, "
                                f"error bound {last_errbound:.3e} in w")


def default_eps_on(lo, hi, rel=1e-12):
    return rel * float(np.linalg.norm(np.asarray(hi) - np.asarray(lo)))


def gwn2d(curves, q, eps_on=None, threads=0, strict=True):
    """Direct FP64 GWN of a ``Curves2D`` set at points ``q`` [n, 2].  The
    count of panels the adaptive quadrature accepted unconverged and the
    largest per-query bound on their error are kept in ``last_unconverged``
    and ``last_errbound``; with ``strict`` a bound above ``STRICT_ERRBOUND``
    raises ``OracleUnconverged``."""
    q = _c(q, np.float64).reshape(-1, 2)
    deg = _c(curves.degree, np.int32)
    off = _c(curves.cp_offset, np.int64)
    xy = _c(curves.cp_xy, np.float64)
    w = _c(curves.cp_w, np.float64)
    if eps_on is None:
        eps_on = default_eps_on(*curves.bbox()) if curves.n else 1e-12
    out = np.empty(q.shape[0])
    r = lib().oracle_gwn2d(curves.n, _ptr(deg), _ptr(off), _ptr(xy), _ptr(w), q.shape[0], _ptr(q), _ptr(out),
                           float(eps_on), int(threads))
    if r != 0:
        raise ValueError(f"oracle_gwn2d rejected the input (code {r})")
    _converged(strict)
    return out


def gwn3d(patches, q, eps_on=None, threads=0, strict=True):
    """Direct FP64 GWN of a ``Patches3D`` set at points ``q`` [n, 3]
    (``strict`` and ``last_unconverged`` as for ``gwn2d``)."""
    q = _c(q, np.float64).reshape(-1, 3)
    cp = _c(patches.cp_xyz, np.float64)
    w = _c(patches.cp_w, np.float64)
    toff = _c(patches.trim_offset, np.int64)
    tdeg = _c(patches.trim_degree, np.int32)
    tcoff = _c(patches.trim_cp_offset, np.int64)
    tuv = _c(patches.trim_cp_uv, np.float64)
    tw = _c(patches.trim_cp_w, np.float64)
    if eps_on is None:
        eps_on = default_eps_on(*patches.bbox()) if patches.n else 1e-12
    out = np.empty(q.shape[0])
    r = lib().oracle_gwn3d(patches.n, _ptr(cp), _ptr(w), _ptr(toff), _ptr(tdeg), _ptr(tcoff), _ptr(tuv), _ptr(tw),
                           q.shape[0], _ptr(q), _ptr(out), float(eps_on), int(threads))
    if r != 0:
        raise ValueError(f"oracle_gwn3d rejected the input (code {r})")
    _converged(strict)
    return out


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def gl_nodes():
    x = np.empty(10)
    w = np.empty(10)
    n = lib().oracle_gl_nodes(_ptr(x), _ptr(w))
    return x[:n], w[:n]
