"""Seeded synthetic inputs: rational Bezier curve sets (2D), trimmed rational
bicubic patch sets (3D) and query point sets.

This module builds geometry only.  It contains no winding-number, moment,
hierarchy or quadrature arithmetic, so both the CPU oracle and the GPU engine
can be fed from it without sharing any of the method's code.

Randomness comes from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), used as
a counter-based generator: draw ``k`` of stream ``s`` under seed ``seed`` is
``mix(base(seed, s) + k * GAMMA)``.  Every purpose (radii, weights, queries,
...) has its own stream, so changing one size never shifts another stream.

Data layout (matches the C ABI in ``include/gwn.h``):

* ``Curves2D``: ``degree`` int32[n], ``cp_offset`` int64[n+1] (CSR into the
  control-point arrays), ``cp_xy`` float64[n_cp, 2] Euclidean control points,
  ``cp_w`` float64[n_cp] weights (> 0).
* ``Patches3D``: ``cp_xyz`` float64[n, 16, 3] bicubic control points stored
  with the u index major (``4*i + j``, i along u, j along v), ``cp_w``
  float64[n, 16], and trim curves in CSR form: ``trim_offset`` int64[n+1]
  (empty range = untrimmed), ``trim_degree`` int32[n_trim] (1 or 2),
  ``trim_cp_offset`` int64[n_trim+1], ``trim_cp_uv`` float64[n_tcp, 2],
  ``trim_cp_w`` float64[n_tcp].  A patch's trim curves form closed loops of
  consecutive curves; the outer loop runs counter-clockwise in (u, v), holes
  clockwise, and when present the outer square is listed explicitly.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

# --------------------------------------------------------------------------
# SplitMix64
# --------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


class Rng:
    """Counter-based SplitMix64 stream ``(seed, purpose)``."""

    def __init__(self, seed: int, purpose: str):
        h = hashlib.sha256(f"{int(seed)}/{purpose}".encode()).digest()
        self._base = _mix64(np.array([int.from_bytes(h[:8], "little")], dtype=np.uint64))[0]
        self._count = 0

    def u64(self, n: int) -> np.ndarray:
        k = np.arange(self._count + 1, self._count + n + 1, dtype=np.uint64)
        self._count += n
        with np.errstate(over="ignore"):
            return _mix64(self._base + k * _GAMMA)

    def uniform(self, n, lo=0.0, hi=1.0) -> np.ndarray:
        if isinstance(n, tuple):
            size = int(np.prod(n))
            return self.uniform(size, lo, hi).reshape(n)
        u = (self.u64(int(n)) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def integers(self, n: int, lo: int, hi: int) -> np.ndarray:
        """Uniform integers in [lo, hi]."""
        u = self.uniform(n)
        return np.minimum(lo + np.floor(u * (hi - lo + 1)).astype(np.int64), hi)

    def permutation(self, n: int) -> np.ndarray:
        return np.argsort(self.u64(n), kind="stable")


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Curves2D:
    degree: np.ndarray      # int32[n]
    cp_offset: np.ndarray   # int64[n+1]
    cp_xy: np.ndarray       # float64[n_cp, 2]
    cp_w: np.ndarray        # float64[n_cp]

    @property
    def n(self) -> int:
        return int(self.degree.shape[0])

    def curve(self, i):
        a, b = int(self.cp_offset[i]), int(self.cp_offset[i + 1])
        return self.cp_xy[a:b], self.cp_w[a:b]

    @staticmethod
    def from_list(curves) -> "Curves2D":
        """``curves``: iterable of (points[k,2], weights[k])."""
        deg, off, xy, w = [], [0], [], []
        for p, wt in curves:
            p = np.asarray(p, dtype=np.float64).reshape(-1, 2)
            wt = np.asarray(wt, dtype=np.float64).reshape(-1)
            assert p.shape[0] == wt.shape[0] and 2 <= p.shape[0] <= 4
            deg.append(p.shape[0] - 1)
            off.append(off[-1] + p.shape[0])
            xy.append(p)
            w.append(wt)
        if not deg:
            return Curves2D(np.zeros(0, np.int32), np.zeros(1, np.int64),
                            np.zeros((0, 2)), np.zeros(0))
        return Curves2D(np.asarray(deg, np.int32), np.asarray(off, np.int64),
                        np.ascontiguousarray(np.concatenate(xy)), np.ascontiguousarray(np.concatenate(w)))

    def to_list(self):
        return [self.curve(i) for i in range(self.n)]

    def subset(self, idx) -> "Curves2D":
        return Curves2D.from_list([self.curve(int(i)) for i in idx])

    def concat(self, other: "Curves2D") -> "Curves2D":
        return Curves2D.from_list(self.to_list() + other.to_list())

    def bbox(self):
        return self.cp_xy.min(axis=0), self.cp_xy.max(axis=0)


@dataclasses.dataclass
class Nurbs2D:
    """2D NURBS curves (input of ``gwn.gwn_nurbs2d_extract``): degree 1..3,
    clamped knot vectors, CSR control points and knots."""
    degree: np.ndarray       # int32[n]
    cp_offset: np.ndarray    # int64[n+1]
    cp_xy: np.ndarray        # float64[n_cp, 2]
    cp_w: np.ndarray         # float64[n_cp]
    knot_offset: np.ndarray  # int64[n+1]
    knots: np.ndarray        # float64[n_knots]

    @property
    def n(self) -> int:
        return int(self.degree.shape[0])

    @staticmethod
    def from_list(curves) -> "Nurbs2D":
        """``curves``: iterable of (degree, points[k,2], weights[k], knots[k+degree+1])."""
        deg, off, xy, w, koff, kn = [], [0], [], [], [0], []
        for p, pts, wt, U in curves:
            pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
            deg.append(int(p))
            off.append(off[-1] + pts.shape[0])
            xy.append(pts)
            w.append(np.asarray(wt, dtype=np.float64).reshape(-1))
            kn.append(np.asarray(U, dtype=np.float64).reshape(-1))
            koff.append(koff[-1] + kn[-1].shape[0])
        cat = (lambda a, shape: np.ascontiguousarray(np.concatenate(a)) if a else np.zeros(shape))
        return Nurbs2D(np.asarray(deg, np.int32), np.asarray(off, np.int64), cat(xy, (0, 2)), cat(w, (0,)),
                       np.asarray(koff, np.int64), cat(kn, (0,)))


@dataclasses.dataclass
class Nurbs3D:
    """Trimmed NURBS surfaces (input of ``gwn.gwn_nurbs3d_extract``): degrees
    1..3 per direction, clamped knot vectors, an n_u x n_v net per surface
    (u-major), trim curves as 2D NURBS of degree 1..2 in the surface's
    parameter domain."""
    degree_u: np.ndarray        # int32[n]
    degree_v: np.ndarray        # int32[n]
    n_u: np.ndarray             # int32[n]
    n_v: np.ndarray             # int32[n]
    cp_offset: np.ndarray       # int64[n+1]
    cp_xyz: np.ndarray          # float64[n_cp, 3]
    cp_w: np.ndarray            # float64[n_cp]
    knot_u_offset: np.ndarray   # int64[n+1]
    knots_u: np.ndarray
    knot_v_offset: np.ndarray   # int64[n+1]
    knots_v: np.ndarray
    trim_offset: np.ndarray     # int64[n+1]
    trims: Nurbs2D              # all trim curves, surface after surface

    @property
    def n(self) -> int:
        return int(self.degree_u.shape[0])

    @staticmethod
    def from_list(surfaces) -> "Nurbs3D":
        """``surfaces``: iterable of (pu, pv, cp[n_u, n_v, 3], w[n_u, n_v],
        U, V, trims) with ``trims`` a list of (degree, uv[k, 2], w[k], knots)
        2D NURBS curves (empty = untrimmed)."""
        pu, pv, nu, nv, off, xyz, w, kuo, ku, kvo, kv, toff, tr = ([], [], [], [], [0], [], [], [0], [], [0], [],
                                                                    [0], [])
        for p_u, p_v, cp, wt, U, V, trims in surfaces:
            cp = np.asarray(cp, np.float64)
            pu.append(int(p_u))
            pv.append(int(p_v))
            nu.append(cp.shape[0])
            nv.append(cp.shape[1])
            off.append(off[-1] + cp.shape[0] * cp.shape[1])
            xyz.append(cp.reshape(-1, 3))
            w.append(np.asarray(wt, np.float64).reshape(-1))
            ku.append(np.asarray(U, np.float64).reshape(-1))
            kv.append(np.asarray(V, np.float64).reshape(-1))
            kuo.append(kuo[-1] + ku[-1].shape[0])
            kvo.append(kvo[-1] + kv[-1].shape[0])
            tr.extend(trims)
            toff.append(toff[-1] + len(trims))
        cat = (lambda a, shape: np.ascontiguousarray(np.concatenate(a)) if a else np.zeros(shape))
        i32 = (lambda a: np.asarray(a, np.int32))
        i64 = (lambda a: np.asarray(a, np.int64))
        return Nurbs3D(i32(pu), i32(pv), i32(nu), i32(nv), i64(off), cat(xyz, (0, 3)), cat(w, (0,)), i64(kuo),
                       cat(ku, (0,)), i64(kvo), cat(kv, (0,)), i64(toff), Nurbs2D.from_list(tr))


@dataclasses.dataclass
class Patches3D:
    cp_xyz: np.ndarray          # float64[n,16,3]
    cp_w: np.ndarray            # float64[n,16]
    trim_offset: np.ndarray     # int64[n+1]
    trim_degree: np.ndarray     # int32[n_trim]
    trim_cp_offset: np.ndarray  # int64[n_trim+1]
    trim_cp_uv: np.ndarray      # float64[n_tcp,2]
    trim_cp_w: np.ndarray       # float64[n_tcp]

    @property
    def n(self) -> int:
        return int(self.cp_xyz.shape[0])

    def trims(self, i):
        """List of (uv[k,2], w[k]) trim curves of patch i."""
        out = []
        for c in range(int(self.trim_offset[i]), int(self.trim_offset[i + 1])):
            a, b = int(self.trim_cp_offset[c]), int(self.trim_cp_offset[c + 1])
            out.append((self.trim_cp_uv[a:b], self.trim_cp_w[a:b]))
        return out

    @staticmethod
    def from_list(patches) -> "Patches3D":
        """``patches``: iterable of (cp_xyz[16,3] or [4,4,3], cp_w[16], trims)
        with ``trims`` a list of (uv[k,2], w[k]) curves (empty = untrimmed)."""
        cps, ws, toff, tdeg, tcoff, tuv, tw = [], [], [0], [], [0], [], []
        for cp, w, trims in patches:
            cps.append(np.asarray(cp, np.float64).reshape(16, 3))
            ws.append(np.asarray(w, np.float64).reshape(16))
            for uv, tws in trims:
                uv = np.asarray(uv, np.float64).reshape(-1, 2)
                tws = np.asarray(tws, np.float64).reshape(-1)
                tdeg.append(uv.shape[0] - 1)
                tcoff.append(tcoff[-1] + uv.shape[0])
                tuv.append(uv)
                tw.append(tws)
            toff.append(toff[-1] + len(trims))
        n = len(cps)
        return Patches3D(
            np.ascontiguousarray(np.stack(cps)) if n else np.zeros((0, 16, 3)),
            np.ascontiguousarray(np.stack(ws)) if n else np.zeros((0, 16)),
            np.asarray(toff, np.int64), np.asarray(tdeg, np.int32), np.asarray(tcoff, np.int64),
            np.ascontiguousarray(np.concatenate(tuv)) if tuv else np.zeros((0, 2)),
            np.ascontiguousarray(np.concatenate(tw)) if tw else np.zeros(0))

    def to_list(self):
        return [(self.cp_xyz[i], self.cp_w[i], self.trims(i)) for i in range(self.n)]

    def subset(self, idx) -> "Patches3D":
        lst = self.to_list()
        return Patches3D.from_list([lst[int(i)] for i in idx])

    def concat(self, other: "Patches3D") -> "Patches3D":
        return Patches3D.from_list(self.to_list() + other.to_list())

    def bbox(self):
        p = self.cp_xyz.reshape(-1, 3)
        return p.min(axis=0), p.max(axis=0)


# --------------------------------------------------------------------------
# exact conic arcs and degree elevation (geometric construction only)
# --------------------------------------------------------------------------
def arc_quadratic(center, radius, a0, a1):
    """Rational quadratic Bezier of the circular arc from angle a0 to a1
    (|a1 - a0| < pi): control points and weights."""
    am = 0.5 * (a0 + a1)
    half = 0.5 * abs(a1 - a0)
    c = np.asarray(center, np.float64)
    p0 = c + radius * np.array([math.cos(a0), math.sin(a0)])
    p2 = c + radius * np.array([math.cos(a1), math.sin(a1)])
    p1 = c + (radius / math.cos(half)) * np.array([math.cos(am), math.sin(am)])
    return np.stack([p0, p1, p2]), np.array([1.0, math.cos(half), 1.0])


def elevate_homogeneous(h: np.ndarray, axis: int = 0) -> np.ndarray:
    """Degree elevation by one of homogeneous Bezier control points along
    ``axis`` (points indexed 0..n along that axis)."""
    h = np.moveaxis(np.asarray(h, np.float64), axis, 0)
    n = h.shape[0] - 1
    out = np.empty((n + 2,) + h.shape[1:])
    out[0] = h[0]
    out[n + 1] = h[n]
    for i in range(1, n + 1):
        a = i / (n + 1)
        out[i] = a * h[i - 1] + (1 - a) * h[i]
    return np.moveaxis(out, 0, axis)


def elevate_curve(p, w, to_degree=3):
    """Elevate a rational Bezier curve (points, weights) to ``to_degree``."""
    p = np.asarray(p, np.float64)
    w = np.asarray(w, np.float64)
    h = np.concatenate([p * w[:, None], w[:, None]], axis=1)
    while h.shape[0] - 1 < to_degree:
        h = elevate_homogeneous(h, 0)
    return h[:, :2] / h[:, 2:3], h[:, 2].copy()


def circle_curves(center=(0.0, 0.0), radius=1.0, n_arcs=4, ccw=True, degree=3, phase=0.0):
    """Closed circle as ``n_arcs`` exact rational arcs (degree 2 or elevated)."""
    out = []
    step = 2 * math.pi / n_arcs * (1 if ccw else -1)
    first = None
    for k in range(n_arcs):
        p, w = arc_quadratic(center, radius, phase + k * step, phase + (k + 1) * step)
        if first is None:
            first = p[0].copy()
        if k == n_arcs - 1:
            p[-1] = first        # close the loop exactly
        if degree > 2:
            p, w = elevate_curve(p, w, degree)
        out.append((p, w))
    return out


# --------------------------------------------------------------------------
# 2D workloads
# --------------------------------------------------------------------------
def bbox_queries_uniform(rng: Rng, lo, hi, n, scale=1.1):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo) * scale
    d = lo.shape[0]
    u = rng.uniform((n, d))
    return np.ascontiguousarray(c - h + 2 * h * u)


def grid_queries(lo, hi, shape):
    """Cell-centred grid over [lo, hi], x fastest (row-major in y)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    axes = [lo[k] + (np.arange(shape[k]) + 0.5) * (hi[k] - lo[k]) / shape[k] for k in range(len(shape))]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    return np.ascontiguousarray(np.stack([m.reshape(-1) for m in mesh], axis=1))


def star_loop(seed=1, n_curves=64):
    """One closed star-shaped loop of ``n_curves`` rational cubics: 3*n control
    points at equal angles, radius 1 + 0.3*U(-1,1), weights U(0.5, 2) per curve
    and control point, C0 joins."""
    rr = Rng(seed, "star/radius")
    rw = Rng(seed, "star/weight")
    m = 3 * n_curves
    th = 2 * math.pi * np.arange(m) / m
    rad = 1.0 + 0.3 * rr.uniform(m, -1.0, 1.0)
    pts = np.stack([rad * np.cos(th), rad * np.sin(th)], axis=1)
    wts = rw.uniform((n_curves, 4), 0.5, 2.0)
    curves = []
    for i in range(n_curves):
        idx = [(3 * i + k) % m for k in range(4)]
        curves.append((pts[idx], wts[i]))
    return Curves2D.from_list(curves)


def config1(seed=1, n_query=4096):
    """2D plain FP64 case: star loop of 64 rational cubics, 4096 queries
    uniform in the control bbox enlarged by 10%."""
    curves = star_loop(seed, 64)
    lo, hi = curves.bbox()
    q = bbox_queries_uniform(Rng(seed, "cfg1/query"), lo, hi, n_query, 1.1)
    return curves, q


def overlapping_polygons(k, sides=15, seed=8):
    """``k`` closed, nearly overlapping regular polygons of ``sides`` linear
    edges (the overlap stress case of Sec. 4.3, Fig. overlap_demo):
    polygon j is the unit polygon rotated by a seeded angle in [0, 0.02) rad
    and scaled by 1 + U(0, 0.01), all counter-clockwise, so the winding number
    reaches k where all of them overlap."""
    rng = Rng(seed, "overlap")
    rot = rng.uniform(k, 0.0, 0.02)
    scl = 1.0 + rng.uniform(k, 0.0, 0.01)
    curves = []
    for j in range(k):
        th = rot[j] + 2 * math.pi * np.arange(sides + 1) / sides
        pts = scl[j] * np.stack([np.cos(th), np.sin(th)], axis=1)
        pts[-1] = pts[0]
        for e in range(sides):
            curves.append((pts[e:e + 2], np.ones(2)))
    return Curves2D.from_list(curves)


def svg_like(seed=2, n_groups=50, loops_per_group=4, curves_per_loop=100, delete_frac=0.05):
    """SVG-like drawing: groups of concentric jittered loops (nested and
    overlapping), degree 2-3 rational curves, weights U(0.5, 2), loops CCW with
    probability 0.8, then a seeded fraction of curves deleted (non-watertight)."""
    rg = Rng(seed, "svg/group")
    rj = Rng(seed, "svg/jitter")
    rw = Rng(seed, "svg/weight")
    rd = Rng(seed, "svg/degree")
    ro = Rng(seed, "svg/orient")
    ring_scale = [1.0, 0.75, 0.5, 0.3, 0.2, 0.12][:loops_per_group]
    curves = []
    centres = rg.uniform((n_groups, 2))
    rhos = np.exp(rg.uniform(n_groups, math.log(0.05), math.log(0.35)))
    for g in range(n_groups):
        for ring in ring_scale:
            r0 = rhos[g] * ring
            m = curves_per_loop
            degs = rd.integers(m, 2, 3)
            ccw = ro.uniform(1)[0] < 0.8
            # join points
            th_j = 2 * math.pi * np.arange(m + 1) / m
            rad_j = r0 * (1.0 + 0.3 * rj.uniform(m, -1.0, 1.0))
            rad_j = np.append(rad_j, rad_j[0])
            loop = []
            for k in range(m):
                d = int(degs[k])
                ts = np.linspace(0.0, 1.0, d + 1)
                th = th_j[k] + ts * (th_j[k + 1] - th_j[k])
                rad = np.empty(d + 1)
                rad[0], rad[-1] = rad_j[k], rad_j[k + 1]
                if d > 1:
                    rad[1:-1] = r0 * (1.0 + 0.3 * rj.uniform(d - 1, -1.0, 1.0))
                p = np.stack([centres[g, 0] + rad * np.cos(th), centres[g, 1] + rad * np.sin(th)], axis=1)
                w = rw.uniform(d + 1, 0.5, 2.0)
                loop.append((p, w))
            if not ccw:
                loop = [(p[::-1].copy(), w[::-1].copy()) for p, w in loop[::-1]]
            curves.extend(loop)
    n = len(curves)
    n_del = int(round(delete_frac * n))
    drop = set(Rng(seed, "svg/delete").permutation(n)[:n_del].tolist())
    curves = [c for i, c in enumerate(curves) if i not in drop]
    return Curves2D.from_list(curves)


def config2(seed=2, grid=1024, n_groups=50):
    """2D SVG-like case: 200 loops (50 groups x 4), 20k curves before 5%
    deletion, queries on a grid x grid cell-centred grid over the control bbox."""
    curves = svg_like(seed, n_groups=n_groups)
    lo, hi = curves.bbox()
    return curves, grid_queries(lo, hi, (grid, grid))


# --------------------------------------------------------------------------
# 3D workloads
# --------------------------------------------------------------------------
def _revolution_net(profile, n_rev=32):
    """Biquadratic homogeneous control grid of a surface of revolution about z.

    ``profile``: list of quadratic arcs ((rho,z) points[3], weights[3]) joined
    end to end.  Returns H[n_rev*2, 2*len(profile)+1, 4] with the revolution
    (u) index first, periodic in u (index 2*n_rev wraps to 0)."""
    n_pro = len(profile)
    prof_pts = np.zeros((2 * n_pro + 1, 2))
    prof_w = np.zeros(2 * n_pro + 1)
    for k, (p, w) in enumerate(profile):
        prof_pts[2 * k:2 * k + 3] = p
        prof_w[2 * k:2 * k + 3] = w
    rev_pts = np.zeros((2 * n_rev, 2))
    rev_w = np.zeros(2 * n_rev)
    step = 2 * math.pi / n_rev
    for k in range(n_rev):
        p, w = arc_quadratic((0.0, 0.0), 1.0, k * step, (k + 1) * step)
        rev_pts[2 * k:2 * k + 2] = p[:2]
        rev_w[2 * k:2 * k + 2] = w[:2]
    nu, nv = 2 * n_rev, 2 * n_pro + 1
    eu = np.zeros((nu, nv, 3))
    eu[:, :, 0] = rev_pts[:, None, 0] * prof_pts[None, :, 0]
    eu[:, :, 1] = rev_pts[:, None, 1] * prof_pts[None, :, 0]
    eu[:, :, 2] = prof_pts[None, :, 1]
    w = rev_w[:, None] * prof_w[None, :]
    return eu, w


def _body_patches(kind, n_pro, n_rev, rng_disp, disp, center, scale, rng_w=None, wlo=1.0, whi=1.0):
    """Closed body (sphere or torus) as n_pro x n_rev rational bicubic patches,
    outward oriented (S_u x S_v points out).  Distinct control points are
    displaced by disp*U(-1,1)^3 and weights scaled by U(wlo, whi), shared
    points identically, so the body stays watertight."""
    if kind == "sphere":
        R = 1.0
        step = math.pi / n_pro
        profile = []
        for k in range(n_pro):
            a0, a1 = -math.pi / 2 + k * step, -math.pi / 2 + (k + 1) * step
            profile.append(arc_quadratic((0.0, 0.0), R, a0, a1))
        periodic_v = False
    elif kind == "torus":
        R, r = 0.75, 0.3
        step = 2 * math.pi / n_pro
        profile = [arc_quadratic((R, 0.0), r, k * step, (k + 1) * step) for k in range(n_pro)]
        periodic_v = True
    else:
        raise ValueError(kind)
    eu, w = _revolution_net(profile, n_rev)
    nu, nv = eu.shape[0], eu.shape[1]
    if periodic_v:
        eu = eu[:, :-1]
        w = w[:, :-1]
        nv -= 1
    # distinct-point perturbation (poles of the sphere are one point each)
    d = disp * rng_disp.uniform((nu, nv, 3), -1.0, 1.0)
    ws = rng_w.uniform((nu, nv), wlo, whi) if rng_w is not None else np.ones((nu, nv))
    if kind == "sphere":
        d[:, 0] = d[0, 0]
        d[:, -1] = d[0, -1]
        ws[:, 0] = ws[0, 0]
        ws[:, -1] = ws[0, -1]
    eu = eu + d
    w = w * ws
    eu = np.asarray(center, np.float64) + scale * eu
    patches = []
    for i in range(n_rev):
        for j in range(n_pro):
            iu = [(2 * i + a) % nu for a in range(3)]
            jv = [(2 * j + b) % nv for b in range(3)] if periodic_v else [2 * j + b for b in range(3)]
            e = eu[np.ix_(iu, jv)]
            ww = w[np.ix_(iu, jv)]
            h = np.concatenate([e * ww[..., None], ww[..., None]], axis=2)   # 3x3x4
            h = elevate_homogeneous(elevate_homogeneous(h, 0), 1)             # 4x4x4
            patches.append((h[..., :3] / h[..., 3:4], h[..., 3]))
    return patches


def square_trim():
    """The CCW outer boundary of [0,1]^2 as four degree-1 curves."""
    c = [(0, 0), (1, 0), (1, 1), (0, 1), (0, 0)]
    return [(np.array([c[k], c[k + 1]], np.float64), np.ones(2)) for k in range(4)]


def circle_trim(center, radius, ccw=False):
    """Circle of four exact rational quadratic arcs in (u, v)."""
    return circle_curves(center, radius, 4, ccw=ccw, degree=2)


def bodies(seed, specs, n_pro=16, n_rev=32, disp=0.02, wlo=1.0, whi=1.0):
    """``specs``: list of (kind, center, scale).  Returns the list of
    (cp_xyz[4,4,3], cp_w[4,4]) patches, body by body."""
    out = []
    for b, (kind, center, scale) in enumerate(specs):
        rd = Rng(seed, f"body{b}/disp")
        rw = Rng(seed, f"body{b}/weight")
        out.extend(_body_patches(kind, n_pro, n_rev, rd, disp * scale, center, scale, rw, wlo, whi))
    return out


def _disjoint_holes(rng: Rng, count, rlo, rhi, margin=0.03, tries=200):
    holes = []
    for _ in range(count):
        for _t in range(tries):
            r = rng.uniform(1, rlo, rhi)[0]
            c = rng.uniform(2, r + margin, 1.0 - r - margin)
            if all(np.hypot(*(c - c2)) > r + r2 + margin for c2, r2 in holes):
                holes.append((c, r))
                break
    return holes


def config3(seed=3, grid=128, hole_frac=0.3):
    """3D FP64 case: 4 spheres + 4 tori on a 2x2x2 lattice (spacing 2.5),
    16x32 rational bicubic patches each, 30% of patches with one CW circular
    hole; queries on a grid^3 cell-centred grid over the bbox enlarged 10%."""
    specs = []
    for k in range(8):
        pos = np.array([(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1], np.float64) * 2.5
        specs.append(("sphere" if k % 2 == 0 else "torus", pos, 1.0))
    raw = bodies(seed, specs)
    rt = Rng(seed, "cfg3/trim")
    sel = rt.uniform(len(raw)) < hole_frac
    rh = Rng(seed, "cfg3/hole")
    patches = []
    for i, (cp, w) in enumerate(raw):
        trims = []
        if sel[i]:
            c = rh.uniform(2, 0.3, 0.7)
            r = rh.uniform(1, 0.1, 0.25)[0]
            trims = square_trim() + circle_trim(c, r, ccw=False)
        patches.append((cp, w, trims))
    P = Patches3D.from_list(patches)
    lo, hi = P.bbox()
    c, h = 0.5 * (lo + hi), 0.55 * (hi - lo)
    q = grid_queries(c - h, c + h, (grid, grid, grid)) if grid else np.zeros((0, 3))
    return P, q


def eval_patch(cp_xyz, cp_w, u, v):
    """Point and unit normal of a rational bicubic at parameters (u, v)
    (vectorised over u, v).  Used only to place near-surface queries."""
    cp = np.asarray(cp_xyz, np.float64).reshape(4, 4, 3)
    w = np.asarray(cp_w, np.float64).reshape(4, 4)
    h = np.concatenate([cp * w[..., None], w[..., None]], axis=2)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)

    def bern(t):
        s = 1 - t
        return np.stack([s ** 3, 3 * s * s * t, 3 * s * t * t, t ** 3], axis=-1)

    def dbern(t):
        s = 1 - t
        return np.stack([-3 * s * s, 3 * s * s - 6 * s * t, 6 * s * t - 3 * t * t, 3 * t * t], axis=-1)

    bu, bv, du, dv = bern(u), bern(v), dbern(u), dbern(v)
    H = np.einsum("...i,...j,ijk->...k", bu, bv, h)
    Hu = np.einsum("...i,...j,ijk->...k", du, bv, h)
    Hv = np.einsum("...i,...j,ijk->...k", bu, dv, h)
    W = H[..., 3:4]
    S = H[..., :3] / W
    Su = (Hu[..., :3] * W - H[..., :3] * Hu[..., 3:4]) / (W * W)
    Sv = (Hv[..., :3] * W - H[..., :3] * Hv[..., 3:4]) / (W * W)
    n = np.cross(Su, Sv)
    nn = np.linalg.norm(n, axis=-1, keepdims=True)
    return S, n / np.where(nn > 0, nn, 1.0), nn[..., 0]


def cad_assembly(seed=4, n_bodies=39, box=12.0, holes=(1, 3), hole_r=(0.05, 0.15)):
    """CAD-like assembly: perturbed spheres/tori with scale U(0.5, 2) at
    positions U([0, box]^3), control weights scaled by U(0.7, 1.5); every patch
    has the CCW square plus 1-3 disjoint CW circular holes."""
    rb = Rng(seed, "cad/body")
    specs = []
    for b in range(n_bodies):
        kind = "sphere" if rb.uniform(1)[0] < 0.5 else "torus"
        scale = rb.uniform(1, 0.5, 2.0)[0]
        pos = rb.uniform(3, 0.0, box)
        specs.append((kind, pos, scale))
    raw = bodies(seed, specs, wlo=0.7, whi=1.5)
    rh = Rng(seed, "cad/hole")
    patches = []
    for cp, w in raw:
        k = int(rh.integers(1, holes[0], holes[1])[0])
        trims = square_trim()
        for c, r in _disjoint_holes(rh, k, hole_r[0], hole_r[1]):
            trims += circle_trim(c, r, ccw=False)
        patches.append((cp, w, trims))
    return Patches3D.from_list(patches)


def _eval_batch(cps, ws, u, v):
    """Vectorised eval_patch over (patch control nets, u, v) triples."""
    h = np.concatenate([cps * ws[..., None], ws[..., None]], axis=-1)      # m,4,4,4

    def bern(t):
        s = 1 - t
        return np.stack([s ** 3, 3 * s * s * t, 3 * s * t * t, t ** 3], -1)

    def dbern(t):
        s = 1 - t
        return np.stack([-3 * s * s, 3 * s * s - 6 * s * t, 6 * s * t - 3 * t * t, 3 * t * t], -1)
    bu, bv, du, dv = bern(u), bern(v), dbern(u), dbern(v)
    H = np.einsum("mi,mj,mijk->mk", bu, bv, h)
    Hu = np.einsum("mi,mj,mijk->mk", du, bv, h)
    Hv = np.einsum("mi,mj,mijk->mk", bu, dv, h)
    W = H[:, 3:4]
    S = H[:, :3] / W
    Su = (Hu[:, :3] * W - H[:, :3] * Hu[:, 3:4]) / (W * W)
    Sv = (Hv[:, :3] * W - H[:, :3] * Hv[:, 3:4]) / (W * W)
    n = np.cross(Su, Sv)
    nn = np.linalg.norm(n, axis=1, keepdims=True)
    return S, n / np.where(nn > 0, nn, 1.0), nn[:, 0]


def near_surface_queries(P: Patches3D, rng: Rng, n, t_max=1e-2, chunk=65536):
    """Points S(u,v) + t*n(u,v): patch chosen area-weighted, (u,v) uniform and
    rejected inside the circular trim holes, t ~ U(-t_max, t_max)."""
    cps = P.cp_xyz.reshape(-1, 4, 4, 3)
    ws = P.cp_w.reshape(-1, 4, 4)
    g = (np.arange(4) + 0.5) / 4
    gu, gv = [a.ravel() for a in np.meshgrid(g, g, indexing="ij")]
    areas = np.zeros(P.n)
    for k in range(16):
        _, _, jac = _eval_batch(cps, ws, np.full(P.n, gu[k]), np.full(P.n, gv[k]))
        areas += jac / 16
    cdf = np.cumsum(areas)
    cdf /= cdf[-1]
    # circular holes: groups of four rational quadratic arcs (middle weight != 1)
    hc = np.zeros((P.n, 3, 2))
    hr = np.zeros((P.n, 3))
    for i in range(P.n):
        arcs = [uv for uv, wt in P.trims(i) if uv.shape[0] == 3 and abs(wt[1] - 1.0) > 1e-12]
        for k in range(0, min(len(arcs), 12), 4):
            ends = np.array([a[0] for a in arcs[k:k + 4]])
            c = ends.mean(axis=0)
            hc[i, k // 4] = c
            hr[i, k // 4] = np.linalg.norm(ends[0] - c)
    out = np.empty((n, 3))
    filled = 0
    while filled < n:
        m = min(n - filled, chunk)
        pid = np.minimum(np.searchsorted(cdf, rng.uniform(m)), P.n - 1)
        u = rng.uniform(m)
        v = rng.uniform(m)
        t = rng.uniform(m, -t_max, t_max)
        d2 = (u[:, None] - hc[pid, :, 0]) ** 2 + (v[:, None] - hc[pid, :, 1]) ** 2
        keep = ~np.any(d2 < hr[pid] ** 2, axis=1)
        pid, u, v, t = pid[keep], u[keep], v[keep], t[keep]
        S, nrm, _ = _eval_batch(cps[pid], ws[pid], u, v)
        q = S + t[:, None] * nrm
        k = min(q.shape[0], n - filled)
        out[filled:filled + k] = q[:k]
        filled += k
    return out


def config4(seed=4, n_query=1_000_000, n_bodies=39):
    """3D mixed-precision case: CAD-like assembly of ~20k trimmed patches;
    half the queries within 1e-2 of the surface, half uniform in the bbox."""
    P = cad_assembly(seed, n_bodies)
    lo, hi = P.bbox()
    n_near = n_query // 2
    near = near_surface_queries(P, Rng(seed, "cfg4/near"), n_near)
    uni = bbox_queries_uniform(Rng(seed, "cfg4/uniform"), lo, hi, n_query - n_near, 1.0)
    q = np.concatenate([near, uni])
    q = q[Rng(seed, "cfg4/shuffle").permutation(q.shape[0])]
    return P, np.ascontiguousarray(q)


def serving_models(seed=5, kinds=("2d", "3d")):
    """Resident serving models: four 2D drawings (about 5k, 10k, 15k, 20k
    curves) and four 3D assemblies (4, 10, 20, 39 bodies; about 2k-20k
    patches), of the kinds asked for."""
    models = []
    if "2d" in kinds:
        for k, g in enumerate([12, 25, 38, 50]):
            models.append(("2d", svg_like(seed * 100 + k, n_groups=g)))
    if "3d" in kinds:
        for k, nb in enumerate([4, 10, 20, 39]):
            models.append(("3d", cad_assembly(seed * 100 + 10 + k, n_bodies=nb)))
    return models
