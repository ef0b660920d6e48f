"""Bezier extraction of 2D NURBS curves (host code of the C ABI, no GPU).

Pins: a B-spline evaluated by de Boor's algorithm, written out here on its
own, against the extracted Bezier segments evaluated in Bernstein form; the
exact rational-quadratic NURBS circle; polylines reproduced bit for bit; and
the winding number of an extracted circle, by the CPU oracle, equal to 1
inside and 0 outside."""
import math

import numpy as np
import pytest

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import workloads as W


def de_boor(p, U, P, t):
    """Homogeneous point of the B-spline (degree p, knots U, points P[k] =
    (w x, w y, w)) at t in [U[p], U[-p-1]]: de Boor's triangle."""
    n = len(P) - 1
    k = p
    while k < n and not (U[k] <= t < U[k + 1]):
        k += 1
    d = [np.array(P[j], dtype=float) for j in range(k - p, k + 1)]
    for r in range(1, p + 1):
        for i in range(p, r - 1, -1):
            j = k - p + i
            a = (t - U[j]) / (U[j + p + 1 - r] - U[j])
            d[i] = (1 - a) * d[i - 1] + a * d[i]
    return d[p]


def bezier_point(xy, w, s):
    """Euclidean point of a rational Bezier curve at s in [0, 1]."""
    p = len(w) - 1
    b = np.array([math.comb(p, i) * (1 - s) ** (p - i) * s ** i for i in range(p + 1)])
    h = (b * w) @ xy
    return h / (b @ w)


def homog(pts, w):
    return [np.array([wi * x, wi * y, wi]) for (x, y), wi in zip(pts, w)]


def circle_nurbs():
    s = math.sqrt(0.5)
    pts = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0)]
    w = [1, s, 1, s, 1, s, 1, s, 1]
    U = [0, 0, 0, 0.25, 0.25, 0.5, 0.5, 0.75, 0.75, 1, 1, 1]
    return (2, pts, w, U)


def random_nurbs(rng, p, n_cp):
    inner = np.sort(rng.uniform(n_cp - p - 1, 0.05, 0.95))
    # repeat a few interior knots (multiplicity up to p)
    mult = rng.integers(n_cp - p - 1, 1, 3)
    U = [0.0] * (p + 1)
    for u, m in zip(inner, mult):
        U += [float(u)] * int(min(m, p))
    U = U[:n_cp]   # keep n_cp + p + 1 knots in all
    U = U + [1.0] * (n_cp + p + 1 - len(U))
    pts = rng.uniform((n_cp, 2), -1, 1)
    w = rng.uniform(n_cp, 0.3, 3.0)
    return (p, pts, w, U)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_extraction_matches_de_boor(p):
    rng = W.Rng(70 + p, "nurbs")
    curves = [random_nurbs(rng, p, n) for n in (p + 1, p + 3, 9, 14)]
    N = W.Nurbs2D.from_list(curves)
    B = G.gwn_nurbs2d_extract(N)
    seg = 0
    for deg, pts, w, U in curves:
        P = homog(pts, w)
        spans = [k for k in range(deg, len(pts)) if U[k] < U[k + 1]]
        for k in spans:
            xy, ww = B.curve(seg)
            assert B.degree[seg] == deg and xy.shape[0] == deg + 1
            for s in np.linspace(0, 1, 7):
                t = U[k] + s * (U[k + 1] - U[k])
                h = de_boor(deg, U, P, min(t, np.nextafter(U[k + 1], -np.inf)) if s == 1 else t)
                ref = h[:2] / h[2]
                got = bezier_point(xy, ww, s)
                assert np.abs(got - ref).max() < 1e-12 * (1 + np.abs(ref).max()), (deg, k, s)
            seg += 1
    assert seg == B.n


def test_circle_is_exact():
    B = G.gwn_nurbs2d_extract(W.Nurbs2D.from_list([circle_nurbs()]))
    assert B.n == 4 and np.all(B.degree == 2)
    for i in range(4):
        xy, w = B.curve(i)
        for s in np.linspace(0, 1, 33):
            assert abs(np.linalg.norm(bezier_point(xy, w, s)) - 1) < 1e-15
        # middle weight of a quarter arc is cos(pi/4) relative to its ends
        assert abs(w[1] / w[0] - math.sqrt(0.5)) < 1e-15


def test_circle_winding_number(oracle):
    B = G.gwn_nurbs2d_extract(W.Nurbs2D.from_list([circle_nurbs()]))
    rng = W.Rng(77, "circ")
    ang = rng.uniform(64, 0, 2 * math.pi)
    rad = np.concatenate([rng.uniform(32, 0, 0.98), rng.uniform(32, 1.02, 3)])
    q = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    w = oracle.gwn2d(B, q)
    assert np.abs(w - (rad < 1)).max() < 1e-12


def test_polyline_bitwise():
    pts = np.array([[0, 0], [1, 0.5], [2, -1], [3, 0.25], [2.5, 2]])
    w = np.array([1.0, 2.0, 0.5, 1.0, 3.0])
    U = [0, 0, 0.1, 0.4, 0.7, 1, 1]
    B = G.gwn_nurbs2d_extract(W.Nurbs2D.from_list([(1, pts, w, U)]))
    assert B.n == 4
    for i in range(4):
        xy, ww = B.curve(i)
        assert np.array_equal(xy, pts[i:i + 2]) and np.array_equal(ww, w[i:i + 2])


def test_zero_length_spans_and_orientation():
    # a doubled interior knot of a quadratic gives two segments meeting at a
    # C0 joint, in the parameter order of the input
    pts = [(0, 0), (1, 1), (2, 0), (3, 1), (4, 0)]
    w = [1, 1, 1, 1, 1]
    B = G.gwn_nurbs2d_extract(W.Nurbs2D.from_list([(2, pts, w, [0, 0, 0, 0.5, 0.5, 1, 1, 1])]))
    assert B.n == 2
    assert np.array_equal(B.curve(0)[0][0], [0, 0]) and np.array_equal(B.curve(1)[0][-1], [4, 0])
    assert np.allclose(B.curve(0)[0][-1], B.curve(1)[0][0])


def test_empty_input():
    B = G.gwn_nurbs2d_extract(W.Nurbs2D.from_list([]))
    assert B.n == 0


@pytest.mark.parametrize("bad", ["degree", "knot_count", "unclamped", "decreasing", "weight", "nan", "multiplicity"])
def test_invalid_nurbs(bad):
    p, pts, w, U = circle_nurbs()
    pts, w, U = list(pts), list(w), list(U)
    if bad == "degree":
        p = 4
    if bad == "knot_count":
        U = U[:-1]
    if bad == "unclamped":
        U[0] = -0.1
    if bad == "decreasing":
        U[4], U[5] = 0.6, 0.5
    if bad == "weight":
        w[3] = 0.0
    if bad == "nan":
        pts[2] = (np.nan, 1)
    if bad == "multiplicity":
        U = [0, 0, 0, 0.5, 0.5, 0.5, 0.5, 0.75, 0.75, 1, 1, 1]
    with pytest.raises(G.GwnError) as ei:
        G.gwn_nurbs2d_extract(W.Nurbs2D.from_list([(p, pts, w, U)]))
    assert ei.value.status == G.GWN_EINVAL and G.gwn_last_error()


def test_capacity_checked():
    import ctypes
    N = W.Nurbs2D.from_list([circle_nurbs()])
    arrs = [np.ascontiguousarray(a) for a in (N.degree.astype(np.int32), N.cp_offset, N.cp_xy, N.cp_w,
                                              N.knot_offset, N.knots)]
    c = G.gwn_nurbs2d(N.n, *[ctypes.c_void_p(a.ctypes.data) for a in arrs])
    ns, npt = ctypes.c_int64(3), ctypes.c_int64(12)   # one segment short
    deg, off = np.zeros(4, np.int32), np.zeros(5, np.int64)
    xy, w = np.zeros((12, 2)), np.zeros(12)
    st = G.lib().gwn_nurbs2d_extract(ctypes.byref(c), ctypes.byref(ns), ctypes.byref(npt),
                                     *[ctypes.c_void_p(a.ctypes.data) for a in (deg, off, xy, w)])
    assert st == G.GWN_EINVAL and "capacity" in G.gwn_last_error()
