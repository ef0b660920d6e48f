"""Pins of the 2D CPU oracle against facts fixed by the mathematics.

Each test targets a way the oracle could be wrong: a wrong sign or swapped
operand in the angle integrand (segment closed form, orientation reversal),
a mishandled weight (Moebius reweighting, degree elevation), a broken near
field (circle interior/exterior, jump condition, dense brute force), a broken
boundary rule (on-curve 0.5, square corner 0.25), a broken hull test (star
containment by exact crossing counts).
"""
import math

import numpy as np
import pytest

from paper_2605_19200_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")


def seg_angle(a, b, q):
    ax, ay = a[0] - q[0], a[1] - q[1]
    bx, by = b[0] - q[0], b[1] - q[1]
    return math.atan2(ax * by - ay * bx, ax * bx + ay * by) / (2 * math.pi)


def hom(p, w):
    return np.concatenate([np.asarray(p) * np.asarray(w)[:, None], np.asarray(w)[:, None]], axis=1)


def dehom(h):
    return h[:, :2] / h[:, 2:3], h[:, 2].copy()


def split_at(p, w, t):
    """de Casteljau split of a rational Bezier (homogeneous) at t."""
    h = hom(p, w)
    left, right = [h[0]], [h[-1]]
    cur = h
    while cur.shape[0] > 1:
        cur = (1 - t) * cur[:-1] + t * cur[1:]
        left.append(cur[0])
        right.append(cur[-1])
    return dehom(np.array(left)), dehom(np.array(right[::-1]))


def test_gl_nodes_exact_for_polynomials(oracle):
    x, w = oracle.gl_nodes()
    for k in range(20):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14


def test_segment_closed_form(oracle):
    rng = W.Rng(11, "seg")
    for _ in range(40):
        a, b, q = rng.uniform(2, -1, 1), rng.uniform(2, -1, 1), rng.uniform(2, -1, 1)
        C = W.Curves2D.from_list([(np.stack([a, b]), np.ones(2))])
        assert abs(oracle.gwn2d(C, q[None])[0] - seg_angle(a, b, q)) < 1e-15


def test_straight_cubic_equals_segment(oracle):
    a, b = np.array([-0.3, 0.2]), np.array([0.9, -0.4])
    p = np.stack([a, a + (b - a) / 3, a + 2 * (b - a) / 3, b])
    C = W.Curves2D.from_list([(p, np.array([1.0, 0.7, 1.6, 1.2]))])
    rng = W.Rng(12, "q")
    qs = rng.uniform((50, 2), -1, 1)
    got = oracle.gwn2d(C, qs)
    ref = np.array([seg_angle(a, b, q) for q in qs])
    assert np.abs(got - ref).max() < 1e-14


def test_circle_inside_outside_boundary(oracle):
    circ = W.Curves2D.from_list(W.circle_curves((0.2, -0.1), 0.8))
    rng = W.Rng(13, "circ")
    r = rng.uniform(200, 0, 0.99 * 0.8)
    th = rng.uniform(200, 0, 2 * math.pi)
    inside = np.stack([0.2 + r * np.cos(th), -0.1 + r * np.sin(th)], 1)
    r = rng.uniform(200, 1.01 * 0.8, 3.0)
    outside = np.stack([0.2 + r * np.cos(th), -0.1 + r * np.sin(th)], 1)
    assert np.abs(oracle.gwn2d(circ, inside) - 1).max() < 1e-13
    assert np.abs(oracle.gwn2d(circ, outside)).max() < 1e-13
    on = np.stack([0.2 + 0.8 * np.cos(th[:20]), -0.1 + 0.8 * np.sin(th[:20])], 1)
    assert np.abs(oracle.gwn2d(circ, on) - 0.5).max() < 1e-8


def test_square_corner_and_edge(oracle):
    sq = W.Curves2D.from_list([(p, w) for p, w in W.square_trim()])
    q = np.array([[0, 0], [1, 1], [0.5, 0], [1, 0.3], [0.5, 0.5], [1.5, 0.5]], float)
    got = oracle.gwn2d(sq, q)
    assert np.allclose(got, [0.25, 0.25, 0.5, 0.5, 1.0, 0.0], atol=1e-14)


def _crossings(curves, q):
    """Number of crossings of the segment [0, q] with the curves: roots of the
    cubic H_x(t) q_y - H_y(t) q_x on [0, 1] whose point lies on the segment."""
    n = 0
    for p, w in curves.to_list():
        h = hom(p, w)
        d = h.shape[0] - 1
        # power-basis coefficients of sum_i B_i(t) c_i
        c = h[:, 0] * q[1] - h[:, 1] * q[0]
        poly = np.zeros(d + 1)
        for i in range(d + 1):
            # B_i = C(d,i) t^i (1-t)^(d-i)
            bi = np.poly1d([1.0])
            for _ in range(i):
                bi = bi * np.poly1d([1.0, 0.0])
            for _ in range(d - i):
                bi = bi * np.poly1d([-1.0, 1.0])
            poly = np.polyadd(poly, math.comb(d, i) * c[i] * bi.coeffs)
        for t in np.roots(poly):
            if abs(t.imag) > 1e-9 or not (0 <= t.real <= 1):
                continue
            t = t.real
            B = np.array([math.comb(d, i) * t ** i * (1 - t) ** (d - i) for i in range(d + 1)])
            pt = (B @ h[:, :2]) / (B @ h[:, 2])
            s = pt @ q / (q @ q)
            if 0 <= s <= 1:
                n += 1
    return n


def test_star_loop_containment_by_crossings(oracle):
    curves, q = W.config1()
    q = q[:300]
    w = oracle.gwn2d(curves, q)
    assert np.abs(w - np.round(w)).max() < 1e-12
    for k in range(q.shape[0]):
        inside = _crossings(curves, q[k]) % 2 == 0
        assert inside == (w[k] >= 0.5), k


def _dense_angle(p, wts, q, panels=4000):
    """Composite 5-point Gauss-Legendre of d(theta)/dt over [0,1] in numpy."""
    x5, w5 = np.polynomial.legendre.leggauss(5)
    a = np.arange(panels) / panels
    t = (a[:, None] + (x5[None, :] + 1) / (2 * panels)).reshape(-1)
    ww = np.tile(w5 / (2 * panels), panels)
    h = hom(p, wts)
    d = h.shape[0] - 1
    B = np.stack([math.comb(d, i) * t ** i * (1 - t) ** (d - i) for i in range(d + 1)], 1)
    hd = d * (h[1:] - h[:-1])
    Bd = np.stack([math.comb(d - 1, i) * t ** i * (1 - t) ** (d - 1 - i) for i in range(d)], 1)
    H, Hd = B @ h, Bd @ hd
    A = H[:, :2] - np.outer(H[:, 2], q)
    Ad = Hd[:, :2] - np.outer(Hd[:, 2], q)
    f = (A[:, 0] * Ad[:, 1] - A[:, 1] * Ad[:, 0]) / (A ** 2).sum(1)
    return (ww * f).sum() / (2 * math.pi)


def test_dense_bruteforce_near_field(oracle):
    rng = W.Rng(14, "brute")
    for trial in range(6):
        d = 2 + trial % 2
        p = rng.uniform((d + 1, 2), -1, 1)
        wt = rng.uniform(d + 1, 0.5, 2.0)
        C = W.Curves2D.from_list([(p, wt)])
        # points inside the control hull region but at distance >= 0.05
        qs = []
        while len(qs) < 5:
            cand = rng.uniform(2, -1, 1)
            tt = np.linspace(0, 1, 2001)
            B = np.stack([math.comb(d, i) * tt ** i * (1 - tt) ** (d - i) for i in range(d + 1)], 1)
            H = B @ hom(p, wt)
            pts = H[:, :2] / H[:, 2:3]
            if np.min(np.hypot(*(pts - cand).T)) > 0.05:
                qs.append(cand)
        got = oracle.gwn2d(C, np.array(qs))
        ref = np.array([_dense_angle(p, wt, q) for q in qs])
        assert np.abs(got - ref).max() < 1e-11


def test_hairpin_curve_against_dense(oracle):
    """A sharply turning quadratic from the SVG-like drawing, with q inside its
    hull but away from the turn: the angle integrand has a feature far from
    the closest point that a coarse adaptive start can miss."""
    p = np.array([[0.38020299, 0.93432087], [0.26739145, 0.95485183], [0.37813275, 0.92541035]])
    wt = np.array([0.62127915, 1.23228282, 0.94014809])
    q = np.array([0.34729583, 0.93765536])
    C = W.Curves2D.from_list([(p, wt)])
    ref = _dense_angle(p, wt, q, panels=20000)
    assert abs(oracle.gwn2d(C, q[None])[0] - ref) < 1e-12


def test_orientation_elevation_reweighting_subdivision(oracle):
    curves, q = W.config1()
    curves = curves.subset(range(0, 20))
    q = q[:200]
    base = oracle.gwn2d(curves, q)
    rev = W.Curves2D.from_list([(p[::-1], w[::-1]) for p, w in curves.to_list()])
    assert np.abs(oracle.gwn2d(rev, q) + base).max() < 1e-12
    # Moebius reweighting w_i -> w_i c^i leaves the curve unchanged
    rw = W.Curves2D.from_list([(p, w * 1.7 ** np.arange(len(w))) for p, w in curves.to_list()])
    assert np.abs(oracle.gwn2d(rw, q) - base).max() < 1e-12
    # degree 3 curves elevated cannot go higher; use quadratic arcs -> cubic
    arcs2 = W.Curves2D.from_list(W.circle_curves((0.1, 0.0), 0.9, 5, degree=2))
    arcs3 = W.Curves2D.from_list(W.circle_curves((0.1, 0.0), 0.9, 5, degree=3))
    assert np.abs(oracle.gwn2d(arcs2, q) - oracle.gwn2d(arcs3, q)).max() < 1e-12
    # subdivision at t = 0.37 (Sec. 3.2: subdivision leaves the GWN unchanged)
    parts = []
    for p, w in curves.to_list():
        (pl, wl), (pr, wr) = split_at(p, w, 0.37)
        parts += [(pl, wl), (pr, wr)]
    assert np.abs(oracle.gwn2d(W.Curves2D.from_list(parts), q) - base).max() < 1e-12


def test_additivity_and_jump(oracle):
    a = W.Curves2D.from_list(W.circle_curves((0, 0), 1.0))
    b = W.Curves2D.from_list(W.circle_curves((0.5, 0.2), 0.7, 3, ccw=False))
    q = W.Rng(15, "add").uniform((100, 2), -2, 2)
    assert np.abs(oracle.gwn2d(a.concat(b), q) - oracle.gwn2d(a, q) - oracle.gwn2d(b, q)).max() < 1e-13
    # jump of exactly 1 across a closed boundary (approached from both sides)
    star, _ = W.config1()
    eps = 1e-7
    for k in range(0, 64, 8):
        p, w = star.curve(k)
        h = hom(p, w)
        t = 0.41
        B = np.array([math.comb(3, i) * t ** i * (1 - t) ** (3 - i) for i in range(4)])
        dB = np.array([3 * ((i * t ** (i - 1) if i else 0) * (1 - t) ** (3 - i)
                            - (3 - i) * t ** i * ((1 - t) ** (2 - i) if i < 3 else 0)) * math.comb(3, i) / 3
                       for i in range(4)])
        H, Hd = B @ h, dB @ h
        pt = H[:2] / H[2]
        tan = (Hd[:2] * H[2] - H[:2] * Hd[2])
        nrm = np.array([tan[1], -tan[0]]) / np.linalg.norm(tan)
        inner, outer = oracle.gwn2d(star, np.stack([pt - eps * nrm, pt + eps * nrm]))
        assert abs((inner - outer) - 1.0) < 1e-6
