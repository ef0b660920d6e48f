"""Bezier extraction of trimmed NURBS surfaces (host code of the C ABI, no
GPU).

Pins: a NURBS surface evaluated from its definition (Cox-de Boor basis
functions, written out here on their own) against the extracted rational
bicubic patches evaluated in Bernstein form, for every degree pair and knot
multiplicity; a one-span bicubic surface reproduced exactly; the visible
area of a face with a circular hole cut across knot lines equal to the
square's minus the disk's; and, by the CPU oracle, the winding number of a
closed cube built from NURBS faces -- one of them holed, the hole closed by
the same surface trimmed to the disk -- equal to 1 inside and 0 outside."""
import math

import numpy as np
import pytest

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import workloads as W


def basis(U, p, i, t):
    """N_(i,p)(t) by the Cox-de Boor recursion; the last non-empty span is
    closed on the right so that t = U[-1] belongs to it."""
    last = max(k for k in range(len(U) - 1) if U[k] < U[k + 1])
    if p == 0:
        return 1.0 if (U[i] <= t < U[i + 1]) or (i == last and t == U[i + 1]) else 0.0
    a = 0.0 if U[i + p] == U[i] else (t - U[i]) / (U[i + p] - U[i]) * basis(U, p - 1, i, t)
    b = 0.0 if U[i + p + 1] == U[i + 1] else (U[i + p + 1] - t) / (U[i + p + 1] - U[i + 1]) * basis(U, p - 1, i + 1, t)
    return a + b


def surface_point(pu, pv, cp, w, U, V, u, v):
    """S(u, v) = sum N_i(u) N_j(v) w_ij P_ij / sum N_i(u) N_j(v) w_ij."""
    Nu = np.array([basis(U, pu, i, u) for i in range(cp.shape[0])])
    Nv = np.array([basis(V, pv, j, v) for j in range(cp.shape[1])])
    B = np.outer(Nu, Nv) * w
    return np.einsum("ij,ijk->k", B, cp) / B.sum()


def patch_point(cp, w, s, t):
    """Rational bicubic Bezier patch (cp[16, 3], w[16], a indexes u) at (s, t)."""
    bs = np.array([math.comb(3, i) * (1 - s) ** (3 - i) * s ** i for i in range(4)])
    bt = np.array([math.comb(3, i) * (1 - t) ** (3 - i) * t ** i for i in range(4)])
    B = np.outer(bs, bt).reshape(16) * w
    return B @ cp / B.sum()


def clamped(p, inner, lo=0.0, hi=1.0):
    return np.array([lo] * (p + 1) + list(inner) + [hi] * (p + 1))


def spans(U, p, n):
    return [(U[k], U[k + 1]) for k in range(p, n) if U[k] < U[k + 1]]


def random_surface(rng, pu, pv, nu, nv, inner_u, inner_v, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    # inner knots given as fractions of the domain
    U = clamped(pu, [lo[0] + t * (hi[0] - lo[0]) for t in inner_u], lo[0], hi[0])
    V = clamped(pv, [lo[1] + t * (hi[1] - lo[1]) for t in inner_v], lo[1], hi[1])
    assert len(U) == nu + pu + 1 and len(V) == nv + pv + 1
    cp = rng.uniform(nu * nv * 3, -1.0, 1.0).reshape(nu, nv, 3)
    w = rng.uniform(nu * nv, 0.4, 2.5).reshape(nu, nv)
    return cp, w, U, V


@pytest.mark.parametrize("pu,pv", [(1, 1), (1, 3), (2, 2), (3, 1), (3, 3), (2, 3)])
def test_extraction_matches_definition(pu, pv):
    rng = W.Rng(100 + 10 * pu + pv, "nurbs3d")
    # a double knot where the surface stays continuous across it
    inner_u = [0.2, 0.45, 0.45, 0.8] if pu > 1 else [0.2, 0.45, 0.8]
    inner_v = [0.3, 0.6] + ([0.6] if pv > 2 else [])
    nu, nv = len(inner_u) + pu + 1, len(inner_v) + pv + 1
    cp, w, U, V = random_surface(rng, pu, pv, nu, nv, inner_u, inner_v, lo=(-1.0, 2.0), hi=(3.0, 2.5))
    out = G.gwn_nurbs3d_extract(W.Nurbs3D.from_list([(pu, pv, cp, w, U, V, [])]))
    su, sv = spans(U, pu, nu), spans(V, pv, nv)
    assert out.n == len(su) * len(sv) and out.trim_offset[-1] == 0
    ss = [0.0, 0.3, 0.71, 1.0]
    for a, (u0, u1) in enumerate(su):
        for b, (v0, v1) in enumerate(sv):
            k = a * len(sv) + b
            for s in ss:
                for t in ss:
                    want = surface_point(pu, pv, cp, w, U, V, u0 + s * (u1 - u0), v0 + t * (v1 - v0))
                    got = patch_point(out.cp_xyz[k], out.cp_w[k], s, t)
                    assert np.abs(got - want).max() < 1e-12, (a, b, s, t)


def test_single_bicubic_span_is_the_patch():
    rng = W.Rng(7, "bez")
    cp = rng.uniform(48, -1, 1).reshape(4, 4, 3)
    w = rng.uniform(16, 0.5, 2.0).reshape(4, 4)
    U = clamped(3, [])
    out = G.gwn_nurbs3d_extract(W.Nurbs3D.from_list([(3, 3, cp, w, U, U, [])]))
    assert out.n == 1
    assert np.allclose(out.cp_xyz[0], cp.reshape(16, 3), rtol=0, atol=1e-15)
    assert np.allclose(out.cp_w[0], w.reshape(16), rtol=0, atol=1e-15)


# trim curves in the surface's domain: a closed polyline (degree 1) and the
# exact rational-quadratic NURBS circle
def polyline(pts):
    pts = np.asarray(pts, float)
    n = len(pts)
    return (1, pts, np.ones(n), [0.0] + list(range(n)) + [n - 1.0])


def circle(cx, cy, r, ccw=True):
    h = math.sqrt(0.5)
    P = np.array([[1, 0], [1, 1], [0, 1], [-1, 1], [-1, 0], [-1, -1], [0, -1], [1, -1], [1, 0]], float) * r + [cx, cy]
    wt = np.array([1, h, 1, h, 1, h, 1, h, 1])
    if not ccw:
        P, wt = P[::-1].copy(), wt[::-1].copy()
    return (2, P, wt, [0, 0, 0, .25, .25, .5, .5, .75, .75, 1, 1, 1])


def loop_area(trims):
    """Area enclosed by closed rational trim curves (Green: 1/2 int u dv - v du),
    by 24-point Gauss-Legendre quadrature per curve."""
    x, gw = np.polynomial.legendre.leggauss(24)
    t, gw = 0.5 * (x + 1), 0.5 * gw
    area = 0.0
    for uv, w in trims:
        d = len(w) - 1
        B = np.array([[math.comb(d, i) * (1 - s) ** (d - i) * s ** i for i in range(d + 1)] for s in t])
        dB = np.array([[math.comb(d, i) * (i * s ** max(i - 1, 0) * (1 - s) ** (d - i)
                                           - (d - i) * s ** i * (1 - s) ** max(d - i - 1, 0)) for i in range(d + 1)]
                       for s in t])
        hw, dhw = B @ w, dB @ w
        h, dh = B @ (uv * w[:, None]), dB @ (uv * w[:, None])
        p = h / hw[:, None]
        dp = (dh * hw[:, None] - h * dhw[:, None]) / hw[:, None] ** 2
        area += 0.5 * np.sum(gw * (p[:, 0] * dp[:, 1] - p[:, 1] * dp[:, 0]))
    return area


def planar_face(origin, e1, e2, pu, pv, inner_u, inner_v, lo, hi, weights=None, rng=None):
    """A NURBS surface on the unit square origin + x e1 + y e2 whose
    parametrisation is affine when the weights are 1 (control points at the
    Greville abscissae): (u, v) in [lo, hi] -> ((u - lo_u) / L_u, ...)."""
    U, V = clamped(pu, inner_u, lo[0], hi[0]), clamped(pv, inner_v, lo[1], hi[1])
    nu, nv = len(U) - pu - 1, len(V) - pv - 1
    gu = np.array([U[i + 1:i + pu + 1].mean() for i in range(nu)])
    gv = np.array([V[j + 1:j + pv + 1].mean() for j in range(nv)])
    x = (gu - lo[0]) / (hi[0] - lo[0])
    y = (gv - lo[1]) / (hi[1] - lo[1])
    cp = np.asarray(origin, float) + x[:, None, None] * np.asarray(e1, float) + y[None, :, None] * np.asarray(e2, float)
    w = np.ones((nu, nv)) if weights is None else rng.uniform(nu * nv, *weights).reshape(nu, nv)
    return pu, pv, cp, w, U, V


def holed_face(ccw_hole=False, hole_only=False, weights=None, rng=None):
    lo, hi = (1.0, -2.0), (3.0, 2.0)
    f = planar_face((0, 0, 1), (1, 0, 0), (0, 1, 0), 3, 2, [1.5, 2.1, 2.6], [-1.0, 0.3, 0.3, 1.1], lo, hi,
                    weights, rng)
    hole = circle(2.0, 0.05, 0.42, ccw=hole_only)
    outer = polyline([[1, -2], [3, -2], [3, 2], [1, 2], [1, -2]])
    return (*f, [hole] if hole_only else [outer, hole])


def test_holed_face_area_and_span_classes():
    """The holed top face of the cube: visible area = 1 - pi r'^2 (r' the hole
    radius in face units), spans away from the circle come back untrimmed,
    spans inside it are dropped; the plug (the same surface trimmed to the
    disk) has the disk's area."""
    face = holed_face()
    out = G.gwn_nurbs3d_extract(W.Nurbs3D.from_list([face]))
    n_span = 4 * 4
    area, untrimmed = 0.0, 0
    for k in range(out.n):
        c = out.cp_xyz[k].reshape(4, 4, 3)
        jac = abs(np.cross(c[3, 0] - c[0, 0], c[0, 3] - c[0, 0])[2])
        tr = out.trims(k)
        untrimmed += len(tr) == 0
        area += jac * (1.0 if not tr else loop_area(tr))
    rx, ry = 0.42 / 2.0, 0.42 / 4.0     # the circle's semi-axes in face units
    assert abs(area - (1.0 - math.pi * rx * ry)) < 1e-12
    assert out.n <= n_span and untrimmed >= 6
    plug = G.gwn_nurbs3d_extract(W.Nurbs3D.from_list([holed_face(hole_only=True)]))
    parea = sum(abs(np.cross(plug.cp_xyz[k].reshape(4, 4, 3)[3, 0] - plug.cp_xyz[k].reshape(4, 4, 3)[0, 0],
                             plug.cp_xyz[k].reshape(4, 4, 3)[0, 3] - plug.cp_xyz[k].reshape(4, 4, 3)[0, 0])[2])
                * loop_area(plug.trims(k)) for k in range(plug.n))
    assert abs(parea - math.pi * rx * ry) < 1e-12
    assert plug.n < n_span and all(len(plug.trims(k)) > 0 for k in range(plug.n))


def nurbs_cube(rng):
    """The unit cube from six NURBS faces of mixed degrees, knots and
    weights, normals S_u x S_v outward; the top face holed and plugged."""
    faces = [
        planar_face((0, 0, 0), (0, 0, 1), (0, 1, 0), 1, 1, [0.4], [0.5, 0.7], (0, 0), (1, 1)),        # x = 0
        planar_face((1, 0, 0), (0, 1, 0), (0, 0, 1), 2, 3, [0.3, 0.3], [0.6], (0, 0), (2, 1), (0.5, 2.0), rng),
        planar_face((0, 0, 0), (1, 0, 0), (0, 0, 1), 3, 1, [0.25, 0.5], [], (0, 0), (1, 1), (0.7, 1.5), rng),
        planar_face((0, 1, 0), (0, 0, 1), (1, 0, 0), 2, 2, [], [0.45], (-1, -1), (1, 1)),              # y = 1
        planar_face((0, 0, 0), (0, 1, 0), (1, 0, 0), 3, 3, [0.5], [0.2, 0.8], (0, 0), (1, 1), (0.5, 2.0), rng),
    ]
    faces = [(*f, []) for f in faces]
    faces.append(holed_face(weights=(0.6, 1.6), rng=rng))
    # the plug must be the same surface as the holed face: reuse its net
    plug = list(faces[-1])
    plug[6] = [circle(2.0, 0.05, 0.42, ccw=True)]
    faces.append(tuple(plug))
    return W.Nurbs3D.from_list(faces)


def test_nurbs_cube_winding_number(oracle):
    P = G.gwn_nurbs3d_extract(nurbs_cube(W.Rng(5, "cube")))
    assert P.n > 12
    rng = W.Rng(9, "cubeq")
    inside = rng.uniform(60, 0.05, 0.95).reshape(20, 3)
    outside = rng.uniform(60, -1.0, 2.0).reshape(20, 3)
    outside = outside[np.any((outside < -0.05) | (outside > 1.05), axis=1)]
    # just below and above the hole and the rest of the top face
    top = np.array([[0.5, 0.5, 0.99], [0.5, 0.5, 1.01], [0.52, 0.48, 0.999], [0.1, 0.9, 0.995], [0.1, 0.9, 1.005]])
    q = np.concatenate([inside, outside, top])
    want = np.concatenate([np.ones(len(inside)), np.zeros(len(outside)), [1, 0, 1, 1, 0]])
    w = oracle.gwn3d(P, q)
    assert np.abs(w - want).max() < 1e-9, np.abs(w - want).max()


def test_empty_and_untrimmed_only():
    out = G.gwn_nurbs3d_extract(W.Nurbs3D.from_list([]))
    assert out.n == 0


def _one(**kw):
    f = dict(zip(["pu", "pv", "cp", "w", "U", "V", "trims"], holed_face()))
    f.update(kw)
    return W.Nurbs3D.from_list([(f["pu"], f["pv"], f["cp"], f["w"], f["U"], f["V"], f["trims"])])


@pytest.mark.parametrize("bad", ["degree", "unclamped", "weight", "outside", "open", "junction", "trim_degree"])
def test_invalid_nurbs3d(bad):
    f = holed_face()
    if bad == "degree":
        n = _one(pu=4)
    elif bad == "unclamped":
        U = f[4].copy()
        U[0] = U[0] - 0.5
        n = _one(U=U)
    elif bad == "weight":
        w = f[3].copy()
        w[1, 1] = 0.0
        n = _one(w=w)
    elif bad == "outside":
        n = _one(trims=[polyline([[0.5, -2], [3, -2], [3, 2], [1, 2], [0.5, -2]])])
    elif bad == "open":
        n = _one(trims=[polyline([[1, -2], [3, -2], [3, 2], [1, 2]])])
    elif bad == "junction":
        # a corner of the loop on the interior knot line u = 2.1
        n = _one(trims=[polyline([[1, -2], [2.1, -1.0], [3, -2], [3, 2], [1, 2], [1, -2]])])
    else:
        n = _one(trims=[(3, np.array([[1, -2], [3, -2], [3, 2], [1, -2.0]]), np.ones(4), [0, 0, 0, 0, 1, 1, 1, 1])])
    with pytest.raises(G.GwnError):
        G.gwn_nurbs3d_extract(n)


@pytest.mark.gpu
def test_nurbs_cube_on_gpu(oracle):
    """The extracted NURBS cube through the FP64 form, against the oracle."""
    torch = pytest.importorskip("torch")
    from paper_2605_19200_amd import presets
    P = G.gwn_nurbs3d_extract(nurbs_cube(W.Rng(5, "cube")))
    rng = W.Rng(11, "cubeg")
    q = np.concatenate([rng.uniform(300, -0.5, 1.5).reshape(100, 3),
                        np.array([[0.5, 0.5, 0.99], [0.5, 0.5, 1.01], [0.4, 0.45, 1.0 - 1e-4], [0.9, 0.1, 1e-3]])])
    ref = oracle.gwn3d(P, q)
    m = G.Model(P, presets.params(presets.FP64_3D))
    out, ins = m.query(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    w = out.cpu().numpy()
    m.close()
    assert np.abs(w - ref).max() <= 1e-6
    sure = np.abs(ref - 0.5) > 1e-3
    assert np.array_equal(ins.cpu().numpy()[sure].astype(bool), (ref >= 0.5)[sure])
