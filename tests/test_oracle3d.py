"""Pins of the 3D CPU oracle against facts fixed by the mathematics.

Each targets a way the oracle could be wrong: the solid-angle integrand's
sign or operand order (Van Oosterom-Strackee triangles, bilinear quads,
orientation reversal), the Green's-theorem treatment of trims (flat plate
with a hole, visible-area fraction at a trimmed sphere's centre, brute-force
hole integral), the near field (sphere 0/1/0.5, jump of 1 across the
surface), and patch handling in general (dense tensor quadrature, subdivision
invariance, additivity).
"""
import math

import numpy as np
import pytest

from paper_2605_19200_amd import workloads as W


def vos(A, B, C, q):
    """Signed solid angle of triangle ABC at q (Van Oosterom & Strackee, IEEE
    TBME 1983): tan(Omega/2) = a.(b x c) / (abc + (a.b)c + (a.c)b + (b.c)a)."""
    a, b, c = np.asarray(A) - q, np.asarray(B) - q, np.asarray(C) - q
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = a @ np.cross(b, c)
    den = la * lb * lc + (a @ b) * lc + (a @ c) * lb + (b @ c) * la
    return 2 * math.atan2(num, den)


def bilinear_patch(P00, P10, P11, P01, w=None):
    """Bicubic control net of the bilinear patch with the given corners
    (index [i along u][j along v]), optionally with weights."""
    h = np.zeros((2, 2, 4))
    corners = {(0, 0): P00, (1, 0): P10, (1, 1): P11, (0, 1): P01}
    for (i, j), p in corners.items():
        wt = 1.0 if w is None else w[i][j]
        h[i, j, :3] = np.asarray(p, float) * wt
        h[i, j, 3] = wt
    for _ in range(2):
        h = W.elevate_homogeneous(h, 0)
        h = W.elevate_homogeneous(h, 1)
    return h[..., :3] / h[..., 3:4], h[..., 3]


def patches(*items):
    return W.Patches3D.from_list(items)


def hom_grid(cp, w, u, v):
    """Homogeneous point and partials on a tensor grid (numpy, for brute force)."""
    cp = np.asarray(cp).reshape(4, 4, 3)
    w = np.asarray(w).reshape(4, 4)
    h = np.concatenate([cp * w[..., None], w[..., None]], axis=2)

    def bern(t):
        s = 1 - t
        return np.stack([s ** 3, 3 * s * s * t, 3 * s * t * t, t ** 3], -1)

    def dbern(t):
        s = 1 - t
        return np.stack([-3 * s * s, 3 * s * s - 6 * s * t, 6 * s * t - 3 * t * t, 3 * t * t], -1)
    H = np.einsum("...i,...j,ijk->...k", bern(u), bern(v), h)
    Hu = np.einsum("...i,...j,ijk->...k", dbern(u), bern(v), h)
    Hv = np.einsum("...i,...j,ijk->...k", bern(u), dbern(v), h)
    return H, Hu, Hv


def density(cp, w, q, u, v):
    """det[A, A_u, A_v] / |A|^3 with A = H - q W."""
    H, Hu, Hv = hom_grid(cp, w, u, v)
    A = H[..., :3] - H[..., 3:4] * q
    Au = Hu[..., :3] - Hu[..., 3:4] * q
    Av = Hv[..., :3] - Hv[..., 3:4] * q
    det = np.einsum("...k,...k->...", A, np.cross(Au, Av))
    return det / np.linalg.norm(A, axis=-1) ** 3


def tensor_gl(cp, w, q, n=120):
    x, wt = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (x + 1)
    u, v = np.meshgrid(t, t, indexing="ij")
    ww = np.outer(wt, wt) / 4
    return (ww * density(cp, w, q, u, v)).sum() / (4 * math.pi)


def disk_gl(cp, w, q, c, r, n=120):
    """Integral of the density over the disk |(u,v) - c| < r (polar GL)."""
    x, wt = np.polynomial.legendre.leggauss(n)
    rho = 0.5 * r * (x + 1)
    phi = math.pi * (x + 1)
    R, P = np.meshgrid(rho, phi, indexing="ij")
    ww = np.outer(wt * 0.5 * r, wt * math.pi) * R
    return (ww * density(cp, w, q, c[0] + R * np.cos(P), c[1] + R * np.sin(P))).sum() / (4 * math.pi)


@pytest.fixture(scope="module")
def sphere():
    return W.Patches3D.from_list([(cp, w, []) for cp, w in W.bodies(0, [("sphere", (0, 0, 0), 1.0)], disp=0.0)])


def test_sphere_inside_outside_surface(oracle, sphere):
    rng = W.Rng(31, "sph")
    d = rng.uniform((8, 3), -1, 1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    inside = d * rng.uniform(8, 0.0, 0.95)[:, None]
    outside = d * rng.uniform(8, 1.05, 3.0)[:, None]
    assert np.abs(oracle.gwn3d(sphere, inside) - 1).max() < 1e-10
    assert np.abs(oracle.gwn3d(sphere, outside)).max() < 1e-10
    k = rng.integers(4, 0, sphere.n - 1)
    uv = rng.uniform((4, 2), 0.1, 0.9)
    on = np.array([W.eval_patch(sphere.cp_xyz[i], sphere.cp_w[i], a, b)[0] for i, (a, b) in zip(k, uv)])
    assert np.abs(oracle.gwn3d(sphere, on) - 0.5).max() < 1e-7


def test_jump_across_surface(oracle, sphere):
    i = 100
    S, n, _ = W.eval_patch(sphere.cp_xyz[i], sphere.cp_w[i], 0.37, 0.61)
    wi, wo = oracle.gwn3d(sphere, np.stack([S - 1e-6 * n, S + 1e-6 * n]))
    assert abs((wi - wo) - 1.0) < 1e-6


def test_triangles_van_oosterom_strackee(oracle):
    rng = W.Rng(32, "tri")
    for _ in range(6):
        A, B, C = rng.uniform((3, 3), -1, 1)
        cp, w = bilinear_patch(A, B, C, C)
        P = patches((cp, w, []))
        qs = rng.uniform((4, 3), -2, 2)
        got = oracle.gwn3d(P, qs)
        ref = np.array([vos(A, B, C, q) for q in qs]) / (4 * math.pi)
        assert np.abs(got - ref).max() < 1e-10


def test_bilinear_quad_equals_two_triangles(oracle):
    rng = W.Rng(33, "quad")
    A, B, C, D = np.array([[0, 0, 0], [1, 0, 0.2], [1, 1, -0.1], [0, 1, 0.3]], float)
    cp, w = bilinear_patch(A, B, C, D, w=[[1.0, 1.7], [0.6, 1.2]])
    P = patches((cp, w, []))
    # points outside the tetrahedron ABCD (|z| well above its extent)
    qs = np.concatenate([rng.uniform((3, 2), -0.5, 1.5), rng.uniform((3, 1), 0.6, 2.0)], 1)
    qs[1, 2] *= -1
    got = oracle.gwn3d(P, qs)
    ref = np.array([vos(A, B, C, q) + vos(A, C, D, q) for q in qs]) / (4 * math.pi)
    assert np.abs(got - ref).max() < 1e-10


def test_flat_plate_with_hole_on_axis(oracle):
    cp, w = bilinear_patch((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0))
    c, R = (0.5, 0.45), 0.2
    P = patches((cp, w, W.square_trim() + W.circle_trim(c, R, ccw=False)))
    for h in [0.05, 0.3, -0.2]:
        q = np.array([c[0], c[1], h])
        sq = vos((0, 0, 0), (1, 0, 0), (1, 1, 0), q) + vos((0, 0, 0), (1, 1, 0), (0, 1, 0), q)
        disk = -math.copysign(1.0, h) * 2 * math.pi * (1 - abs(h) / math.hypot(h, R))
        got = oracle.gwn3d(P, q[None])[0]
        assert abs(got - (sq - disk) / (4 * math.pi)) < 1e-10, h


def random_patch(rng, warp=0.25):
    cp, w = bilinear_patch((0, 0, 0), (1, 0, 0.1), (1, 1, 0), (0, 1, -0.1))
    cp = cp + warp * rng.uniform((4, 4, 3), -1, 1)
    w = rng.uniform((4, 4), 0.5, 2.0)
    return cp, w


def test_dense_tensor_quadrature(oracle):
    rng = W.Rng(34, "dense")
    for _ in range(3):
        cp, w = random_patch(rng)
        P = patches((cp, w, []))
        qs = np.array([[0.5, 0.5, 0.9], [1.6, 0.4, 0.2], [-0.5, -0.4, -0.6]])
        got = oracle.gwn3d(P, qs)
        ref = np.array([tensor_gl(cp, w, q) for q in qs])
        assert np.abs(got - ref).max() < 1e-10


def test_trimmed_patch_against_brute_force(oracle):
    rng = W.Rng(35, "trim")
    cp, w = random_patch(rng, warp=0.15)
    c, r = np.array([0.45, 0.55]), 0.22
    P = patches((cp, w, W.square_trim() + W.circle_trim(c, r, ccw=False)))
    qs = np.array([[0.5, 0.5, 0.8], [1.5, 0.3, -0.3], [0.2, 1.4, 0.4]])
    got = oracle.gwn3d(P, qs)
    ref = np.array([tensor_gl(cp, w, q) - disk_gl(cp, w, q, c, r) for q in qs])
    assert np.abs(got - ref).max() < 1e-10


def test_trimmed_sphere_visible_area_at_centre(oracle, sphere):
    """At the centre of an exact sphere the density is dA / R^2, so the GWN
    of a sphere with one hole is its visible area over 4 pi R^2."""
    i, c, r = 200, np.array([0.5, 0.45]), 0.3
    lst = sphere.to_list()
    cp, w, _ = lst[i]
    lst[i] = (cp, w, W.square_trim() + W.circle_trim(c, r, ccw=False))
    P = W.Patches3D.from_list(lst)
    # hole area on the surface: integral of |S_u x S_v| over the disk
    x, wt = np.polynomial.legendre.leggauss(80)
    rho, phi = 0.5 * r * (x + 1), math.pi * (x + 1)
    R, Ph = np.meshgrid(rho, phi, indexing="ij")
    _, _, jac = W.eval_patch(cp, w, c[0] + R * np.cos(Ph), c[1] + R * np.sin(Ph))
    area = (np.outer(wt * 0.5 * r, wt * math.pi) * R * jac).sum()
    got = oracle.gwn3d(P, np.zeros((1, 3)))[0]
    assert abs(got - (1 - area / (4 * math.pi))) < 1e-10


def test_orientation_subdivision_additivity(oracle):
    rng = W.Rng(36, "inv")
    cp, w = random_patch(rng)
    qs = np.array([[0.3, 0.6, 0.5], [0.7, 0.2, -0.25], [1.3, 1.1, 0.1]])
    base = oracle.gwn3d(patches((cp, w, [])), qs)
    # swapping u and v reverses the normal
    flip = oracle.gwn3d(patches((cp.transpose(1, 0, 2), w.T, [])), qs)
    assert np.abs(flip + base).max() < 1e-11
    # de Casteljau split at u = 1/2 (Sec. 3.2: subdivision keeps the GWN)
    h = np.concatenate([cp * w[..., None], w[..., None]], axis=2)
    left, right = [h[0]], [h[3]]
    cur = h
    while cur.shape[0] > 1:
        cur = 0.5 * (cur[:-1] + cur[1:])
        left.append(cur[0])
        right.append(cur[-1])
    L, R = np.array(left), np.array(right[::-1])
    halves = patches((L[..., :3] / L[..., 3:], L[..., 3], []), (R[..., :3] / R[..., 3:], R[..., 3], []))
    assert np.abs(oracle.gwn3d(halves, qs) - base).max() < 1e-11
    # additivity over primitives
    cp2, w2 = random_patch(rng)
    both = oracle.gwn3d(patches((cp, w, []), (cp2, w2, [])), qs)
    assert np.abs(both - base - oracle.gwn3d(patches((cp2, w2, [])), qs)).max() < 1e-12


def test_open_trim_loop_rejected(oracle):
    cp, w = bilinear_patch((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0))
    P = patches((cp, w, W.square_trim()[:3]))
    with pytest.raises(ValueError):
        oracle.gwn3d(P, np.zeros((1, 3)))


def test_on_surface_of_trimmed_patch_complementary_trims(oracle, sphere):
    """On-surface branch for trimmed patches.  One patch of the exact sphere
    is replaced by two copies with complementary trims: copy A keeps the
    square with a CW circular hole, copy B has the matching CCW disk as its
    only loop.  The two visible regions tile the original patch, so the
    surface stays closed: w = 0.5 exactly on the surface both where A is
    visible and in A's hole (where B is), and 1 / 0 just inside / outside.
    A query on the surface lies on the visible part of exactly one copy and
    on the trimmed-away part of the other, which exercises the oracle's
    visibility test in both directions."""
    i, c, r = 230, np.array([0.45, 0.55]), 0.25
    lst = sphere.to_list()
    cp, w, _ = lst[i]
    lst[i] = (cp, w, W.square_trim() + W.circle_trim(c, r, ccw=False))
    lst.append((cp, w, W.circle_trim(c, r, ccw=True)))
    P = W.Patches3D.from_list(lst)
    rng = W.Rng(36, "comp")
    # (u, v) inside the disk (hole of A) and outside it (visible part of A),
    # at least 0.05 from the trim circle
    ang = rng.uniform(6, 0, 2 * math.pi)
    rad_in = rng.uniform(6, 0.0, r - 0.05)
    uv_in = c + rad_in[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    uv_out = rng.uniform((12, 2), 0.05, 0.95)
    uv_out = uv_out[np.linalg.norm(uv_out - c, axis=1) > r + 0.05][:6]
    assert uv_out.shape[0] == 6
    uv = np.concatenate([uv_in, uv_out])
    S, n, _ = W.eval_patch(cp, w, uv[:, 0], uv[:, 1])
    got = oracle.gwn3d(P, S)
    assert np.abs(got - 0.5).max() < 1e-7, got
    for d in (1e-2, 1e-5):
        wi = oracle.gwn3d(P, S - d * n)
        wo = oracle.gwn3d(P, S + d * n)
        assert np.abs(wi - 1).max() < 1e-9 and np.abs(wo).max() < 1e-9, d
    assert oracle.last_errbound <= oracle.STRICT_ERRBOUND


def test_unconverged_quadrature_is_reported(oracle, sphere, tmp_path):
    """Non-convergence is reported, not silent.  The oracle rebuilt with a
    split budget of 0 per adaptive call (every panel is accepted as first
    estimated) and no room for graded breakpoints (only the two uniform
    panels per level) cannot resolve the density's peak 1e-4 from the
    sphere: the count and the error bound must show it.  The same query with the normal budget converges (count 0 or a bound
    far below the strict threshold)."""
    import ctypes
    import subprocess
    lib = tmp_path / "oracle_small_budget.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-DMAX_SPLITS=0", "-DMAX_BREAKS=3", "-o",
                           str(lib), oracle.SRC, "-lm"])
    L = ctypes.CDLL(str(lib))
    L.oracle_gwn3d.argtypes = oracle.lib().oracle_gwn3d.argtypes
    L.oracle_last_unconverged.restype = ctypes.c_longlong
    L.oracle_last_errbound.restype = ctypes.c_double
    S, n, _ = W.eval_patch(sphere.cp_xyz[100], sphere.cp_w[100], 0.37, 0.61)
    q = np.ascontiguousarray((S - 1e-4 * n)[None])
    arrs = [np.ascontiguousarray(a, dtype=t) for a, t in
            [(sphere.cp_xyz, np.float64), (sphere.cp_w, np.float64), (sphere.trim_offset, np.int64),
             (sphere.trim_degree, np.int32), (sphere.trim_cp_offset, np.int64), (sphere.trim_cp_uv, np.float64),
             (sphere.trim_cp_w, np.float64)]]
    out = np.empty(1)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert L.oracle_gwn3d(sphere.n, *[ptr(a) for a in arrs], 1, ptr(q), ptr(out),
                          oracle.default_eps_on(*sphere.bbox()), 1) == 0
    assert L.oracle_last_unconverged() > 0 and L.oracle_last_errbound() > oracle.STRICT_ERRBOUND, \
        (L.oracle_last_unconverged(), L.oracle_last_errbound())
    w = oracle.gwn3d(sphere, q)
    assert oracle.last_errbound <= oracle.STRICT_ERRBOUND and abs(w[0] - 1.0) < 1e-9
