"""The 3D near-field rule with its error control, built for the host and
checked against the oracle on the CPU (no GPU): per leaf, the value is
within the tolerance eps_q, or the rule reports that it could not meet it
(never a silent value); errors and work move with eps_q.  Cases: sub-patches
of a sphere's polar patch (the edge collapsed to the pole, split as the
adaptive subdivision does), with queries near the pole and on its axis, and
the leaves of the CAD assembly (trimmed, split) around near-surface queries."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import presets
from paper_2605_19200_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(HERE, "..", "paper_2605_19200_amd")


@pytest.fixture(scope="module")
def rule(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    G.lib()   # the engine's library must exist
    out = str(tmp_path_factory.mktemp("near") / "libnear3d_host.so")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "near3d_host.cpp"), "-L", PKG, "-lgwn",
                           "-Wl,-rpath," + os.path.abspath(PKG), "-o", out],
                          stderr=subprocess.DEVNULL)
    L = ctypes.CDLL(out)
    L.near_leaf.restype = ctypes.c_double
    L.near_leaf.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int] + [ctypes.c_double] * 5 + \
        [ctypes.c_void_p, ctypes.c_void_p]

    def near(net, trims, q, eps_on, eps_q):
        h = np.ascontiguousarray(net, dtype=np.float64).reshape(-1)
        t = np.ascontiguousarray(trims, dtype=np.float64).reshape(-1) if len(trims) else np.zeros(9)
        ev, bud = ctypes.c_longlong(0), ctypes.c_int(0)
        v = L.near_leaf(h.ctypes.data, t.ctypes.data, len(trims), *map(float, q), eps_on, eps_q, ctypes.byref(ev),
                        ctypes.byref(bud))
        return v, ev.value, bool(bud.value)
    near.lib = L
    return near


# the 7/15 Gauss-Kronrod pair on [-1, 1] as published with QUADPACK
# (Piessens et al. 1983): Kronrod abscissae (descending, the Gauss ones at
# odd positions) and weights
K15_X = [0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
         0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
         0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
         0.207784955007898467600689403773245, 0.0]
K15_W = [0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
         0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
         0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
         0.204432940075298892414161999234649, 0.209482141084727828012999174891714]


@pytest.mark.parametrize("n", [4, 6, 7])
def test_kronrod_tables(rule, n):
    """The near-field rule's Gauss-Kronrod pairs: the Kronrod rule contains
    the n Gauss nodes, integrates polynomials of degree 3n + 1 exactly and
    fails two degrees above its exact degree; the Gauss weights integrate
    degree 2n - 1; the 7/15 pair equals the published one."""
    L = rule.lib
    L.gk_table.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 3
    xk, wk, wg = np.zeros(2 * n + 1), np.zeros(2 * n + 1), np.zeros(n)
    L.gk_table(n, xk.ctypes.data, wk.ctypes.data, wg.ctypes.data)
    assert np.all(np.diff(xk) > 0) and xk[0] > 0 and xk[-1] < 1 and np.all(wk > 0) and np.all(wg > 0)
    xg = xk[1::2]
    gx, gw = np.polynomial.legendre.leggauss(n)
    assert np.allclose(xg, (gx + 1) / 2, atol=1e-15) and np.allclose(wg, gw / 2, atol=1e-15)
    for k in range(3 * n + 2):
        assert abs(np.dot(wk, xk ** k) - 1.0 / (k + 1)) < 1e-15, k
    for k in range(2 * n):
        assert abs(np.dot(wg, xg ** k) - 1.0 / (k + 1)) < 1e-15, k
    # the Kronrod degree is 3n + 1 (n even) or 3n + 2 (n odd, by symmetry);
    # two degrees higher it is no longer exact
    top = 3 * n + 1 + (n % 2)
    xs = 2 * xk - 1
    assert abs(np.dot(wk, xs ** (top + 2)) * 2 - 2.0 / (top + 3)) > 1e-8
    if n == 7:
        assert np.allclose(np.sort(xs)[::-1][:8], K15_X, atol=2e-16)
        assert np.allclose((wk * 2)[::-1][:8], K15_W, atol=2e-16)


def split(h, d):
    h = np.moveaxis(h, d, 0)
    c = [h[i] for i in range(4)]
    b = [0.5 * (c[i] + c[i + 1]) for i in range(3)]
    cc = [0.5 * (b[i] + b[i + 1]) for i in range(2)]
    dd = 0.5 * (cc[0] + cc[1])
    return np.moveaxis(np.stack([c[0], b[0], cc[0], dd]), 0, d), np.moveaxis(np.stack([dd, cc[1], b[2], c[3]]), 0, d)


def leaves_of(h, levels):
    out = [h]
    for lev in range(levels):
        out = [x for y in out for x in split(y, lev % 2)]
    return out


def as_patch(net, trims=()):
    tl = [(c.reshape(3, 3)[:, :2] / c.reshape(3, 3)[:, 2:3], c.reshape(3, 3)[:, 2].copy()) for c in trims]
    return W.Patches3D.from_list([(net[..., :3] / net[..., 3:4], net[..., 3], tl)])


@pytest.fixture(scope="module")
def polar_cases(oracle):
    sph = W.bodies(0, [("sphere", (0, 0, 0), 1.0)], disp=0.0)
    cp, w = sph[32]                                  # its edge v = 0 is the pole (0, 0, -1)
    net = np.concatenate([cp * w[..., None], w[..., None]], -1)
    pole = np.array([0.0, 0.0, -1.0])
    t = np.cross(pole, [0.3, 0.5, 0.8])
    t /= np.linalg.norm(t)
    eps_on = 1e-12 * math.sqrt(12)
    rng = W.Rng(38, "polar")
    cases = []
    for levels in (0, 2, 4):
        for h in leaves_of(net, levels)[:4]:
            P = as_patch(h)
            for d in (1e-2, 1e-4, 1e-6):                  # near points away from the axis
                u, v = rng.uniform(2, 0.05, 0.95)
                S, n, _ = W.eval_patch(P.cp_xyz[0], P.cp_w[0], u, v)
                cases.append(("off", h, S + d * n))
                cases.append(("off", h, pole + d * pole + 3e-2 * t))
            for d in (1e-3, 1e-4, 1e-6):                  # on the polar axis
                cases.append(("axis", h, pole - d * pole))
    refs = [oracle.gwn3d(as_patch(h), q[None], eps_on=eps_on, strict=False)[0] for _, h, q in cases]
    return cases, refs, eps_on


def test_polar_subpatches(rule, polar_cases):
    """Split polar sub-patches meet the tolerance away from the pole's axis;
    on the axis within 1e-3 of the pole (the foot point is then the whole
    collapsed edge) the rule either meets it or reports the budget overrun."""
    cases, refs, eps_on = polar_cases
    eps_q = 1e-8
    for (kind, h, q), ref in zip(cases, refs):
        v, _, budget = rule(h, [], q, eps_on, eps_q)
        err = abs(v - ref)
        if kind == "off":
            assert not budget and err <= eps_q, (err, q)
        else:
            assert err <= eps_q or budget, (err, q)


@pytest.fixture(scope="module")
def cad_pairs(oracle):
    P = W.cad_assembly(4, n_bodies=2)
    h = G.gwn_build3d(P, presets.params(presets.FP64_3D, device=-1))
    leaves = G.gwn_inspect(h, G.GWN_I_LEAVES)
    trims = G.gwn_inspect(h, G.GWN_I_LEAF_TRIMS)
    G.gwn_free(h)
    nets = leaves[:, 1:].reshape(-1, 4, 4, 4)
    eu = nets[..., :3] / nets[..., 3:4]
    lo, hi = eu.reshape(-1, 16, 3).min(1), eu.reshape(-1, 16, 3).max(1)
    diag = np.linalg.norm(hi - lo, axis=1)
    q = W.near_surface_queries(P, W.Rng(39, "pairs"), 24)
    blo, bhi = P.bbox()
    eps_on = 1e-12 * np.linalg.norm(bhi - blo)
    pairs = []
    for k in range(q.shape[0]):
        d = np.linalg.norm(np.maximum(np.maximum(lo - q[k], q[k] - hi), 0), axis=1)
        for l in np.nonzero(d < 0.25 * diag)[0][:4]:
            tl = trims[trims[:, 0] == l, 1:]
            pairs.append((nets[l], tl, q[k]))
    refs = [oracle.gwn3d(as_patch(n, t), qq[None], eps_on=eps_on, strict=False)[0] for n, t, qq in pairs]
    return pairs, refs, eps_on


def test_cad_leaves_and_eps_q(rule, cad_pairs):
    """Trimmed CAD leaves: within eps_q at every tolerance, the worst error
    does not grow and the work does not shrink as eps_q tightens."""
    pairs, refs, eps_on = cad_pairs
    assert len(pairs) >= 40
    worst, work = [], []
    for eps_q in (1e-6, 1e-8, 1e-10):
        errs, ev = [], 0
        for (net, tl, q), ref in zip(pairs, refs):
            v, e, budget = rule(net, tl, q, eps_on, eps_q)
            assert not budget
            errs.append(abs(v - ref))
            ev += e
        assert max(errs) <= eps_q, (eps_q, max(errs))
        worst.append(max(errs))
        work.append(ev)
    assert worst[0] >= worst[1] * 0.999 >= 0 and worst[1] >= worst[2] * 0.999, worst
    assert work[0] <= work[1] <= work[2], work
