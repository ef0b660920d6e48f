"""GPU parity of the 3D query path against the CPU oracle and closed forms.
Every call goes through the C ABI."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import presets
from paper_2605_19200_amd import workloads as W
from tests.test_oracle3d import bilinear_patch, patches, vos

pytestmark = pytest.mark.gpu
TOL = 1e-6
BAND = 1e-3


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run(model, q):
    out, ins = model.query(dev(q))
    torch.cuda.synchronize()
    return out.cpu().numpy(), ins.cpu().numpy()


def check(w, ins, ref, tol=TOL):
    err = np.abs(w - ref)
    assert np.all(np.isfinite(w))
    assert err.max() <= tol, f"max |dw| = {err.max():.3e} at {int(np.argmax(err))}"
    sure = np.abs(ref - 0.5) > BAND
    assert np.array_equal(ins[sure].astype(bool), (ref >= 0.5)[sure])


@pytest.fixture(scope="module")
def sphere():
    return W.Patches3D.from_list([(cp, w, []) for cp, w in W.bodies(0, [("sphere", (0, 0, 0), 1.0)], disp=0.0)])


def sphere_points(sphere, rng, k):
    idx = rng.integers(k, 0, sphere.n - 1)
    uv = rng.uniform((k, 2), 0.05, 0.95)
    S, n = [], []
    for i, (a, b) in zip(idx, uv):
        s, nn, _ = W.eval_patch(sphere.cp_xyz[i], sphere.cp_w[i], a, b)
        S.append(s)
        n.append(nn)
    return np.array(S), np.array(n)


@pytest.mark.parametrize("frac,near_tol", [(0.1, 1e-8), (presets.FP64_3D["max_diag_frac"], 1e-8)])
def test_sphere_all_direct(sphere, frac, near_tol):
    # every leaf evaluated directly, polar patches split like the others at
    # the preset's subdivision.  The bar is below what the presets are sized
    # for: the near-field tolerance is set below it (the preset's 1e-8 per
    # leaf serves the 1e-6 bar), and leaves within half their diagonal take
    # the error-controlled near-field rule (the fixed node-set rules farther
    # out err by ~1e-9 per leaf, which at the preset's 0.25 adds to ~1e-8
    # over the many small leaves near q)
    m = G.Model(sphere, presets.params(presets.FP64_3D, beta=1e8, far_tol=0.0, max_diag_frac=frac, eps_q=1e-11,
                                       near_ratio=0.5))
    print(f"sphere all direct, max_diag_frac {frac}: {int(m.inspect(G.GWN_I_SUMMARY)[0][2])} leaves", flush=True)
    rng = W.Rng(41, "sph")
    d = rng.uniform((64, 3), -1, 1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    w, _ = run(m, d * rng.uniform(64, 0.0, 0.95)[:, None])
    assert np.abs(w - 1).max() < 1e-9
    w, _ = run(m, d * rng.uniform(64, 1.05, 3.0)[:, None])
    assert np.abs(w).max() < 1e-9
    S, n = sphere_points(sphere, rng, 48)
    for dd in [1e-2, 1e-4, 1e-6]:
        wi, _ = run(m, S - dd * n)
        wo, _ = run(m, S + dd * n)
        print(f"  d={dd:g}: max |w - 1| inside {np.abs(wi - 1).max():.2e}, max |w| outside {np.abs(wo).max():.2e}",
              flush=True)
        assert np.abs(wi - 1).max() < near_tol and np.abs(wo).max() < near_tol, dd
    w, _ = run(m, S)
    assert np.abs(w - 0.5).max() < 1e-7


def test_sphere_fp64_form(sphere, oracle):
    m = G.Model(sphere, presets.params(presets.FP64_3D))
    rng = W.Rng(42, "sph")
    S, n = sphere_points(sphere, rng, 32)
    q = np.concatenate([S - 1e-3 * n, S + 2e-2 * n, rng.uniform((32, 3), -1.5, 1.5)])
    w, ins = run(m, q)
    check(w, ins, oracle.gwn3d(sphere, q))


def test_closed_forms_triangle_and_holed_plate():
    rng = W.Rng(43, "cf")
    A, B, C = np.array([[0, 0, 0], [1, 0.1, 0], [0.2, 1, 0.1]])
    m = G.Model(patches((*bilinear_patch(A, B, C, C), [])), presets.params(presets.FP64_3D, beta=1e8, far_tol=0.0))
    qs = rng.uniform((64, 3), -1, 1.5)
    w, _ = run(m, qs)
    ref = np.array([vos(A, B, C, q) for q in qs]) / (4 * math.pi)
    assert np.abs(w - ref).max() < 1e-9
    cp, wt = bilinear_patch((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0))
    c, R = (0.5, 0.45), 0.2
    m = G.Model(patches((cp, wt, W.square_trim() + W.circle_trim(c, R, ccw=False))),
                presets.params(presets.FP64_3D, beta=1e8, far_tol=0.0))
    hs = np.array([0.001, 0.05, 0.3, -0.2, -1e-5])
    q = np.stack([np.full(hs.shape, c[0]), np.full(hs.shape, c[1]), hs], 1)
    w, _ = run(m, q)
    for k, h in enumerate(hs):
        sq = vos((0, 0, 0), (1, 0, 0), (1, 1, 0), q[k]) + vos((0, 0, 0), (1, 1, 0), (0, 1, 0), q[k])
        disk = -math.copysign(1.0, h) * 2 * math.pi * (1 - abs(h) / math.hypot(h, R))
        assert abs(w[k] - (sq - disk) / (4 * math.pi)) < 1e-9, h


@pytest.fixture(scope="module")
def cfg3(oracle):
    P, q = W.config3()
    idx = W.Rng(44, "s3").permutation(q.shape[0])[:96]
    near = W.near_surface_queries(P, W.Rng(44, "n3"), 48)
    qs = np.concatenate([q[idx], near])
    return P, q, qs, oracle.gwn3d(P, qs)


def test_config3_fp64_sampled(cfg3):
    P, q, qs, ref = cfg3
    m = G.Model(P, presets.params(presets.FP64_3D))
    w, ins = run(m, qs)
    check(w, ins, ref)


def test_config3_full_grid_subset_consistent(cfg3):
    """The full 128^3 launch gives the same values as the sampled call, and
    no query of the grid hits a stack or near-field slot limit (NaN).  (The
    holed bodies are not closed, so w is not confined to [0, 1].)"""
    P, q, qs, ref = cfg3
    m = G.Model(P, presets.params(presets.FP64_3D, wave_accept=0))
    w_full, _ = run(m, q)
    assert np.all(np.isfinite(w_full))
    idx = W.Rng(44, "s3").permutation(q.shape[0])[:96]
    assert np.array_equal(w_full[idx], run(m, q[idx])[0])
    check(w_full[idx], (w_full[idx] >= 0.5).astype(np.uint8), ref[:96])


@pytest.fixture(scope="module")
def cfg4(oracle):
    P = W.cad_assembly(4, n_bodies=10)
    lo, hi = P.bbox()
    near = W.near_surface_queries(P, W.Rng(45, "n4"), 40)
    uni = W.bbox_queries_uniform(W.Rng(45, "u4"), lo, hi, 40, 1.0)
    qs = np.concatenate([near, uni])
    return P, qs, oracle.gwn3d(P, qs)


def test_config4_fp64_and_mixed(cfg4):
    P, qs, ref = cfg4
    m = G.Model(P, presets.params(presets.FP64_3D))
    w, ins = run(m, qs)
    check(w, ins, ref)
    mm = G.Model(P, presets.params(presets.MIXED_3D))
    sure = np.abs(ref - 0.5) > BAND
    for wa in (0, 1):   # per-query far tests, then wave acceptance in both passes
        mm.set(wave_accept=wa)
        wm, insm = run(mm, qs)
        assert np.abs(wm - ref).max() < 5e-3
        assert np.array_equal(insm[sure].astype(bool), (ref >= 0.5)[sure])


@pytest.mark.parametrize("preset", ["FP64_3D", "MIXED_3D"])
def test_stackless_walk_single_lane_3d(cfg4, preset):
    """A one-query call is a wave of one lane: the stackless walk of wave
    acceptance gives the stack walk's value bit for bit (far terms, node
    sets and the near-field list in the same order)."""
    P, qs, _ = cfg4
    m = G.Model(P, presets.params(getattr(presets, preset), wave_accept=0))
    sel = qs[::4]
    w0 = np.array([run(m, sel[i:i + 1])[0][0] for i in range(sel.shape[0])])
    m.set(wave_accept=1)
    w1 = np.array([run(m, sel[i:i + 1])[0][0] for i in range(sel.shape[0])])
    assert np.all(np.isfinite(w0)) and np.array_equal(w0, w1)
    m.close()


@pytest.mark.parametrize("scale", [1e-6, 1e6])
def test_scale_invariance_3d(cfg4, scale):
    """The trimmed assembly scaled as a whole keeps its w in both forms:
    far field, node sets and near-field rule work in scale-free units."""
    P, qs, ref = cfg4
    S = W.Patches3D(P.cp_xyz * scale, P.cp_w, P.trim_offset, P.trim_degree, P.trim_cp_offset,
                    P.trim_cp_uv, P.trim_cp_w)
    m = G.Model(S, presets.params(presets.FP64_3D))
    w, ins = run(m, qs * scale)
    check(w, ins, ref)
    mm = G.Model(S, presets.params(presets.MIXED_3D))
    wm, insm = run(mm, qs * scale)
    assert np.all(np.isfinite(wm)) and np.abs(wm - ref).max() < 5e-3
    sure = np.abs(ref - 0.5) > BAND
    assert np.array_equal(insm[sure].astype(bool), (ref >= 0.5)[sure])


def test_batch_bitwise_3d(cfg4, sphere):
    P, qs, _ = cfg4
    m1 = G.Model(P, presets.params(presets.FP64_3D, wave_accept=0))
    m2 = G.Model(sphere, presets.params(presets.MIXED_3D, wave_accept=0))
    q2 = W.Rng(46, "b").uniform((100, 3), -1.2, 1.2)
    s1, _ = run(m1, qs)
    s2, _ = run(m2, q2)
    parts = [(m1, qs[:30]), (m2, q2[:64]), (m1, qs[30:]), (m2, q2[64:])]
    pts = np.concatenate([p for _, p in parts])
    off = np.cumsum([0] + [p.shape[0] for _, p in parts])
    out = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
    G.gwn_query_batch([m.h for m, _ in parts], off, dev(pts), out, None)
    torch.cuda.synchronize()
    w = out.cpu().numpy()
    assert np.array_equal(w[off[0]:off[1]], s1[:30]) and np.array_equal(w[off[2]:off[3]], s1[30:])
    assert np.array_equal(w[off[1]:off[2]], s2[:64]) and np.array_equal(w[off[3]:off[4]], s2[64:])


def test_empty_and_ragged_3d(sphere):
    m = G.Model(W.Patches3D.from_list([]), presets.params(presets.FP64_3D))
    w, _ = run(m, np.ones((5, 3)))
    assert np.all(w == 0)
    m = G.Model(sphere, presets.params(presets.FP64_3D, wave_accept=0))
    q = W.Rng(47, "r").uniform((200, 3), -1.5, 1.5)
    full, _ = run(m, q)
    for n in [1, 63, 65, 129]:
        assert np.array_equal(run(m, q[:n])[0], full[:n])


def test_error_decreases_with_order_3d(cfg3):
    """Far-field error of the bodies scene at beta = 3 falls with the
    expansion order (orders above the paper's 2 through solid harmonics)."""
    P, q, qs, ref = cfg3
    errs = []
    for order in (0, 2, 4, 6):
        m = G.Model(P, presets.params(presets.FP64_3D, beta=3.0, far_tol=0.0, taylor_order=order))
        w, _ = run(m, qs)
        errs.append(np.abs(w - ref).max())
        m.close()
    assert errs[1] < errs[0] and errs[2] < errs[1] and errs[3] < errs[2], errs
    assert errs[3] < 1e-5


def test_paper_order_3d(cfg3):
    """The paper's order 2 at the beta that meets the bound."""
    P, q, qs, ref = cfg3
    m = G.Model(P, presets.params(presets.PAPER_ORDER_3D))
    w, ins = run(m, qs)
    check(w, ins, ref)


def test_stretched_patch_near_field(cfg3, oracle):
    """A query 1.4e-4 from a bodies-scene patch whose distance function has a
    second local minimum 4.9e-3 away (strongly non-uniform parametrisation
    near a pole): the near-field rule splits the patch between the minima."""
    P = cfg3[0]
    q = np.array([[-0.1256628870943714, 2.3888418271647667, 3.493370704897016]])
    q = np.concatenate([q, q + np.array([[2e-4, -1e-4, 5e-5]]), q + np.array([[-3e-4, 2e-4, 1e-4]])])
    m = G.Model(P, presets.params(presets.FP64_3D))
    w, ins = run(m, q)
    check(w, ins, oracle.gwn3d(P, q))


def test_far_budget_repack_on_device(cfg3):
    """Changing far_tol on a device model rewrites the 3D cluster radii in
    place: results equal a fresh build with the new setting bit for bit, in
    both directions, and the budget keeps the preset's accuracy."""
    P, q, qs, ref = cfg3
    m = G.Model(P, presets.params(presets.FP64_3D))
    assert presets.FP64_3D["far_tol"] > 0
    w_budget, ins = run(m, qs)
    check(w_budget, ins, ref)
    m.set(far_tol=0.0)
    w_uniform, _ = run(m, qs)
    fresh = G.Model(P, presets.params(presets.FP64_3D, far_tol=0.0))
    assert np.array_equal(w_uniform, run(fresh, qs)[0])
    fresh.close()
    assert not np.array_equal(w_uniform, w_budget)
    m.set(far_tol=presets.FP64_3D["far_tol"])
    assert np.array_equal(run(m, qs)[0], w_budget)
    fb = m.inspect(G.GWN_I_FARBETA)[:, 0]
    assert np.all(np.isfinite(fb)) and np.all(fb >= 1.5)
    m.close()


def test_device_lbvh_matches_host():
    """A model built for a device sorts its leaves, links the radix tree and
    runs the leaf quadrature there (moments, multipole moments, node sets).
    Against a host-only build of the same patches: the same tree and leaf
    order, bit for bit; the same boxes; centres, moments and multipole
    moments to rounding (the device sums the quadrature nodes in another
    order)."""
    P = W.bodies(3, [("sphere", np.array([0.0, 0.0, 0.0]), 1.0), ("torus", np.array([2.5, 0.3, 0.1]), 0.8)])
    P = W.Patches3D.from_list([(cp, w, W.square_trim()) for cp, w in P]).concat(W.config4()[0].subset(range(0, 512, 7)))
    hd = G.gwn_build3d(P, presets.params(presets.FP64_3D))
    hh = G.gwn_build3d(P, presets.params(presets.FP64_3D, device=-1))
    try:
        assert np.array_equal(G.gwn_inspect(hd, G.GWN_I_LEAVES), G.gwn_inspect(hh, G.GWN_I_LEAVES))
        nd, nh = G.gwn_inspect(hd, G.GWN_I_NODES), G.gwn_inspect(hh, G.GWN_I_NODES)
        assert np.array_equal(nd[:, :3], nh[:, :3]) and np.array_equal(nd[:, 7:], nh[:, 7:])
        scale = np.abs(nh[:, 3:7]).max()
        assert np.abs(nd[:, 3:7] - nh[:, 3:7]).max() <= 1e-13 * scale
        for what in (G.GWN_I_MOMENTS, G.GWN_I_MULTIPOLE):
            a, b = G.gwn_inspect(hd, what), G.gwn_inspect(hh, what)
            assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max(), (what, np.abs(a - b).max(), np.abs(b).max())
        fd, fh = G.gwn_inspect(hd, G.GWN_I_FARBETA), G.gwn_inspect(hh, G.GWN_I_FARBETA)
        assert np.abs(fd - fh).max() <= 1e-6 * np.abs(fh).max()
    finally:
        G.gwn_free(hd)
        G.gwn_free(hh)
