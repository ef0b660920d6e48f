"""Error-budgeted far test (far_tol > 0): each cluster's own factor beta_c
must keep the truncation error of its order-p expansion within the budget at
every point with ||q - c|| > beta_c r.  Checked on the CPU from host-only
builds.  2D: the exact angle of the cluster's chords (atan2 per chord, the
plain definition) against the truncated Laurent series of the chord integral,
evaluated just outside beta_c r in many directions.  3D: the oracle's direct
solid angle of the cluster's patches against its order-p multipole series."""
import numpy as np
import pytest

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import workloads as W


def _host(curves, **kw):
    return G.gwn_build2d(curves, G.gwn_default_params(device=-1, **kw))


def _subtree_ends(nodes):
    n = nodes.shape[0]
    end = np.zeros(n, dtype=np.int64)
    for i in range(n - 1, -1, -1):
        end[i] = i + 1 if nodes[i, 0] else end[int(nodes[i, 2])]
    return end


def _chords(leaves, nodes, end, i):
    idx = [int(nodes[j, 1]) for j in range(i, end[i]) if nodes[j, 0]]
    h = leaves[idx, 1:].reshape(-1, 4, 3)
    a = (h[:, 0, 0] + 1j * h[:, 0, 1]) / h[:, 0, 2]
    b = (h[:, 3, 0] + 1j * h[:, 3, 1]) / h[:, 3, 2]
    return a, b


def _exact_turns(a, b, q):
    """Angle subtended by the chords a -> b at q, in turns."""
    return np.angle((b - q) / (a - q)).sum() / (2 * np.pi)


def _series_turns(a, b, c, q, p):
    """Order-p Laurent truncation of the same chord integral about c:
    integral dz / (z - q) = -sum_k m_k / (q - c)^(k+1), m_k = integral (z - c)^k dz."""
    u = 1.0 / (q - c)
    s = 0.0
    for k in range(p + 1):
        m = (((b - c) ** (k + 1) - (a - c) ** (k + 1)) / (k + 1)).sum()
        s += m * u ** (k + 1)
    return -s.imag / (2 * np.pi)


@pytest.mark.parametrize("order,tol", [(2, 1e-7), (6, 1e-9), (12, 1e-10)])
def test_bound_holds_outside_beta_c(order, tol):
    curves = W.star_loop(seed=3, n_curves=64)
    h = _host(curves, taylor_order=order, far_tol=tol, max_diag_frac=0.05)
    nodes = G.gwn_inspect(h, G.GWN_I_NODES)
    leaves = G.gwn_inspect(h, G.GWN_I_LEAVES)
    fb = G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0]
    G.gwn_free(h)
    end = _subtree_ends(nodes)
    internal = np.flatnonzero(nodes[:, 0] == 0)
    assert internal.size > 10
    assert np.all(fb[internal] >= 2.0) and np.all(fb[nodes[:, 0] == 1] == 0.0)
    ang = np.linspace(0.0, 2 * np.pi, 48, endpoint=False)
    worst = 0.0
    checked = 0
    for i in internal:
        bc, r = fb[i], nodes[i, 6]
        if not np.isfinite(bc) or r <= 0:
            continue
        a, b = _chords(leaves, nodes, end, i)
        c = nodes[i, 3] + 1j * nodes[i, 4]
        for rad in (bc * r * (1 + 1e-9), 1.5 * bc * r):
            for t in ang:
                q = c + rad * np.exp(1j * t)
                err = abs(_exact_turns(a, b, q) - _series_turns(a, b, c, q, order))
                worst = max(worst, err / tol)
                checked += 1
    assert checked > 1000
    assert worst <= 1.0 + 1e-6, worst


def test_factor_follows_budget_and_order():
    curves = W.star_loop(seed=3, n_curves=64)
    fbs = {}
    for order, tol in [(4, 1e-6), (4, 1e-9), (12, 1e-9)]:
        h = _host(curves, taylor_order=order, far_tol=tol, max_diag_frac=0.05)
        fbs[(order, tol)] = G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0]
        nodes = G.gwn_inspect(h, G.GWN_I_NODES)
        G.gwn_free(h)
    internal = nodes[:, 0] == 0
    # a tighter budget or a lower order never lets a cluster be accepted closer
    assert np.all(fbs[(4, 1e-9)][internal] >= fbs[(4, 1e-6)][internal])
    assert np.all(fbs[(4, 1e-9)][internal] >= fbs[(12, 1e-9)][internal])
    assert np.any(fbs[(4, 1e-9)][internal] > fbs[(4, 1e-6)][internal])


def test_uniform_beta_without_budget_and_set_params():
    curves = W.star_loop(seed=3, n_curves=64)
    h = _host(curves, beta=3.5, taylor_order=8)
    nodes = G.gwn_inspect(h, G.GWN_I_NODES)
    fb = G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0]
    assert np.all(fb[nodes[:, 0] == 0] == 3.5)
    p = G.gwn_get_params(h)
    p.far_tol = 1e-8
    G.gwn_set_params(h, p)
    fb2 = G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0]
    assert not np.all(fb2[nodes[:, 0] == 0] == 3.5) and np.all(fb2[nodes[:, 0] == 0] >= 2.0)
    p.far_tol = -1.0
    with pytest.raises(G.GwnError):
        G.gwn_set_params(h, p)
    p.far_tol = float("nan")
    with pytest.raises(G.GwnError):
        G.gwn_set_params(h, p)
    G.gwn_free(h)


def _host3d(P, **kw):
    return G.gwn_build3d(P, G.gwn_default_params(device=-1, max_diag_frac=10.0, **kw))


@pytest.mark.parametrize("order,tol", [(2, 1e-6), (4, 1e-8), (6, 1e-9)])
def test_3d_estimate_holds_outside_beta_c(oracle, order, tol):
    """3D: beta_c comes from an estimate of the first two omitted harmonic
    degrees (with a factor 2), so the error of the order-p multipole series
    against the oracle's direct solid angle of the cluster's patches, just
    outside beta_c r and further out, stays within the budget."""
    from tests.test_hostbuild3d import multipole_omega
    P = W.config3(grid=0)[0].subset(range(0, 4096, 13))
    h = _host3d(P, taylor_order=order, far_tol=tol)
    nodes = G.gwn_inspect(h, G.GWN_I_NODES)
    MP = G.gwn_inspect(h, G.GWN_I_MULTIPOLE)
    leaves = G.gwn_inspect(h, G.GWN_I_LEAVES)
    fb = G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0]
    G.gwn_free(h)
    assert np.all(fb >= 1.5) and np.all(np.isfinite(fb))
    end = _subtree_ends(nodes)
    rng = W.Rng(17, "fartol3d")
    worst, checked = 0.0, 0
    for i in range(0, nodes.shape[0], 9):
        bc, r = fb[i], nodes[i, 6]
        if r <= 0:
            continue
        src = sorted({int(leaves[int(nodes[j, 1]), 0]) for j in range(i, end[i]) if nodes[j, 0]})
        c = nodes[i, 3:6]
        d = rng.uniform(48, -1.0, 1.0).reshape(16, 3)
        d /= np.linalg.norm(d, axis=1)[:, None]
        qs = np.concatenate([c + bc * r * (1 + 1e-9) * d, c + 1.5 * bc * r * d])
        direct = oracle.gwn3d(P.subset(src), qs)
        approx = np.array([multipole_omega(MP[i], q - c, order) for q in qs]) / (4 * np.pi)
        worst = max(worst, np.abs(direct - approx).max() / tol)
        checked += qs.shape[0]
    assert checked > 2000
    assert worst <= 1.0, worst


def test_3d_factor_follows_budget_and_order():
    P = W.config3(grid=0)[0].subset(range(0, 4096, 13))
    fbs = {}
    for order, tol in [(4, 1e-6), (4, 1e-9), (6, 1e-9)]:
        h = _host3d(P, taylor_order=order, far_tol=tol)
        fbs[(order, tol)] = G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0]
        G.gwn_free(h)
    assert np.all(fbs[(4, 1e-9)] >= fbs[(4, 1e-6)])
    assert np.any(fbs[(4, 1e-9)] > fbs[(4, 1e-6)])
    # one more order tightens most factors (an estimate, not a bound, so not all)
    assert np.mean(fbs[(6, 1e-9)] <= fbs[(4, 1e-9)]) > 0.9
    h = _host3d(P, taylor_order=6, beta=4.0)
    assert np.all(G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0] == 4.0)
    p = G.gwn_get_params(h)
    p.far_tol = 1e-9
    G.gwn_set_params(h, p)
    assert np.array_equal(G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0], fbs[(6, 1e-9)])
    # a loose budget floors at 1.5
    p.far_tol = 1.0
    G.gwn_set_params(h, p)
    assert np.all(G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0] == 1.5)
    G.gwn_free(h)


def test_loose_budget_floors_at_two_and_tight_budget_is_finite():
    curves = W.star_loop(seed=3, n_curves=64)
    for tol, check in ((1.0, lambda b: np.all(b == 2.0)), (1e-15, lambda b: np.all(np.isfinite(b)) and np.all(b > 2.0))):
        h = _host(curves, taylor_order=12, far_tol=tol, max_diag_frac=0.05)
        nodes = G.gwn_inspect(h, G.GWN_I_NODES)
        fb = G.gwn_inspect(h, G.GWN_I_FARBETA)[:, 0]
        G.gwn_free(h)
        assert check(fb[nodes[:, 0] == 0]), (tol, fb[nodes[:, 0] == 0].min(), fb[nodes[:, 0] == 0].max())
