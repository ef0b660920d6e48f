"""Host preprocessing of 2D models (Alg. 1: subdivision, moments, BVH,
up-sweep, centering) checked on the CPU against independent computations."""
import math

import numpy as np
import pytest

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import workloads as W


def build(curves, **kw):
    h = G.gwn_build2d(curves, G.gwn_default_params(device=-1, **kw))
    out = {k: G.gwn_inspect(h, v) for k, v in [("summary", G.GWN_I_SUMMARY), ("leaves", G.GWN_I_LEAVES),
                                                ("nodes", G.GWN_I_NODES), ("M", G.GWN_I_MOMENTS),
                                                ("U", G.GWN_I_UNCENTERED)]}
    G.gwn_free(h)
    return out


def leaf_points(leaves):
    h = leaves[:, 1:].reshape(-1, 4, 3)
    return h[:, :, :2] / h[:, :, 2:3]


def chord_moments(a, b):
    d = b - a
    N = np.array([d[1], -d[0]])
    U0 = N
    U1 = np.outer(a + d / 2, N)
    S = np.outer(a, a) + (np.outer(a, d) + np.outer(d, a)) / 2 + np.outer(d, d) / 3
    U2 = S[:, :, None] * N[None, None, :]
    return np.concatenate([U0, U1.ravel(), U2.ravel()])


def test_tree_structure_and_subdivision():
    curves, _ = W.config1()
    B = build(curves)
    nodes, leaves = B["nodes"], B["leaves"]
    n_leaves = leaves.shape[0]
    assert nodes.shape[0] == 2 * n_leaves - 1
    seen = []
    for i, nd in enumerate(nodes):
        if nd[0]:
            seen.append(int(nd[1]))
        else:
            l, r = int(nd[1]), int(nd[2])
            assert l == i + 1 and r > l
            for ch in (l, r):   # child AABB inside parent AABB
                assert np.all(nodes[ch, 7:9] >= nd[7:9] - 1e-15) and np.all(nodes[ch, 10:12] <= nd[10:12] + 1e-15)
    assert sorted(seen) == list(range(n_leaves))
    # 10% rule: every leaf AABB diagonal below 10% of the model diagonal
    diag = B["summary"][0][5]
    P = leaf_points(leaves)
    d = np.hypot(*(P.max(1) - P.min(1)).T)
    assert np.all(d < 0.1 * diag)
    # leaves of each source curve chain from its first to its last point
    for src in range(curves.n):
        idx = np.nonzero(leaves[:, 0] == src)[0]
        pts = P[idx]
        p, w = curves.curve(src)
        starts = {tuple(np.round(x, 12)) for x in pts[:, 0]}
        ends = {tuple(np.round(x, 12)) for x in pts[:, 3]}
        assert tuple(np.round(p[0], 12)) in starts and tuple(np.round(p[-1], 12)) in ends
        assert len(starts - ends) == 1 and len(ends - starts) == 1


def test_moments_upsweep_and_centering():
    curves, _ = W.config2(grid=4, n_groups=3)
    B = build(curves)
    nodes, leaves, U, M = B["nodes"], B["leaves"], B["U"], B["M"]
    P = leaf_points(leaves)
    leafU = np.array([chord_moments(P[l, 0], P[l, 3]) for l in range(P.shape[0])])
    # per-node recompute from the leaves of its subtree
    def subtree(i):
        if nodes[i, 0]:
            return [int(nodes[i, 1])]
        return subtree(int(nodes[i, 1])) + subtree(int(nodes[i, 2]))
    for i in range(0, nodes.shape[0], 7):
        ls = subtree(i)
        ref = leafU[ls].sum(0)
        assert np.allclose(U[i], ref, atol=1e-12, rtol=1e-12)
        c = nodes[i, 3:5]
        # centred moments from the definition: int (x - c) n, int (x - c)(x - c) n
        refM = np.zeros(14)
        for l in ls:
            refM += chord_moments(P[l, 0] - c, P[l, 3] - c)
        assert np.allclose(M[i], refM, atol=1e-12, rtol=1e-10)
        # centroid inside the AABB
        assert np.all(c >= nodes[i, 7:9] - 1e-15) and np.all(c <= nodes[i, 10:12] + 1e-15)


def test_closed_loop_identities():
    # divergence theorem on the closed chord polygon: int n = 0,
    # int x_i n_j = A delta_ij, int x_i x_j n_k = A (delta_ik c_j + delta_jk c_i)
    curves = W.Curves2D.from_list(W.circle_curves((0.3, -0.2), 0.7, 8))
    B = build(curves)
    root = B["U"][0]
    P = leaf_points(B["leaves"])
    poly = np.array([P[l, 0] for l in np.argsort(np.arctan2(P[:, 0, 1] + 0.2, P[:, 0, 0] - 0.3))])
    x, y = poly[:, 0], poly[:, 1]
    xs, ys = np.roll(x, -1), np.roll(y, -1)
    cr = x * ys - xs * y
    A = cr.sum() / 2
    cx = ((x + xs) * cr).sum() / (6 * A)
    cy = ((y + ys) * cr).sum() / (6 * A)
    c = np.array([cx, cy])
    assert np.allclose(root[:2], 0, atol=1e-14)
    assert np.allclose(root[2:6].reshape(2, 2), A * np.eye(2), atol=1e-14)
    U2 = root[6:].reshape(2, 2, 2)
    I = np.eye(2)
    ref = A * (I[:, None, :] * c[None, :, None] + I[None, :, :] * c[:, None, None])
    assert np.allclose(U2, ref, atol=1e-14)


def cart_taylor(M, c, q, order):
    """Order-p expansion of Eq. taylor with the derivative tensors of
    G2 = ln|x - q| / 2 pi written out (s = c - q)."""
    s = c - q
    r2 = s @ s
    k = 1 / (2 * math.pi)
    I = np.eye(2)
    g = k * s / r2
    dg = k * (I / r2 - 2 * np.outer(s, s) / r2 ** 2)
    ddg = k * (-2 * (I[None, :, :] * s[:, None, None] + I[:, None, :] * s[None, :, None]
                     + I[:, :, None] * s[None, None, :]) / r2 ** 2
               + 8 * np.einsum("i,j,k->ijk", s, s, s) / r2 ** 3)
    M0, M1, M2 = M[:2], M[2:6].reshape(2, 2), M[6:].reshape(2, 2, 2)
    out = M0 @ g
    if order >= 1:
        out += np.sum(M1 * dg)
    if order >= 2:
        out += 0.5 * np.sum(M2 * ddg)
    return out


def complex_taylor(M, c, q, order):
    """The same expansion in complex form: -Im sum m_k u^(k+1) / 2 pi."""
    M0, M1, M2 = M[:2], M[2:6].reshape(2, 2), M[6:].reshape(2, 2, 2)
    m0 = complex(-M0[1], M0[0])
    m1 = complex(-(M1[0, 1] + M1[1, 0]), M1[0, 0] - M1[1, 1])
    re2 = M2[0, 0, 0] - M2[1, 1, 0] - 2 * M2[0, 1, 1]
    im2 = M2[0, 0, 1] - M2[1, 1, 1] + 2 * M2[0, 1, 0]
    m2 = complex(-im2, re2)
    u = 1 / complex(q[0] - c[0], q[1] - c[1])
    ms = [m0, m1, m2][:order + 1]
    return -sum(m * u ** (k + 1) for k, m in enumerate(ms)).imag / (2 * math.pi)


def test_far_field_forms_agree_and_converge():
    curves, _ = W.config2(grid=4, n_groups=2)
    B = build(curves)
    nodes, M, leaves = B["nodes"], B["M"], B["leaves"]
    P = leaf_points(leaves)
    i = 1   # a large internal node
    while nodes[i, 0]:
        i += 1
    def subtree(j):
        if nodes[j, 0]:
            return [int(nodes[j, 1])]
        return subtree(int(nodes[j, 1])) + subtree(int(nodes[j, 2]))
    ls = subtree(i)
    c, r = nodes[i, 3:5], nodes[i, 6]
    errs = {p: [] for p in range(3)}
    for beta in [4.0, 8.0, 16.0, 32.0]:
        q = c + beta * r * np.array([math.cos(0.7), math.sin(0.7)])
        exact = sum(math.atan2(*(lambda a, b: (a[0] * b[1] - a[1] * b[0], a @ b))(P[l, 0] - q, P[l, 3] - q))
                    for l in ls) / (2 * math.pi)
        for p in range(3):
            ct, cx = cart_taylor(M[i], c, q, p), complex_taylor(M[i], c, q, p)
            assert abs(ct - cx) < 1e-13 * max(1, abs(ct))
            errs[p].append(abs(ct - exact))
    for p in range(3):   # error ~ beta^-(p+2): slope check over a factor 8 in beta
        ratio = errs[p][0] / errs[p][-1]
        assert ratio > 0.3 * 8 ** (p + 2), (p, errs[p])


def test_complex_moments_direct_and_high_order():
    """Per-node complex moments m_k = int (z - c)^k dz over the chords: equal
    to the complex form of the Cartesian order-2 moments for k <= 2, and to a
    direct sum over the subtree's chords for every stored order."""
    curves, _ = W.config2(grid=4, n_groups=3)
    h = G.gwn_build2d(curves, G.gwn_default_params(device=-1))
    nodes = G.gwn_inspect(h, G.GWN_I_NODES)
    M = G.gwn_inspect(h, G.GWN_I_MOMENTS)
    CM = G.gwn_inspect(h, G.GWN_I_COMPLEX)
    leaves = G.gwn_inspect(h, G.GWN_I_LEAVES)
    G.gwn_free(h)
    P = leaf_points(leaves)

    def subtree(i):
        if nodes[i, 0]:
            return [int(nodes[i, 1])]
        return subtree(int(nodes[i, 1])) + subtree(int(nodes[i, 2]))
    for i in range(0, nodes.shape[0], 11):
        if nodes[i, 0]:
            assert np.all(CM[i] == 0)
            continue
        c = complex(*nodes[i, 3:5])
        K = CM.shape[1] // 2
        ref = np.zeros(K, complex)
        for l in subtree(i):
            a, b = complex(*P[l, 0]) - c, complex(*P[l, 3]) - c
            for k in range(K):
                ref[k] += (b ** (k + 1) - a ** (k + 1)) / (k + 1)
        got = CM[i, 0::2] + 1j * CM[i, 1::2]
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-12 * scale + 1e-300
        Mi = M[i]
        M0, M1, M2 = Mi[:2], Mi[2:6].reshape(2, 2), Mi[6:].reshape(2, 2, 2)
        m0 = complex(-M0[1], M0[0])
        m1 = complex(-(M1[0, 1] + M1[1, 0]), M1[0, 0] - M1[1, 1])
        m2 = complex(-(M2[0, 0, 1] - M2[1, 1, 1] + 2 * M2[0, 1, 0]), M2[0, 0, 0] - M2[1, 1, 0] - 2 * M2[0, 1, 1])
        for k, mk in enumerate([m0, m1, m2]):
            assert abs(got[k] - mk) <= 1e-9 * max(abs(mk), np.abs(ref[:3]).max())
