"""Host preprocessing of 3D models (Alg. 1: subdivision, Green-scattered
Gauss-Legendre moments, BVH, up-sweep, centering) checked on the CPU."""
import math

import numpy as np
import pytest

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import workloads as W
from tests.test_oracle3d import bilinear_patch, patches


def build(P, **kw):
    h = G.gwn_build3d(P, G.gwn_default_params(device=-1, **kw))
    out = {k: G.gwn_inspect(h, v) for k, v in [("summary", G.GWN_I_SUMMARY), ("leaves", G.GWN_I_LEAVES),
                                                ("nodes", G.GWN_I_NODES), ("M", G.GWN_I_MOMENTS),
                                                ("U", G.GWN_I_UNCENTERED)]}
    G.gwn_free(h)
    return out


@pytest.mark.parametrize("centre,radius", [((0, 0, 0), 1.0), ((1.0, 2.0, -0.5), 0.6)])
def test_closed_sphere_moment_identities(centre, radius):
    """Divergence theorem on a closed outward surface: int n = 0,
    int x_i n_j = V delta_ij, int x_i x_j n_k = V (delta_ik c_j + delta_jk c_i)."""
    P = W.Patches3D.from_list([(cp, w, []) for cp, w in
                               W.bodies(0, [("sphere", centre, radius)], disp=0.0)])
    B = build(P)
    U = B["U"][0]
    V = 4 / 3 * math.pi * radius ** 3
    c = np.array(centre, float)
    I = np.eye(3)
    assert np.abs(U[:3]).max() < 1e-10
    assert np.abs(U[3:12].reshape(3, 3) - V * I).max() < 1e-9 * max(1, V)
    ref = V * (I[:, None, :] * c[None, :, None] + I[None, :, :] * c[:, None, None])
    assert np.abs(U[12:].reshape(3, 3, 3) - ref).max() < 1e-9 * max(1, np.abs(ref).max())
    # the centroid of a sphere's surface is its centre
    assert np.abs(B["nodes"][0, 3:6] - c).max() < 1e-9


def test_subdivision_of_large_patch_and_moment_sum():
    big = bilinear_patch((0, 0, 0), (4, 0, 0.5), (4, 4, 0), (0, 4, 0.3))
    small = bilinear_patch((1, 1, 1), (1.2, 1, 1), (1.2, 1.2, 1), (1, 1.2, 1))
    B = build(patches((*big, []), (*small, [])))
    leaves = B["leaves"]
    diag = B["summary"][0][5]
    pts = leaves[:, 1:].reshape(-1, 16, 4)
    eu = pts[..., :3] / pts[..., 3:4]
    d = np.linalg.norm(eu.max(1) - eu.min(1), axis=1)
    assert np.all(d < 0.1 * diag)
    assert np.sum(leaves[:, 0] == 0) > 4 and np.sum(leaves[:, 0] == 1) == 1
    # moments of the subdivided big patch equal those of the unsplit patch
    whole = build(patches((*big, [])), max_diag_frac=10.0)["U"][0]
    split = build(patches((*big, [])))["U"][0]
    assert np.abs(split - whole).max() < 1e-10 * np.abs(whole).max()


def leaf_patches(P, **kw):
    """The leaves of a host-only build as a patch set of their own: each
    leaf's control net and its clipped trim loops in its own square."""
    h = G.gwn_build3d(P, G.gwn_default_params(device=-1, **kw))
    leaves = G.gwn_inspect(h, G.GWN_I_LEAVES)
    trims = G.gwn_inspect(h, G.GWN_I_LEAF_TRIMS)
    G.gwn_free(h)
    items = []
    for l in range(leaves.shape[0]):
        net = leaves[l, 1:].reshape(4, 4, 4)
        cp, wt = net[..., :3] / net[..., 3:4], net[..., 3]
        mine = trims[trims[:, 0] == l, 1:].reshape(-1, 3, 3)
        tl = [(c[:, :2] / c[:, 2:3], c[:, 2].copy()) for c in mine]
        items.append((cp, wt, tl))
    return W.Patches3D.from_list(items), leaves[:, 0].astype(int)


def test_trimmed_patch_split_and_validation():
    cp, w = bilinear_patch((0, 0, 0), (4, 0, 0), (4, 4, 0), (0, 4, 0))
    trims = W.square_trim() + W.circle_trim((0.5, 0.5), 0.2)
    small = bilinear_patch((5, 5, 5), (5.1, 5, 5), (5.1, 5.1, 5), (5, 5.1, 5))
    B = build(patches((cp, w, trims), (*small, [])))
    assert np.sum(B["leaves"][:, 0] == 0) > 4 and np.sum(B["leaves"][:, 0] == 1) == 1
    # flat square with a hole: int n dA = (area of square - hole) * normal,
    # exact up to quadrature, whether the patch is split or not
    for frac in (10.0, 0.1):
        U = build(patches((cp, w, trims)), max_diag_frac=frac)["U"][0]
        assert abs(U[2] - 16 * (1 - math.pi * 0.04)) < 1e-9 and abs(U[0]) < 1e-12 and abs(U[1]) < 1e-12
    for bad in ["open", "outside", "degree"]:
        t = [(uv.copy(), wt.copy()) for uv, wt in trims]
        if bad == "open":
            t = t[:3]
        if bad == "outside":
            t[5] = (t[5][0] + 0.9, t[5][1])
        if bad == "degree":
            t[0] = (np.array([[0, 0], [0.3, 0], [0.6, 0], [1, 0.0]]), np.ones(4))
        with pytest.raises(G.GwnError) as ei:
            build(patches((cp, w, t)))
        assert ei.value.status == G.GWN_EINVAL


def test_trimmed_subdivision_leaves_sum_to_the_original(oracle):
    """Subdivision leaves the ground-truth GWN unchanged (Sec. 4.2): the
    leaves of split trimmed patches -- control nets cut by de Casteljau,
    trim loops clipped to each half and mapped to its square, halves with
    nothing visible dropped -- are closed valid loops, and the oracle's sum
    over them equals its value for the original patches.  Cases: a warped
    patch with three holes (one of them crossed by the first cuts), a
    sphere patch with a hole, and a patch whose visible region is a disk
    only (so some halves are empty)."""
    rng = W.Rng(37, "clip")
    cp, w = bilinear_patch((0, 0, 0), (2, 0, 0.3), (2, 2, -0.2), (0, 2, 0.1), w=[[1.0, 1.4], [0.8, 1.2]])
    cp = cp + 0.15 * rng.uniform((4, 4, 3), -1, 1)
    holes = W.square_trim() + W.circle_trim((0.5, 0.62), 0.12) + W.circle_trim((0.25, 0.25), 0.1) + \
        W.circle_trim((0.72, 0.3), 0.15)
    sph = W.bodies(0, [("sphere", (3, 0, 0), 1.0)], disp=0.0)[200]
    disk_only = bilinear_patch((0, 3, 0), (1, 3, 0), (1, 4, 0.4), (0, 4, 0.2))
    P = patches((cp, w, holes), (*sph, W.square_trim() + W.circle_trim((0.4, 0.55), 0.3)),
                (*disk_only, W.circle_trim((0.3, 0.35), 0.2, ccw=True)))
    L, src = leaf_patches(P, max_diag_frac=0.02)
    counts = np.bincount(src, minlength=3)
    assert np.all(counts >= 8), counts
    lo, hi = P.bbox()
    q = np.concatenate([W.bbox_queries_uniform(rng, lo, hi, 24, 1.2),
                        W.near_surface_queries(P, rng, 24, t_max=1e-3)])
    eps = oracle.default_eps_on(lo, hi)
    ref = oracle.gwn3d(P, q, eps_on=eps)
    got = oracle.gwn3d(L, q, eps_on=eps)
    assert np.abs(got - ref).max() < 1e-10, np.abs(got - ref).max()


def test_cad_assembly_trimmed_patches_are_split():
    """Every patch of the CAD assembly is trimmed; at the presets'
    subdivision they are split like untrimmed ones (more leaves than
    patches), and the root's uncentered moments -- sums over the leaves'
    visible parts -- equal those of the unsplit build."""
    from paper_2605_19200_amd import presets
    P = W.cad_assembly(4, n_bodies=6)
    frac = presets.FP64_3D["max_diag_frac"]
    whole = build(P, max_diag_frac=10.0)
    split = build(P, max_diag_frac=frac)
    assert split["summary"][0][2] > 1.3 * P.n, (split["summary"][0][2], P.n)
    # uncentered moments of the root are sums over the leaves: unchanged
    Uw, Us = whole["U"][0], split["U"][0]
    assert np.abs(Us - Uw).max() < 1e-9 * np.abs(Uw).max()


def test_upsweep_and_centering_3d():
    P, _ = W.config3(grid=0)
    P = P.subset(range(0, 4096, 37))
    B = build(P)
    nodes, U, M = B["nodes"], B["U"], B["M"]

    def subtree(i):
        if nodes[i, 0]:
            return [i]
        return subtree(int(nodes[i, 1])) + subtree(int(nodes[i, 2]))
    for i in range(0, nodes.shape[0], 5):
        if nodes[i, 0]:
            continue
        ref = sum(U[j] for j in subtree(i))
        assert np.allclose(U[i], ref, rtol=1e-12, atol=1e-14)
        c = nodes[i, 3:6]
        U0, U1, U2 = U[i][:3], U[i][3:12].reshape(3, 3), U[i][12:].reshape(3, 3, 3)
        M1 = U1 - np.outer(c, U0)
        M2 = U2 - c[:, None, None] * U1[None, :, :] - c[None, :, None] * U1[:, None, :] \
            + c[:, None, None] * c[None, :, None] * U0[None, None, :]
        assert np.allclose(M[i][3:12], M1.ravel(), atol=1e-12)
        assert np.allclose(M[i][12:], M2.ravel(), atol=1e-12)


def multipole_omega(mp, s, order):
    """Solid angle from the GWN_I_MULTIPOLE record (1/r, 0, scaled N_l^m)
    at s = q - c, truncated at degree order + 1."""
    L = order + 1
    x, y, z = np.asarray(s) * mp[0]
    inv2 = 1.0 / (x * x + y * y + z * z)
    xi = complex(x, y)
    I = {}
    for m in range(L + 1):
        I[m, m] = np.sqrt(inv2) if m == 0 else I[m - 1, m - 1] * (2 * m - 1) * xi * inv2
        for l in range(m + 1, L + 1):
            prev2 = I.get((l - 2, m), 0.0)
            I[l, m] = ((2 * l - 1) * z * I[l - 1, m] - (l + m - 1) * (l - m - 1) * prev2) * inv2
    om = 0.0
    for l in range(1, L + 1):
        for m in range(l + 1):
            k = l * (l + 1) // 2 - 1 + m
            N = complex(mp[2 + 2 * k], mp[3 + 2 * k])
            om += (1 if m == 0 else 2) * (I[l, m] * N).real
    return om


def cartesian_omega(M, s, order):
    """Order 0..2 Taylor term of the solid angle (Eq. taylor) with the centred
    Cartesian moments M0[3], M1[3x3], M2[3x3x3] at s = c - q."""
    s = np.asarray(s)
    r = np.linalg.norm(s)
    I = np.eye(3)
    g = s / r ** 3
    dg = I / r ** 3 - 3 * np.outer(s, s) / r ** 5
    ddg = -3 * (I[None, :, :] * s[:, None, None] + I[:, None, :] * s[None, :, None] + I[:, :, None] * s[None, None, :]) \
        / r ** 5 + 15 * np.einsum("i,j,k->ijk", s, s, s) / r ** 7
    om = g @ M[:3]
    if order >= 1:
        om += np.einsum("jk,jk->", dg, M[3:12].reshape(3, 3))
    if order >= 2:
        om += 0.5 * np.einsum("ijk,ijk->", ddg, M[12:].reshape(3, 3, 3))
    return om


def test_multipole_moments_equal_cartesian_and_converge(oracle):
    """The harmonic form of the far field equals the paper's Cartesian order
    0-2 expansion (independent moment computations) and converges to the
    oracle's direct value as the order grows."""
    P, _ = W.config3(grid=0)
    P = P.subset(range(0, 4096, 29))
    h = G.gwn_build3d(P, G.gwn_default_params(device=-1, max_diag_frac=10.0))
    nodes = G.gwn_inspect(h, G.GWN_I_NODES)
    M = G.gwn_inspect(h, G.GWN_I_MOMENTS)
    MP = G.gwn_inspect(h, G.GWN_I_MULTIPOLE)
    leaves = G.gwn_inspect(h, G.GWN_I_LEAVES)
    G.gwn_free(h)

    def subtree(i):
        if nodes[i, 0]:
            return [int(leaves[int(nodes[i, 1]), 0])]
        return subtree(int(nodes[i, 1])) + subtree(int(nodes[i, 2]))
    rng = W.Rng(71, "mpole")
    checked = 0
    for i in range(1, nodes.shape[0], 7):
        if nodes[i, 0] or len(subtree(i)) < 3:
            continue
        c, r = nodes[i, 3:6], nodes[i, 6]
        d = rng.uniform(3, -1, 1)
        q = c + 5.0 * r * d / np.linalg.norm(d)
        direct = 4 * math.pi * oracle.gwn3d(P.subset(subtree(i)), q[None])[0]
        scale = max(abs(direct), np.abs(M[i][:3]).sum() / (5 * r) ** 2)
        for p in range(3):
            assert abs(multipole_omega(MP[i], q - c, p) - cartesian_omega(M[i], c - q, p)) < 1e-11 * scale, (i, p)
        errs = [abs(multipole_omega(MP[i], q - c, p) - direct) for p in (0, 2, 4, 6)]
        assert errs[3] <= errs[2] + 1e-9 * scale and errs[3] < 0.05 * errs[1] + 1e-9 * scale, (i, errs)
        checked += 1
        if checked == 6:
            break
    assert checked == 6
