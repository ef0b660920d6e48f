"""The arctangent that the 2D kernel uses for the chord-angle sum: its
coefficient table in query.hip must be the one atan_coeffs.py derives, and
the kernel's octant reduction around it must reproduce atan2 to ~1e-15 over
every octant, at the axes and diagonals and at extreme magnitudes.  The
reduction is emulated here in float64 with an exact division in place of
the kernel's refined hardware reciprocal (the GPU parity tests cover the
device arithmetic)."""
import importlib.util
import math
import pathlib
import re

import numpy as np

CSRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2605_19200_amd" / "csrc"


def kernel_table():
    src = (CSRC / "query.hip").read_text()
    m = re.search(r"__constant__ double kAtanP\[(\d+)\] = \{([^}]*)\};", src)
    assert m, "kAtanP table not found in query.hip"
    vals = [float(v) for v in m.group(2).replace("\n", " ").split(",") if v.strip()]
    assert len(vals) == int(m.group(1))
    return np.array(vals)


def generator():
    spec = importlib.util.spec_from_file_location("atan_coeffs", CSRC / "atan_coeffs.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def fast_atan2(y, x, P):
    """The kernel's reduction: t = min/max in [0, 1], (t - 1) / (t + 1)
    above tan(pi/8), the odd polynomial r P(r^2), then the octant."""
    ax, ay = np.abs(x), np.abs(y)
    mn, mx = np.minimum(ax, ay), np.maximum(ax, ay)
    big = mn > 0.41421356237309503 * mx
    num = np.where(big, mn - mx, mn)
    den = np.where(big, mn + mx, mx)
    r = num / den
    s2 = r * r
    p = np.full_like(r, P[-1])
    for c in P[-2:0:-1]:
        p = p * s2 + c
    a = (r * s2) * p + r * P[0]
    a = np.where(big, a + 0.78539816339744831, a)
    a = np.where(ay > ax, 1.5707963267948966 - a, a)
    a = np.where(x < 0.0, 3.1415926535897931 - a, a)
    return np.copysign(a, y)


def test_table_matches_its_generator():
    gen = generator()
    ours = kernel_table()
    fresh = gen.coefficients()
    assert ours.shape == fresh.shape
    assert np.allclose(ours, fresh, rtol=1e-14, atol=0.0)
    assert gen.max_error(ours) < 1e-15


def test_reduction_matches_atan2_everywhere():
    P = kernel_table()
    rng = np.random.default_rng(11)
    ang = rng.uniform(-math.pi, math.pi, 200_000)
    rad = 10.0 ** rng.uniform(-300, 300, ang.size)
    x, y = rad * np.cos(ang), rad * np.sin(ang)
    # axes, diagonals and the tan(pi/8) switch, both signs
    special = []
    for t in (0.0, 0.41421356237309503, 0.41421356237309503 * (1 + 1e-15), 1.0):
        for sx in (1.0, -1.0):
            for sy in (1.0, -1.0):
                special += [(sy * t, sx * 1.0), (sy * 1.0, sx * t)]
    sy_, sx_ = np.array(special).T
    x = np.concatenate([x, sx_])
    y = np.concatenate([y, sy_])
    keep = (x != 0.0) | (y != 0.0)
    x, y = x[keep], y[keep]
    err = np.abs(fast_atan2(y, x, P) - np.arctan2(y, x))
    assert err.max() < 2e-15, err.max()
    # the +0 / -0 convention the chord sum relies on: atan2(+0, x < 0) = +pi
    assert fast_atan2(np.array([0.0]), np.array([-1.0]), P)[0] == math.pi
