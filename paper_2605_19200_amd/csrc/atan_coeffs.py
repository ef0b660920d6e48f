"""Coefficients of the kernel's arctangent on the reduced range.

atan(r) = r * P(r^2) for |r| <= tan(pi/8), P of degree 9, obtained by
Chebyshev interpolation of atan(sqrt(s))/sqrt(s) on s in [0, tan^2(pi/8)] at
400 nodes and conversion to monomials in s.  Prints the table used in
query.hip and the maximum absolute error of r * P(r^2) against numpy's
arctan on a dense grid of the reduced range (about 5e-16).
"""
from math import comb

import numpy as np
from numpy.polynomial import chebyshev as C

DEG = 9


def coefficients(deg: int = DEG) -> np.ndarray:
    smax = np.tan(np.pi / 8) ** 2
    x = np.cos(np.pi * (np.arange(400) + 0.5) / 400)
    s = (x + 1) / 2 * smax
    r = np.sqrt(s)
    f = np.arctan(r) / r
    pm = C.cheb2poly(C.chebfit(x, f, deg))          # polynomial in x = 2 s / smax - 1
    a, b = 2 / smax, -1.0
    ps = np.zeros(deg + 1)
    for j, cj in enumerate(pm):
        for i in range(j + 1):
            ps[i] += cj * comb(j, i) * a ** i * b ** (j - i)
    return ps


def max_error(ps: np.ndarray) -> float:
    rr = np.linspace(-np.tan(np.pi / 8), np.tan(np.pi / 8), 400001)
    val = np.zeros_like(rr)
    for c in ps[::-1]:
        val = val * rr * rr + c
    return float(np.abs(rr * val - np.arctan(rr)).max())


if __name__ == "__main__":
    ps = coefficients()
    print("__constant__ double kAtanP[%d] = {" % len(ps))
    print(",\n".join("    %.17g" % c for c in ps) + "};")
    print("// max |r P(r^2) - atan(r)| = %.3g" % max_error(ps))
