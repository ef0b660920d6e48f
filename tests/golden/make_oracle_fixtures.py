"""Writes the oracle regression fixtures in this folder.

These are not pins: the pins of the oracle are the closed forms, invariants
and brute-force checks in tests/test_oracle*.py.  The fixtures freeze the
oracle's own values on two small seeded cases so that any later change to
its arithmetic shows up as a test failure and has to be justified.  Only
oracle/ and the seeded generators are called.

    python tests/golden/make_oracle_fixtures.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from oracle import oracle  # noqa: E402
from paper_2605_19200_amd import workloads as W  # noqa: E402


def cases():
    curves, q = W.config1()
    yield "star_loop_64", "2d", curves, q[:64]
    P = W.Patches3D.from_list([(cp, w, []) for cp, w in W.bodies(0, [("torus", (0, 0, 0), 1.0)], disp=0.02)][:64])
    lo, hi = P.bbox()
    q3 = W.bbox_queries_uniform(W.Rng(11, "golden/torus"), lo, hi, 16, 1.2)
    yield "torus_patches_16", "3d", P, q3


def main():
    for name, kind, geom, q in cases():
        w = oracle.gwn2d(geom, q) if kind == "2d" else oracle.gwn3d(geom, q)
        path = os.path.join(HERE, f"oracle_{name}.txt")
        with open(path, "w") as fh:
            fh.write(f"# oracle values, {name}: columns = query coordinates, w (written by make_oracle_fixtures.py)\n")
            for row, v in zip(q, w):
                fh.write(" ".join(f"{x:.17g}" for x in row) + f" {v:.17g}\n")
        print("wrote", path)


if __name__ == "__main__":
    main()
