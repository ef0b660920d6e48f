"""Writes oracle values for seeded subsets of the full-size workloads.

The GPU parity tests run the engine on the whole workload (every patch, every
query) and compare it with these values row by row.  Only oracle/ and the
seeded generators are called; nothing here touches the engine.

  cad_assembly_1m   39 bodies, 19,968 trimmed rational bicubic patches with
                    1-3 holes each; 1,000,000 queries, half within 1e-2 of
                    the surface.  512 of the near-surface rows and 512 of the
                    uniform rows, chosen by a seeded permutation.
  bodies_scene      8 bodies, 4,096 patches (30 % with one hole); 512 seeded
                    rows of the 128^3 grid, and 512 near-surface points
                    (within 1e-2 of the surface) drawn by their own stream.
  drawing_1024      the 2D SVG-like drawing (19,000 curves); 1,024 seeded
                    rows of its 1024^2 grid (the parameter studies' and the
                    headline benchmark's workload).

Each file holds one row per query: the row index in the workload's query
array (-1 for the separate near-surface points), the query coordinates and
the oracle's w.  The header records the oracle's non-convergence report.
The direct 3D sum costs about 28 s per query per thread on the assembly, so
the run is long; it writes every finished chunk and resumes from the rows a
file already holds.

    python tests/golden/make_fullsize_fixtures.py [cad|bodies ...] [--threads N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from oracle import oracle  # noqa: E402
from paper_2605_19200_amd import workloads as W  # noqa: E402

N_PER_KIND = 512
CHUNK = 32


def cad_rows(n_query=1_000_000):
    """Rows of the assembly's query array: near-surface ones are those whose
    pre-shuffle index falls in the first half (see workloads.config4)."""
    perm = W.Rng(4, "cfg4/shuffle").permutation(n_query)
    near_rows = np.nonzero(perm < n_query // 2)[0]
    uni_rows = np.nonzero(perm >= n_query // 2)[0]
    pick = W.Rng(404, "fixture/cad")
    a = near_rows[pick.permutation(near_rows.size)[:N_PER_KIND]]
    b = uni_rows[pick.permutation(uni_rows.size)[:N_PER_KIND]]
    return np.sort(a), np.sort(b)


def case_cad():
    P, q = W.config4()
    a, b = cad_rows(q.shape[0])
    rows = np.concatenate([a, b])
    return P, rows, q[rows], f"{N_PER_KIND} near-surface + {N_PER_KIND} uniform rows of the 1M queries"


def bodies_near():
    P, _ = W.config3(grid=0)
    return W.near_surface_queries(P, W.Rng(303, "fixture/bodies/near"), N_PER_KIND)


def case_bodies():
    P, q = W.config3()
    rows = np.sort(W.Rng(303, "fixture/bodies/grid").permutation(q.shape[0])[:N_PER_KIND])
    near = bodies_near()
    allrows = np.concatenate([rows, np.full(N_PER_KIND, -1)])
    return P, allrows, np.concatenate([q[rows], near]), \
        f"{N_PER_KIND} rows of the 128^3 grid + {N_PER_KIND} near-surface points (row -1)"


def drawing_rows(n_query=1024 * 1024):
    return np.sort(W.Rng(202, "fixture/drawing").permutation(n_query)[:2 * N_PER_KIND])


def case_drawing():
    C, q = W.config2()
    rows = drawing_rows(q.shape[0])
    return C, rows, q[rows], f"{2 * N_PER_KIND} seeded rows of the 1024^2 grid"


CASES = {"cad": ("oracle_cad_assembly_1m.txt", case_cad), "bodies": ("oracle_bodies_scene.txt", case_bodies),
         "drawing": ("oracle_drawing_1024.txt", case_drawing)}


def load(path):
    """(rows, q, w, header dict) of a fixture file, possibly partial; q has
    the workload's dimension (2 or 3 coordinates per row)."""
    hdr = {}
    data = []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                if ":" in line:
                    k, v = line[1:].split(":", 1)
                    hdr[k.strip()] = v.strip()
                continue
            data.append([float(x) for x in line.split()])
    dim = int(hdr.get("dim", 3))
    d = np.array(data).reshape(-1, dim + 2)
    return d[:, 0].astype(np.int64), d[:, 1:1 + dim], d[:, 1 + dim], hdr


def write(name, threads):
    fname, make = CASES[name]
    path = os.path.join(HERE, fname)
    P, rows, q, what = make()
    done = 0
    unconv, bound = 0, 0.0
    if os.path.exists(path):
        r0, q0, _, hdr = load(path)
        done = r0.size
        assert np.array_equal(r0, rows[:done]) and np.array_equal(q0, q[:done]), "fixture does not match the inputs"
        unconv = int(hdr.get("oracle unconverged panels", 0))
        bound = float(hdr.get("oracle max error bound", 0.0))
    eps_on = oracle.default_eps_on(*P.bbox())
    dim = q.shape[1]
    body = []
    if done:
        with open(path) as fh:
            body = [ln for ln in fh if not ln.startswith("#")]
    t0 = time.time()
    for s in range(done, rows.size, CHUNK):
        e = min(rows.size, s + CHUNK)
        if dim == 2:
            w = oracle.gwn2d(P, q[s:e], eps_on=eps_on, threads=threads)
        else:
            w = oracle.gwn3d(P, q[s:e], eps_on=eps_on, threads=threads)
        unconv += oracle.last_unconverged
        bound = max(bound, oracle.last_errbound)
        body += [f"{int(r)} " + " ".join(f"{x:.17g}" for x in qq) + f" {v:.17g}\n"
                 for r, qq, v in zip(rows[s:e], q[s:e], w)]
        with open(path + ".tmp", "w") as fh:
            fh.write(f"# oracle values on a full-size workload (written by make_fullsize_fixtures.py): {name}\n")
            fh.write(f"# subset: {what}\n")
            fh.write(f"# {'curves' if dim == 2 else 'patches'}: {P.n}\n")
            fh.write(f"# dim: {dim}\n")
            fh.write(f"# eps_on: {eps_on:.17g}\n")
            fh.write(f"# oracle unconverged panels: {unconv}\n")
            fh.write(f"# oracle max error bound: {bound:.3e}\n")
            fh.write("# columns: row, x, y, w\n" if dim == 2 else "# columns: row, x, y, z, w\n")
            fh.writelines(body)
        os.replace(path + ".tmp", path)
        print(f"[{name}] {e}/{rows.size} rows, {time.time() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=["bodies", "cad", "drawing"])
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    for name in a.cases:
        write(name, a.threads)


if __name__ == "__main__":
    main()
