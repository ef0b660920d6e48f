"""Parameter studies of the accelerated 2D query on the synthetic workloads,
after the paper's experiments on its own datasets:

  order_beta     max |dw| and time against (order, beta)      (Sec. 4.2, Fig. beta_sweep)
  subdivision    leaves, build and query time, error against the subdivision
                 threshold                                     (Sec. 4.1)
  far_tol        error, time and node visits against the error budget of the
                 per-cluster far test                          (Sec. 5, future work)
  disagreement   grid points whose rounded w differs from the rounded
                 reference, binned by the reference's fractional part
                                                               (Sec. 4.3)
  overlap        k nearly overlapping closed 15-gons: absolute and relative
                 error and misclassifications against k       (Sec. 4.3, Fig. overlap_demo)

The order, disagreement and overlap studies use the paper's 10 % subdivision
threshold and one far-field factor for all clusters; the subdivision study
runs the FP64 preset (order 12, error-budgeted far test); far_tol sweeps
the budget of that test.
The reference is the same engine with the far field switched off (beta =
1e8: every leaf evaluated directly), whose agreement with the FP64 oracle is
a GPU test of its own.  Each study prints one JSON line to stdout and its
progress to stderr.

    python -m paper_2605_19200_amd.studies [--only NAME ...]
"""
import argparse
import json
import sys
import time

import numpy as np

from . import gwn as G
from . import presets
from . import workloads as W


def _log(msg):
    print(f"[studies] {msg}", file=sys.stderr, flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _run(model, qd, reps=3):
    """Values and median wall time (ms) of `reps` queries after one warm-up."""
    import torch
    out, ins = model.query(qd)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        model.query(qd, out, ins)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return out.cpu().numpy(), float(np.median(ts) * 1e3)


def _reference(curves, qd):
    m = G.Model(curves, presets.params(presets.FP64_2D, beta=1e8, far_tol=0.0))
    w, ms = _run(m, qd, reps=1)
    m.close()
    return w, ms


def order_beta(grid=1024):
    curves, q = W.config2(grid=grid)
    qd = _dev(q)
    ref, ref_ms = _reference(curves, qd)
    _log(f"order_beta: reference {ref_ms:.1f} ms")
    rows = []
    for order in (0, 1, 2, 4, 8, 12, 16):
        for beta in (2.0, 3.0, 4.0, 6.0, 8.0, 16.0, 32.0, 64.0):
            m = G.Model(curves, presets.params(presets.FP64_2D, beta=beta, taylor_order=order, max_diag_frac=0.1, far_tol=0.0))
            w, ms = _run(m, qd)
            m.close()
            err = np.abs(w - ref)
            rows.append(dict(order=order, beta=beta, max_abs_dw=float(err.max()),
                             p99_abs_dw=float(np.quantile(err, 0.99)), ms=round(ms, 3),
                             queries_per_s=q.shape[0] / (ms * 1e-3)))
        _log(f"order_beta: order {order} done")
    return dict(study="order_beta", workload=f"SVG-like drawing, 19000 curves, {grid}^2 grid",
                reference_ms=round(ref_ms, 1), rows=rows)


def subdivision(grid=1024):
    curves, q = W.config2(grid=grid)
    qd = _dev(q)
    ref, _ = _reference(curves, qd)
    rows = []
    for frac in (1e9, 0.4, 0.2, 0.1, 0.05, 0.025, 0.0125):
        t = time.perf_counter()
        m = G.Model(curves, presets.params(presets.FP64_2D, max_diag_frac=frac))
        build_s = time.perf_counter() - t
        leaves = int(m.inspect(G.GWN_I_SUMMARY)[0][2])
        w, ms = _run(m, qd)
        m.close()
        rows.append(dict(max_diag_frac=None if frac >= 1e9 else frac, leaves=leaves, build_s=round(build_s, 3),
                         ms=round(ms, 3), max_abs_dw=float(np.abs(w - ref).max())))
        _log(f"subdivision: {frac} -> {leaves} leaves, {ms:.2f} ms")
    return dict(study="subdivision", workload=f"SVG-like drawing, 19000 curves, {grid}^2 grid, FP64 form "
                f"(order {presets.FP64_2D['taylor_order']}, far_tol {presets.FP64_2D['far_tol']})", rows=rows)


def far_tol(grid=1024):
    curves, q = W.config2(grid=grid)
    qd = _dev(q)
    ref, _ = _reference(curves, qd)
    rows = []
    for tol in (0.0, 3e-9, 1e-8, 2e-8, 5e-8, 1e-7):
        m = G.Model(curves, presets.params(presets.FP64_2D, far_tol=tol))
        w, ms = _run(m, qd)
        nodes = m.counters(qd)["nodes"]
        m.close()
        err = np.abs(w - ref)
        rows.append(dict(far_tol=tol, max_abs_dw=float(err.max()), p99_abs_dw=float(np.quantile(err, 0.99)),
                         ms=round(ms, 3), node_visits=int(nodes)))
        _log(f"far_tol: {tol} -> {ms:.2f} ms")
    return dict(study="far_tol", workload=f"SVG-like drawing, 19000 curves, {grid}^2 grid, order "
                f"{presets.FP64_2D['taylor_order']} (far_tol 0: uniform beta {presets.FP64_2D['beta']})", rows=rows)


def disagreement(grid=1024, bins=10):
    curves, q = W.config2(grid=grid)
    qd = _dev(q)
    ref, _ = _reference(curves, qd)
    frac = ref - np.floor(ref)
    rows = []
    for order, beta in ((0, 2.0), (1, 2.0), (2, 2.0), (2, 4.0), (12, 3.0)):
        m = G.Model(curves, presets.params(presets.FP64_2D, beta=beta, taylor_order=order, max_diag_frac=0.1, far_tol=0.0))
        w, _ = _run(m, qd, reps=1)
        m.close()
        bad = np.rint(w) != np.rint(ref)
        hist = np.histogram(frac[bad], bins=bins, range=(0.0, 1.0))[0]
        rows.append(dict(order=order, beta=beta, disagreements=int(bad.sum()), hist=hist.tolist(),
                         containment_flips=int(((w >= 0.5) != (ref >= 0.5)).sum())))
        _log(f"disagreement: order {order} beta {beta}: {int(bad.sum())}")
    return dict(study="disagreement", workload=f"SVG-like drawing, 19000 curves, {grid}^2 grid",
                bins=f"{bins} equal bins of the reference's fractional part", rows=rows)


def overlap(grid=512):
    rows = []
    for k in (1, 2, 4, 8, 16):
        curves = W.overlapping_polygons(k)
        q = W.grid_queries((-1.3, -1.3), (1.3, 1.3), (grid, grid))
        qd = _dev(q)
        ref, _ = _reference(curves, qd)
        for order, beta in ((0, 2.0), (2, 2.0), (12, 3.0)):
            m = G.Model(curves, presets.params(presets.FP64_2D, beta=beta, taylor_order=order, max_diag_frac=0.1, far_tol=0.0))
            w, _ = _run(m, qd, reps=1)
            m.close()
            err = np.abs(w - ref)
            rows.append(dict(k=k, order=order, beta=beta, max_abs_dw=float(err.max()),
                             max_rel_dw=float((err / np.maximum(np.abs(ref), 1.0)).max()),
                             misclassified=int((np.rint(w) != np.rint(ref)).sum())))
        _log(f"overlap: k = {k} done")
    return dict(study="overlap", workload=f"k nearly overlapping closed 15-gons, {grid}^2 grid over [-1.3, 1.3]^2",
                rows=rows)


STUDIES = dict(order_beta=order_beta, subdivision=subdivision, far_tol=far_tol, disagreement=disagreement,
               overlap=overlap)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--only", nargs="*", choices=sorted(STUDIES), default=None)
    a = ap.parse_args(argv)
    for name in a.only or list(STUDIES):
        _log(f"{name} ...")
        print(json.dumps(STUDIES[name]()), flush=True)


if __name__ == "__main__":
    main()
