"""Benchmark of the GWN query path on one MI355X.

Workload: the 2D SVG-like drawing (50 groups x 4 nested loops of rational
Bezier curves, 20,000 curves before 5% deletion, degree 2-3, weights
U(0.5, 2)) queried on a 1024 x 1024 cell-centred grid over its bounding box.
One step = one gwn_query over the whole grid (SFC keys, radix sort,
traversal with far field and direct leaves, classification, scatter), inputs
resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic FP64 operations per counted event (2D query path):
#   internal node test: 2 sub + 3 (dx^2 + dy^2) + 1 (beta^2 r^2)    = 6
#   order-p complex Taylor term: 1 reciprocal + 2 (u) + p complex
#     multiply-adds (8 each) + 3 (Im of u * t) + 1 accumulate   = 7 + 8 p
#   direct leaf set-up: 8 (translate end points) + 6 (cross, dot)   = 14
#   bisection piece: 30 lerps x 3 + 4 (t0, t1, 1-t0, 1-t1) + 16
#     (AABB min/max/sign tests)                                     = 110
#   atan2: range reduction + degree-9 odd minimax polynomial         = 20
FLOPS = dict(nodes=6, leaves=14, pieces=110, angles=20)


def algorithmic_flops(c: dict, order: int) -> float:
    return float(sum(FLOPS[k] * c[k] for k in FLOPS) + (7 + 8 * order) * c["far"])


# Algorithmic FP64 operations per near-field integrand node (3D, k_near3d):
#   two cubic Bernstein bases with derivatives                  2 x 23 = 46
#   control net: 16 points x 4 coordinates x 2 (value, v-partial)
#     multiply-adds, then 4 rows x 4 x 3 accumulations     (128 + 48) x 2 = 352
#   A = H - q W and its partials                                 9 x 2 = 18
#   density det[A, A_u, A_v] / |A|^3                                    22
#   radial map (x, expm1, 1/(1+e), tau, Jacobian, u, v)                 17
#   f = Jacobian tau density, rounding weight, Kronrod sums             20
NEAR_FLOPS_PER_NODE = 475
# Algorithmic FP64 operations of the 3D traversal (k_trav3d), per event:
#   node test: q - c (3), |q - c|^2 (5), against beta^2 r^2 (1)            9
#   node-set node: x - q (3), |r|^2 (5), 1/|r| (1), n . r (5), / |r|^3 (2),
#     accumulate (2)                                                      18
#   far term of order 6 (degrees 1..7 of the solid harmonics): scaling and
#     1/rho (9), 7 diagonal steps (8 each), 28 column steps (9 each),
#     35 moment contractions (4 each)                                    461
TRAV_FLOPS_PER_NODE_TEST = 9
TRAV_FLOPS_PER_SET_NODE = 18
TRAV_FLOPS_PER_FAR_TERM = 461


def physical_cores():
    """Physical cores of the host (distinct (core, socket) pairs from
    lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu", "-p=Core,Socket"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    pairs = {ln.strip() for ln in out.splitlines() if ln.strip() and not ln.startswith("#")}
    return len(pairs) or None


PROFILE = os.path.join(ROOT, "profiles", "k_query2d_svg1024.md")
KERNEL_SOURCES = ["query.hip", "query_common.h", "gwn_internal.h"]


def kernel_source_hash() -> str:
    """Hash of the 2D kernel's sources with comments and blank space removed
    (a comment edit does not invalidate the recorded counters), and of the
    FP64 parameter set the timed launch runs with."""
    import hashlib
    import re
    from paper_2605_19200_amd import presets
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_19200_amd", "csrc", f)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update(" ".join(text.split()).encode())
    h.update(repr(sorted(presets.FP64_2D.items())).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the timed kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel
    calibration), or None when the kernel sources changed since."""
    if not os.path.exists(PROFILE):
        return None
    vals = {}
    with open(PROFILE) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bench_small(calls: int = 256) -> dict:
    """The small case (star loop of 64 rational cubics, 4096 queries), which
    is bound by launch latency: one call's wall time, and the throughput of
    `calls` calls issued back to back on one stream."""
    import torch
    from paper_2605_19200_amd import gwn as G
    from paper_2605_19200_amd import presets
    from paper_2605_19200_amd import workloads as W

    curves, q = W.config1()
    pts = torch.from_numpy(q).cuda()
    m = G.Model(curves, presets.params(presets.FP64_2D))
    out = torch.empty(q.shape[0], dtype=torch.float64, device="cuda")
    ins = torch.empty(q.shape[0], dtype=torch.uint8, device="cuda")
    for _ in range(5):
        G.gwn_query(m.h, pts, out, ins)
    torch.cuda.synchronize()
    lat = []
    for _ in range(20):
        t = time.perf_counter()
        G.gwn_query(m.h, pts, out, ins)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
    t = time.perf_counter()
    for _ in range(calls):
        G.gwn_query(m.h, pts, out, ins)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    m.close()
    return {"workload": f"star loop: {curves.n} rational cubics, {q.shape[0]} queries, FP64 form",
            "call_ms_median": float(np.median(lat) * 1e3), "back_to_back_calls": calls,
            "back_to_back_queries_per_s": calls * q.shape[0] / dt}


def _query3d_timed(G, m, pts):
    """One timed 3D launch: wall time, per-kernel event times (traversal,
    near field), and the rows that hit a limit (NaN); the library's report
    of them, made by the next call on the model, is taken outside the timed
    region."""
    import torch
    out = torch.empty(pts.shape[0], dtype=torch.float64, device=pts.device)
    ins = torch.empty(pts.shape[0], dtype=torch.uint8, device=pts.device)
    torch.cuda.synchronize()
    G.gwn_profile(True)
    t = time.perf_counter()
    G.gwn_query(m.h, pts, out, ins)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    G.gwn_profile(False)
    trav = G.gwn_profile_kernel(G.GWN_K_TRAV3D)[0]
    near = G.gwn_profile_kernel(G.GWN_K_NEAR3D)[0]
    w = out.cpu().numpy()
    flagged = int(np.isnan(w).sum())
    if flagged:
        try:
            G.gwn_query(m.h, pts[:0], out[:0], ins[:0])
        except G.GwnError:
            pass
    return dt, trav, near, w, ins.cpu().numpy(), flagged


def bench3d() -> dict:
    """3D side measurement: the bodies scene (4096 trimmed bicubic patches)
    on its 128^3 grid and the CAD assembly (19,968 patches, every one
    trimmed) with its 1M queries, FP64 and mixed forms, one timed launch
    each, with the per-kernel split and, for the CAD assembly, the accuracy
    on the 1,024 rows of the committed oracle fixture.  The near-field
    kernel's roofline comes from the evaluation counter of the bodies grid."""
    import torch
    from paper_2605_19200_amd import gwn as G
    from paper_2605_19200_amd import presets
    from paper_2605_19200_amd import workloads as W

    P, q = W.config3()
    pts = torch.from_numpy(q).cuda()
    out = {"workload": f"bodies scene: {P.n} trimmed rational bicubic patches, 128^3 grid", "queries": q.shape[0]}
    for name, pre in [("fp64", presets.FP64_3D), ("mixed", presets.MIXED_3D)]:
        m = G.Model(P, presets.params(pre))
        m.query(pts[:4096])
        dt, trav, near, _, _, flagged = _query3d_timed(G, m, pts)
        out[name] = {"queries_per_s": q.shape[0] / dt, "ms": dt * 1e3, "beta": pre["beta"],
                     "far_tol": pre.get("far_tol", 0.0), "wave_accept": pre.get("wave_accept", 0),
                     "k_trav3d_ms": trav, "k_near3d_ms": near, "flagged_rows": flagged,
                     "leaves": int(m.inspect(G.GWN_I_SUMMARY)[0][2]), "resident_bytes": int(m.bytes()[0])}
        if name == "fp64":
            c = m.counters(pts)
            flops = c["pieces"] * NEAR_FLOPS_PER_NODE
            tf = flops / (near / 1e3) / 1e12
            out["roofline_k_near3d"] = {
                "bound": "alu", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "traffic": None, "kernel": "k_near3d<false, false>",
                "kernel_ms": near, "integrand_nodes": int(c["pieces"]), "flops_per_node": NEAR_FLOPS_PER_NODE,
                "flops_per_launch": float(flops)}
            tflops = (c["nodes"] * TRAV_FLOPS_PER_NODE_TEST + c["angles"] * TRAV_FLOPS_PER_SET_NODE
                      + c["far"] * TRAV_FLOPS_PER_FAR_TERM)
            tt = tflops / (trav / 1e3) / 1e12
            out["roofline_k_trav3d"] = {
                "bound": "alu", "achieved": tt, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tt / FP64_VECTOR_PEAK_TFLOPS, "traffic": None, "kernel": "k_trav3d<false, false>",
                "kernel_ms": trav, "node_tests": int(c["nodes"]), "node_set_nodes": int(c["angles"]),
                "far_terms": int(c["far"]), "flops_per_launch": float(tflops)}
        m.close()
        print(f"[bench] 3D bodies {name}: {dt * 1e3:.1f} ms per grid (traversal {trav:.1f} ms, near field "
              f"{near:.1f} ms)", file=sys.stderr, flush=True)
    # the CAD assembly, config 4
    P4, q4 = W.config4()
    pts4 = torch.from_numpy(q4).cuda()
    fx = os.path.join(ROOT, "tests", "golden", "oracle_cad_assembly_1m.txt")
    rows, ref = None, None
    if os.path.exists(fx):
        data = np.loadtxt(fx, comments="#")
        rows, ref = data[:, 0].astype(np.int64), data[:, 4]
    cad = {"workload": f"CAD assembly: 39 bodies, {P4.n} trimmed rational bicubic patches (2-4 trim loops "
                       "each), 500k near-surface + 500k uniform queries", "queries": q4.shape[0]}
    for name, pre in [("fp64", presets.FP64_3D), ("mixed", presets.MIXED_3D)]:
        m = G.Model(P4, presets.params(pre))
        m.query(pts4[:4096])
        dt, trav, near, w, ins, flagged = _query3d_timed(G, m, pts4)
        r = {"queries_per_s": q4.shape[0] / dt, "ms": dt * 1e3, "k_trav3d_ms": trav, "k_near3d_ms": near,
             "flagged_rows": flagged, "leaves": int(m.inspect(G.GWN_I_SUMMARY)[0][2])}
        if rows is not None:
            err = np.abs(w[rows] - ref)
            sure = np.abs(ref - 0.5) > 1e-3
            r.update({"oracle_rows": int(rows.size), "max_abs_dw": float(np.nanmax(err)),
                      "p99_abs_dw": float(np.nanquantile(err, 0.99)),
                      "containment_mismatch_outside_1e-3": int(np.sum(((ins[rows] != 0) != (ref >= 0.5)) & sure))})
        cad[name] = r
        m.close()
        print(f"[bench] 3D CAD {name}: {dt * 1e3:.1f} ms per 1M queries (traversal {trav:.1f} ms, near field "
              f"{near:.1f} ms), {flagged} flagged rows", file=sys.stderr, flush=True)
    out["cad_assembly"] = cad
    return out


def served_benchmark(seed: int = 5, n_requests: int = 400, loads=(0.5, 0.8, 0.95), exp3d=(2.0, 3.0),
                     kinds=("2d",)) -> dict:
    """Served form on the serving workload: resident models of the kinds
    asked for among eight (2D drawings of about 5k-20k curves, 3D assemblies
    of 4-39 bodies), mixed form, requests with model uniform over them and
    N = 10^U(3, 6) queries for 2D models, 10^U(exp3d) for 3D models
    (near-surface and uniform queries in equal parts).  A closed-loop pass
    gives the saturation request rate; Poisson arrivals at the given
    fractions of it give p50 / p99 latency."""
    from paper_2605_19200_amd import presets, serve
    from paper_2605_19200_amd import workloads as W

    t = time.time()
    geoms = [(k, g) for k, g in W.serving_models(seed, kinds=kinds)]
    srv = serve.Server(budget_bytes=4 << 30, n_slots=4)
    for kind, g in geoms:
        srv.add_model(g, presets.params(presets.MIXED_2D if kind == "2d" else presets.MIXED_3D))
    build_s = time.time() - t
    rng = W.Rng(seed, "serve/requests")
    models = rng.integers(n_requests, 0, len(geoms) - 1)
    expo = rng.uniform(n_requests, 3.0, 6.0)
    expo = np.where([geoms[m][0] == "3d" for m in models], rng.uniform(n_requests, *exp3d), expo)
    sizes = np.floor(10 ** expo).astype(np.int64)
    rq = W.Rng(seed, "serve/points")

    def points(m, n, i):
        kind, g = geoms[m]
        lo, hi = g.bbox()
        if kind == "2d":
            return W.bbox_queries_uniform(rq, lo, hi, n, 1.0)
        h = n // 2
        return np.concatenate([W.near_surface_queries(g, rq, h), W.bbox_queries_uniform(rq, lo, hi, n - h, 1.0)])

    # query pools per model (near-surface sampling is the slow part of the
    # generation); each request takes a seeded window of its model's pool
    pool_n = int(sizes.max()) * 2
    pools = [points(m, min(pool_n, 2 * int(sizes[models == m].max(initial=1))), -1) for m in range(len(geoms))]
    print(f"[bench] served: models built in {build_s:.1f} s, pools ready at {time.time() - t:.1f} s", file=sys.stderr,
          flush=True)
    starts = rng.uniform(n_requests)
    pts = []
    for i in range(n_requests):
        pool = pools[int(models[i])]
        a = int(starts[i] * (pool.shape[0] - int(sizes[i])))
        pts.append(pool[a:a + int(sizes[i])])
    mk = lambda rate: serve.poisson_requests(W.Rng(seed, f"serve/arrivals/{rate:.6g}"), n_requests, rate,
                                             [int(m) for m in models], sizes, lambda m, n, i: pts[i])
    warm = [serve.Request(int(models[i]), pts[i][:256]) for i in range(min(n_requests, 16))]
    say = lambda msg: print(f"[bench] served: {msg}", file=sys.stderr, flush=True)
    srv.run(warm, closed_loop=True, progress=say)
    say("warm-up done")
    sat = srv.run(mk(1.0), closed_loop=True, progress=say)
    sat_rate = n_requests / sat["wall_s"]
    print(f"[bench] served saturation: {sat_rate:.1f} requests/s, {sat['queries_per_s']:.3e} q/s", file=sys.stderr,
          flush=True)
    desc = {"2d": "4 x 2D drawings of 5k-20k curves, N = 10^U(3,6)",
            "3d": f"4 x 3D assemblies of 4-39 bodies, N = 10^U({exp3d[0]:g},{exp3d[1]:g})"}
    out = {"workload": f"{len(geoms)} resident models ({'; '.join(desc[k] for k in kinds)}), mixed form, "
                       f"{n_requests} requests, Poisson arrivals",
           "resident_bytes": srv.resident_bytes(), "build_s": round(build_s, 2), "queries": int(sizes.sum()),
           "saturation": {"requests_per_s": sat_rate, "queries_per_s": sat["queries_per_s"],
                          "launches": sat["launches"], "overflow_reports": sat["overflow_reports"]},
           "loads": []}
    for f in loads:
        r = srv.run(mk(f * sat_rate), progress=say)
        out["loads"].append({"load": f, "requests_per_s": f * sat_rate, "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                             "queries_per_s": r["queries_per_s"], "peak_in_flight_bytes": r["peak_in_flight_bytes"]})
        print(f"[bench] served load {f}: p50 {r['p50_ms']:.2f} ms, p99 {r['p99_ms']:.2f} ms", file=sys.stderr,
              flush=True)
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0 = auto, ~15 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D side measurement")
    ap.add_argument("--profile-3d", action="store_true",
                    help="short run for rocprofv3: one FP64 and one mixed pass over the 3D bodies scene grid")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3: 3 FP64 steps, then a 256 MiB device copy used to calibrate "
                         "FETCH_SIZE/WRITE_SIZE, then 3 steps of the mixed form (k_query2d_mixed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the engine has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_19200_amd import gwn as G
    from paper_2605_19200_amd import presets
    from paper_2605_19200_amd import workloads as W

    if args.profile_3d:
        print(json.dumps({"profile_3d": True, **bench3d()}))
        return
    t_gen = time.time()
    curves, q = W.config2(grid=args.grid)
    n = q.shape[0]
    print(f"[bench] workload: {curves.n} curves, {n} queries (gen {time.time() - t_gen:.1f} s)", file=sys.stderr,
          flush=True)
    t_b = time.time()
    model = G.Model(curves, presets.params(presets.FP64_2D))
    build_s = time.time() - t_b
    n_leaves = int(model.inspect(G.GWN_I_SUMMARY)[0][2])
    pts = torch.from_numpy(q).cuda()
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ins = torch.empty(n, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        G.gwn_query(model.h, pts, out, ins, stream)

    if args.profile_run:
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        model_m = G.Model(curves, presets.params(presets.MIXED_2D))
        for _ in range(3):
            G.gwn_query(model_m.h, pts, out, ins, stream)
        torch.cuda.synchronize()
        model_m.close()
        print(json.dumps({"profile_run": True, "queries": n, "copy_bytes": 32 * 1024 * 1024 * 8}))
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    G.gwn_profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = G.gwn_profile(False)
    dt = t1 - t0
    qps = n * args.steps / dt
    w64 = out.cpu().numpy().copy()
    print(f"[bench] fp64: {dt / args.steps * 1e3:.3f} ms/step, {qps:.3e} q/s", file=sys.stderr, flush=True)

    counters = model.counters(pts)
    flops = algorithmic_flops(counters, presets.FP64_2D["taylor_order"])
    avg_kernel_s = kern_ms / max(launches, 1) / 1e3
    achieved_tflops = flops / avg_kernel_s / 1e12

    # the paper's default order (2) with the beta meeting the same bound
    model_p = G.Model(curves, presets.params(presets.PAPER_ORDER_2D))
    for _ in range(args.warmup):
        G.gwn_query(model_p.h, pts, out, ins, stream)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(max(args.steps // 4, 2)):
        G.gwn_query(model_p.h, pts, out, ins, stream)
    torch.cuda.synchronize()
    qps_p = n * max(args.steps // 4, 2) / (time.perf_counter() - tp0)
    wp = out.cpu().numpy().copy()
    model_p.close()

    # mixed form on the same workload
    model_m = G.Model(curves, presets.params(presets.MIXED_2D))
    out_m = torch.empty_like(out)
    ins_m = torch.empty_like(ins)
    for _ in range(args.warmup):
        G.gwn_query(model_m.h, pts, out_m, ins_m, stream)
    torch.cuda.synchronize()
    tm0 = time.perf_counter()
    for _ in range(args.steps):
        G.gwn_query(model_m.h, pts, out_m, ins_m, stream)
    torch.cuda.synchronize()
    tm1 = time.perf_counter()
    qps_m = n * args.steps / (tm1 - tm0)
    wm = out_m.cpu().numpy()
    cm = model_m.counters(pts)

    # accuracy on a seeded sample against the oracle, and the CPU baseline
    from oracle import oracle
    rng = W.Rng(99, "bench/sample")
    acc_idx = rng.permutation(n)[:512]
    t_o = time.perf_counter()
    ref = oracle.gwn2d(curves, q[acc_idx])
    t_o = time.perf_counter() - t_o
    err64 = np.abs(w64[acc_idx] - ref)
    errp = np.abs(wp[acc_idx] - ref)
    errm = np.abs(wm[acc_idx] - ref)
    sure = np.abs(ref - 0.5) > 1e-3
    mism64 = int(np.sum(((w64[acc_idx] >= 0.5) != (ref >= 0.5)) & sure))
    mismm = int(np.sum(((wm[acc_idx] >= 0.5) != (ref >= 0.5)) & sure))

    served = None if args.no_served else served_benchmark()
    # the serving workload with 2D and 3D models, 3D requests of 10^U(3, 6)
    # queries like the 2D ones (200 requests)
    served_all = None if args.no_served else served_benchmark(n_requests=200, kinds=("2d", "3d"), exp3d=(3.0, 6.0))
    side3d = None if args.no_3d else bench3d()
    small = bench_small()
    print(f"[bench] star loop: {small['call_ms_median']:.3f} ms per call, "
          f"{small['back_to_back_queries_per_s']:.3e} q/s back to back", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        # the oracle on the host's physical cores (lscpu), within the CPU
        # share this process may use; also 1 thread, and 14 threads as in the
        # paper's measurements
        rate = len(acc_idx) / t_o
        phys = physical_cores()
        avail = len(os.sched_getaffinity(0))
        if os.environ.get("OMP_NUM_THREADS", "").isdigit():
            avail = min(avail, int(os.environ["OMP_NUM_THREADS"]))
        threads = max(1, min(phys or avail, avail))

        def leg(nthreads, m_cpu):
            cidx = rng.permutation(n)[:m_cpu]
            tc = time.perf_counter()
            oracle.gwn2d(curves, q[cidx], threads=nthreads)
            tc = time.perf_counter() - tc
            return m_cpu, tc

        # sample sizes for about 15 s (all cores) and 5 s (1 and 14 threads),
        # from the accuracy sample's rate and then the first leg's
        m_cpu, tc = leg(threads, args.cpu_sample or int(min(max(15.0 * rate, 256), 1 << 20)))
        per_thread = m_cpu / tc / threads
        m1, t1c = leg(1, int(max(5.0 * per_thread, 64)))
        m14, t14 = leg(14, int(max(5.0 * per_thread * 14, 64)))
        cpu = {"value": m_cpu / tc, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "physical_cores_lscpu": phys,
               "sample": f"{m_cpu} seeded queries of the 1024x1024 grid, direct FP64 sum over all {curves.n} "
                         f"curves, OpenMP {threads} threads, {tc:.1f} s",
               "threads_1": {"value": m1 / t1c, "sample": f"{m1} queries, {t1c:.1f} s"},
               "threads_14": {"value": m14 / t14, "sample": f"{m14} queries, {t14:.1f} s"}}

    line = {
        "metric": "GWN containment queries/sec at |dw|<=1e-6 (FP64) vs mixed; p50/p99 served latency",
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D SVG-like drawing: 200 nested/overlapping loops, "
                               f"{curves.n} rational Bezier curves (degree 2-3), {args.grid}x{args.grid} grid",
                   "queries": n, "curves": curves.n, "beta": presets.FP64_2D["beta"],
                   "far_tol": presets.FP64_2D.get("far_tol", 0.0),
                   "wave_accept": presets.FP64_2D.get("wave_accept", 0),
                   "taylor_order": presets.FP64_2D["taylor_order"],
                   "max_diag_frac": presets.FP64_2D.get("max_diag_frac", 0.1), "leaves": n_leaves,
                   "build_s": round(build_s, 3)},
        "accuracy": {"sample": len(acc_idx), "fp64_max_abs_dw": float(err64.max()),
                     "fp64_containment_mismatch_outside_1e-3": mism64,
                     "mixed_max_abs_dw": float(errm.max()), "mixed_p99_abs_dw": float(np.quantile(errm, 0.99)),
                     "mixed_rms_abs_dw": float(np.sqrt(np.mean(errm ** 2))),
                     "mixed_containment_mismatch_outside_1e-3": mismm},
        "paper_order2": {"value": qps_p, "unit": "queries/s", "beta": presets.PAPER_ORDER_2D["beta"],
                         "taylor_order": 2, "max_abs_dw": float(errp.max())},
        "mixed": {"value": qps_m, "unit": "queries/s", "beta_mixed": presets.MIXED_2D["beta_mixed"],
                  "reclassified": int(cm["reclass"]), "ms_per_step": (tm1 - tm0) / args.steps * 1e3,
                  "counters": cm},
        "served": served,
        "served_2d_3d": served_all,
        "3d": side3d,
        "small_case": small,
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "kernel": "k_query2d<false>", "kernel_ms": avg_kernel_s * 1e3,
                     "flops_per_launch": flops, "counters": counters},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
