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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0 = auto, ~15 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3: 3 FP64 steps, then a 256 MiB device copy used to calibrate "
                         "FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the engine has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_19200_amd import gwn as G
    from paper_2605_19200_amd import presets
    from paper_2605_19200_amd import workloads as W

    t_gen = time.time()
    curves, q = W.config2(grid=args.grid)
    n = q.shape[0]
    print(f"[bench] workload: {curves.n} curves, {n} queries (gen {time.time() - t_gen:.1f} s)", file=sys.stderr,
          flush=True)
    t_b = time.time()
    model = G.Model(curves, presets.params(presets.FP64_2D))
    build_s = time.time() - t_b
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
        print(json.dumps({"profile_run": True, "queries": n, "copy_bytes": src.numel() * 8}))
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

    cpu = None
    if not args.no_cpu:
        rate = len(acc_idx) / t_o
        m_cpu = args.cpu_sample or int(min(max(15.0 * rate, 256), 65536))
        cidx = rng.permutation(n)[:m_cpu]
        threads = oracle.max_threads()
        tc = time.perf_counter()
        oracle.gwn2d(curves, q[cidx], threads=threads)
        tc = time.perf_counter() - tc
        cpu = {"value": m_cpu / tc, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"{m_cpu} seeded queries of the 1024x1024 grid, direct FP64 sum over all {curves.n} "
                         f"curves, OpenMP {threads} threads, {tc:.1f} s"}

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
                   "taylor_order": presets.FP64_2D["taylor_order"], "build_s": round(build_s, 3)},
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
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_query2d<false>", "kernel_ms": avg_kernel_s * 1e3,
                     "flops_per_launch": flops, "counters": counters},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
