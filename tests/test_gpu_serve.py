"""Served form: shared launches over several resident models, budget
admission, isolation (each request equals its solo run bitwise)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import presets
from paper_2605_19200_amd import serve
from paper_2605_19200_amd import workloads as W

pytestmark = pytest.mark.gpu


def solo(model: G.Model, pts: np.ndarray):
    w, ins = model.query(torch.from_numpy(np.ascontiguousarray(pts)).cuda())
    torch.cuda.synchronize()
    return w.cpu().numpy(), ins.cpu().numpy()


@pytest.fixture(scope="module")
def models2d():
    a = W.svg_like(501, n_groups=6)
    b = W.Curves2D.from_list(W.circle_curves((0.3, -0.2), 0.7))
    return [(a, presets.params(presets.MIXED_2D)), (a, presets.params(presets.FP64_2D)),
            (b, presets.params(presets.FP64_2D))]


def requests2d(server, geoms, rng, sizes):
    reqs = []
    for i, n in enumerate(sizes):
        m = i % len(geoms)
        lo, hi = geoms[m][0].bbox()
        reqs.append(serve.Request(m, W.bbox_queries_uniform(rng, lo, hi, int(n), 1.2), 0.0))
    return reqs


@pytest.mark.parametrize("budget", [4 << 30, 64 << 20])
def test_isolation_2d(models2d, budget):
    s = serve.Server(budget_bytes=budget, n_slots=2, chunk=1 << 14, max_launch=1 << 16)
    for g, p in models2d:
        s.add_model(g, p)
    rng = W.Rng(61, "serve2d")
    sizes = [1, 63, 64, 65, 1000, 5000, 40000, 3, 20000, 777, 0, 129]
    reqs = requests2d(s, models2d, rng, sizes)
    stats = s.run(reqs, closed_loop=True)
    assert stats["requests"] == len(sizes) and stats["peak_in_flight_bytes"] <= budget
    assert stats["launches"] >= 2
    for r in reqs:
        if r.points.shape[0] == 0:
            continue
        w, ins = solo(s.models[r.model], r.points)
        assert np.array_equal(r.w, w), (r.rid, r.model, r.points.shape)
        assert np.array_equal(r.inside, ins)
    s.close()


def test_budget_forces_pieces(models2d):
    """A 64 MiB budget splits a 2M-query request into pieces and still
    returns its solo values."""
    s = serve.Server(budget_bytes=64 << 20, n_slots=2)
    g, p = models2d[1]
    s.add_model(g, p)
    lo, hi = g.bbox()
    pts = W.bbox_queries_uniform(W.Rng(62, "big"), lo, hi, 2_000_000, 1.1)
    r = serve.Request(0, pts, 0.0)
    stats = s.run([r], closed_loop=True)
    assert stats["launches"] >= 2 and stats["peak_in_flight_bytes"] <= 64 << 20
    w, ins = solo(s.models[0], pts)
    assert np.array_equal(r.w, w) and np.array_equal(r.inside, ins)
    s.close()


def test_isolation_3d_and_open_loop():
    sphere = W.Patches3D.from_list([(cp, w, []) for cp, w in W.bodies(0, [("sphere", (0, 0, 0), 1.0)], disp=0.0)])
    cad = W.cad_assembly(63, n_bodies=2)
    s = serve.Server(budget_bytes=256 << 20, n_slots=2, chunk=4096)
    s.add_model(sphere, presets.params(presets.FP64_3D))
    s.add_model(cad, presets.params(presets.MIXED_3D))
    g2 = W.Curves2D.from_list(W.circle_curves((0.0, 0.0), 1.0))
    s.add_model(g2, presets.params(presets.FP64_2D))
    rng = W.Rng(63, "serve3d")
    geoms = [sphere, cad, g2]
    reqs = []
    for i, n in enumerate([50, 3000, 1, 700, 9000, 64, 200, 5000]):
        m = i % 3
        lo, hi = geoms[m].bbox()
        reqs.append(serve.Request(m, W.bbox_queries_uniform(rng, lo, hi, n, 1.2)))
    reqs = serve.poisson_requests(rng, 8, 400.0, [r.model for r in reqs], np.array([r.points.shape[0] for r in reqs]),
                                  lambda m, n, i: reqs[i].points)
    stats = s.run(reqs)
    assert np.all(np.diff([r.arrival for r in reqs]) >= 0)
    assert all(r.done >= r.arrival for r in reqs)
    assert 0 < stats["p50_ms"] <= stats["p99_ms"]
    for r in reqs:
        w, ins = solo(s.models[r.model], r.points)
        assert np.array_equal(r.w, w) and np.array_equal(r.inside, ins), (r.rid, r.model)
    s.close()


def test_bad_requests():
    s = serve.Server(budget_bytes=1 << 20)
    s.add_model(W.Curves2D.from_list(W.circle_curves((0, 0), 1.0)), presets.params(presets.FP64_2D))
    with pytest.raises(ValueError):
        s.run([serve.Request(1, np.zeros((4, 2)))])
    with pytest.raises(ValueError):
        s.run([serve.Request(0, np.zeros((4, 3)))])
    s.close()


def test_submit_from_live_producer(models2d):
    """A producer thread submits requests while earlier ones are in flight;
    every future resolves to the request's solo values, and an invalid
    request fails its own future only."""
    import threading
    s = serve.Server(budget_bytes=256 << 20, n_slots=2, chunk=1 << 14)
    for g, p in models2d:
        s.add_model(g, p)
    rng = W.Rng(64, "submit")
    sizes = [5, 3000, 64, 20000, 1, 777, 40000, 130]
    jobs = []

    def producer():
        for i, n in enumerate(sizes):
            m = i % len(models2d)
            lo, hi = models2d[m][0].bbox()
            pts = W.bbox_queries_uniform(rng, lo, hi, n, 1.2)
            jobs.append((m, pts, s.submit(m, pts)))

    t = threading.Thread(target=producer)
    t.start()
    t.join()
    bad = s.submit(7, np.zeros((3, 2)))
    for m, pts, f in jobs:
        w, ins = f.result(timeout=120)
        ws, inss = solo(s.models[m], pts)
        assert np.array_equal(w, ws) and np.array_equal(ins, inss)
    with pytest.raises(ValueError):
        bad.result(timeout=60)
    s.close()


def test_launches_overlap_on_device():
    """Closed-loop requests on four slots against a 3D model (each launch's
    device work far longer than the host's preparation of the next): HIP
    events on the slot streams show launches of different slots in flight
    at the same time."""
    from itertools import combinations
    s = serve.Server(budget_bytes=4 << 30, n_slots=4, chunk=1 << 13, max_launch=1 << 14, record_timing=True)
    g = W.cad_assembly(63, n_bodies=2)
    s.add_model(g, presets.params(presets.FP64_3D))
    lo, hi = g.bbox()
    rng = W.Rng(65, "overlap")
    reqs = [serve.Request(0, W.bbox_queries_uniform(rng, lo, hi, 16_000, 1.1)) for _ in range(8)]
    s.run(reqs, closed_loop=True)
    iv = s.launch_intervals()
    assert len(iv) >= 8 and all(b > a for _, a, b in iv)
    pairs = [(x, y) for x, y in combinations(iv, 2) if x[0] != y[0] and x[1] < y[2] and y[1] < x[2]]
    print(f"serve overlap: {len(iv)} launches, {len(pairs)} overlapping pairs on different slots", flush=True)
    assert pairs
    for r in reqs:
        w, ins = solo(s.models[0], r.points)
        assert np.array_equal(r.w, w) and np.array_equal(r.inside, ins)
    s.close()
