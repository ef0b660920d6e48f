"""Error path and memory accounting of the query entry points, on the GPU:
a query that legitimately passes the near-field slot budget gets NaN, the
next call on the handle reports GWN_EOVERFLOW once, and the call after that
succeeds; the scratch figure the library reports for a launch is what the
launch takes from the stream-ordered pool."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import presets
from paper_2605_19200_amd import workloads as W
from tests.test_oracle3d import bilinear_patch

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run(model, q):
    out, ins = model.query(dev(q))
    torch.cuda.synchronize()
    return out.cpu().numpy(), ins.cpu().numpy()


def stacked_planes(k=80, gap=1e-3):
    """k parallel unit squares 1e-3 apart: a query inside the stack is near
    every one of them, more than the 64 near-field slots a query has."""
    return W.Patches3D.from_list([(*bilinear_patch((0, 0, z), (1, 0, z), (1, 1, z), (0, 1, z)), [])
                                  for z in gap * np.arange(k)])


def test_overflow_reported_once_then_cleared():
    P = stacked_planes()
    m = G.Model(P, presets.params(presets.FP64_3D, max_diag_frac=0.0, wave_accept=0))
    q_bad = np.array([[0.5, 0.5, 0.0395]])
    q_ok = np.array([[5.0, 5.0, 5.0], [0.5, 0.5, -3.0], [0.2, 0.7, 2.0]])
    print("overflow test: stacked planes, 1 overflowing + 3 plain queries", flush=True)
    w, _ = run(m, np.concatenate([q_bad, q_ok]))          # the overflowing call itself returns OK
    assert np.isnan(w[0]) and np.all(np.isfinite(w[1:])), w
    with pytest.raises(G.GwnError) as ei:                 # reported by the next call ...
        m.query(dev(q_ok))
    assert ei.value.status == G.GWN_EOVERFLOW
    w2, _ = run(m, q_ok)                                  # ... once
    assert np.array_equal(w2, w[1:])
    w3, _ = run(m, q_ok)
    assert np.array_equal(w3, w2)
    m.close()


def _pool():
    hip = ctypes.CDLL("libamdhip64.so")
    pool = ctypes.c_void_p()
    assert hip.hipDeviceGetDefaultMemPool(ctypes.byref(pool), torch.cuda.current_device()) == 0
    return hip, pool


USED_HIGH = 0x8   # hipMemPoolAttrUsedMemHigh


def pool_used_high(hip, pool):
    v = ctypes.c_uint64(0)
    assert hip.hipMemPoolGetAttribute(pool, USED_HIGH, ctypes.byref(v)) == 0
    return v.value


def reset_used_high(hip, pool):
    z = ctypes.c_uint64(0)
    assert hip.hipMemPoolSetAttribute(pool, USED_HIGH, ctypes.byref(z)) == 0


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_scratch_bytes_match_pool_usage(kind):
    """gwn_query_scratch_bytes equals what a launch takes from the pool (the
    pool may round up to its allocation granule)."""
    if kind == "2d":
        g, _ = W.config1()
        m = G.Model(g, presets.params(presets.FP64_2D))
        lo, hi = g.bbox()
    else:
        g = W.cad_assembly(4, n_bodies=2)
        m = G.Model(g, presets.params(presets.FP64_3D))
        lo, hi = g.bbox()
    hip, pool = _pool()
    rng = W.Rng(70, "scratch")
    for n in [1, 700, 40_000, 300_000]:
        q = dev(W.bbox_queries_uniform(rng, lo, hi, n, 1.0))
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        reset_used_high(hip, pool)
        G.gwn_query(m.h, q, out)
        torch.cuda.synchronize()
        used = pool_used_high(hip, pool)
        need = G.gwn_query_scratch_bytes(m.h, n, 1)
        print(f"scratch {kind} n={n}: library {need} B, pool high-water {used} B", flush=True)
        assert need <= used <= need + (2 << 20), (n, need, used)
    m.close()


def test_served_overflow_stays_in_its_request():
    """The served form: a request with a query that hits the near-field slot
    budget gets NaN for that query, the report of the count (on the next
    launch on the model) does not fail the next request, and every other
    value equals the direct call's."""
    from paper_2605_19200_amd import serve
    P = stacked_planes()
    q_bad = np.array([[0.5, 0.5, 0.0395], [0.3, 0.3, 5.0]])
    q_ok = np.array([[5.0, 5.0, 5.0], [0.5, 0.5, -3.0], [0.2, 0.7, 2.0]])
    srv = serve.Server(budget_bytes=64 << 20, n_slots=1)
    srv.add_model(P, presets.params(presets.FP64_3D, max_diag_frac=0.0))
    print("served overflow test: stacked planes, two requests", flush=True)
    fa = srv.submit(0, q_bad)
    wa, _ = fa.result(timeout=60)
    fb = srv.submit(0, q_ok)
    wb, _ = fb.result(timeout=60)
    srv.close()
    assert np.isnan(wa[0]) and np.isfinite(wa[1])
    assert srv.overflow_reports == 1
    m = G.Model(P, presets.params(presets.FP64_3D, max_diag_frac=0.0, wave_accept=0))   # as served
    w_ref, _ = run(m, q_ok)
    assert np.array_equal(wb, w_ref)
    m.close()
