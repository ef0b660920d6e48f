"""gwn_query_noalloc: the query entry point for callers that cannot allocate.
Its results equal gwn_query's bitwise, on two calls in a row (the second
smaller), in 2D and 3D; it takes nothing from the stream-ordered pool; a
call whose scratch exceeds the fixed array is refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import presets
from paper_2605_19200_amd import workloads as W
from tests.test_gpu_overflow import _pool, pool_used_high, reset_used_high

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def both(m, q):
    n = q.shape[0]
    w1 = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    i1 = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
    w2 = torch.full((n,), -5.0, dtype=torch.float64, device="cuda")
    i2 = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    G.gwn_query(m.h, q, w1, i1)
    torch.cuda.synchronize()
    hip, pool = _pool()
    reset_used_high(hip, pool)
    G.gwn_query_noalloc(m.h, q, w2, i2)
    torch.cuda.synchronize()
    assert pool_used_high(hip, pool) == 0
    return (w1.cpu().numpy(), i1.cpu().numpy()), (w2.cpu().numpy(), i2.cpu().numpy())


@pytest.mark.parametrize("kind", ["2d", "2d-mixed", "3d", "3d-mixed"])
def test_noalloc_equals_query(kind):
    if kind.startswith("2d"):
        g, _ = W.config2(grid=4)
        pre = presets.MIXED_2D if kind.endswith("mixed") else presets.FP64_2D
        sizes = (300_000, 1000)
    else:
        g = W.cad_assembly(4, n_bodies=3)
        pre = presets.MIXED_3D if kind.endswith("mixed") else presets.FP64_3D
        sizes = (40_000, 65)
    m = G.Model(g, presets.params(pre))
    lo, hi = g.bbox()
    rng = W.Rng(90, "noalloc/" + kind)
    for n in sizes:                       # two calls in a row, the second smaller
        print(f"noalloc {kind}: n={n}", flush=True)
        q = dev(W.bbox_queries_uniform(rng, lo, hi, n, 1.1))
        (w1, i1), (w2, i2) = both(m, q)
        assert np.all(np.isfinite(w1))
        assert np.array_equal(w1, w2) and np.array_equal(i1, i2)
    m.close()


def test_noalloc_refuses_oversized_calls():
    g = W.cad_assembly(4, n_bodies=2)
    m = G.Model(g, presets.params(presets.FP64_3D))
    n = 400_000
    assert G.gwn_query_scratch_bytes(m.h, n, 1) > G.GWN_NOALLOC_SCRATCH_BYTES
    lo, hi = g.bbox()
    q = dev(W.bbox_queries_uniform(W.Rng(91, "big"), lo, hi, n, 1.0))
    out = torch.full((n,), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GwnError) as ei:
        G.gwn_query_noalloc(m.h, q, out)
    assert ei.value.status == G.GWN_EINVAL and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(out == 3.0)
    small = q[:1000]
    o1 = torch.empty(1000, dtype=torch.float64, device="cuda")
    o2 = torch.empty(1000, dtype=torch.float64, device="cuda")
    G.gwn_query(m.h, small, o1)
    G.gwn_query_noalloc(m.h, small, o2)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    m.close()
