"""Host-side parts of the served form that need no GPU."""
import numpy as np

from paper_2605_19200_amd import serve
from paper_2605_19200_amd import workloads as W


def test_poisson_arrivals_are_seeded_and_have_the_rate():
    n, rate = 4000, 250.0
    sizes = np.full(n, 10)
    mk = lambda: serve.poisson_requests(W.Rng(5, "arrivals"), n, rate, [i % 3 for i in range(n)], sizes,
                                        lambda m, k, i: np.zeros((k, 2)))
    a, b = mk(), mk()
    ta = np.array([r.arrival for r in a])
    assert np.array_equal(ta, [r.arrival for r in b])
    assert np.all(np.diff(ta) > 0)
    gaps = np.diff(np.concatenate([[0.0], ta]))
    assert abs(gaps.mean() * rate - 1.0) < 0.05          # mean 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.08    # exponential: cv = 1
    assert [r.model for r in a[:6]] == [0, 1, 2, 0, 1, 2] and a[0].points.shape == (10, 2)
    assert np.isnan(a[0].latency)
