"""The parameter-study module runs end to end on small grids, and its
measured trends are the ones the paper reports: the far-field error falls
with beta and with the order, and the order-0 error grows with the number of
overlapping polygons."""
import numpy as np
import pytest

pytest.importorskip("torch")

from paper_2605_19200_amd import studies

pytestmark = pytest.mark.gpu


def test_order_beta_trends():
    out = studies.order_beta(grid=128)
    err = {(r["order"], r["beta"]): r["max_abs_dw"] for r in out["rows"]}
    for order in (0, 2, 12):
        assert err[order, 2.0] > err[order, 8.0] > err[order, 64.0] or err[order, 64.0] < 1e-12
    for beta in (2.0, 4.0):
        assert err[0, beta] > err[2, beta] > err[12, beta]
    assert err[12, 3.0] < 1e-6


def test_overlap_error_grows_with_k():
    out = studies.overlap(grid=64)
    e0 = [r["max_abs_dw"] for r in out["rows"] if r["order"] == 0]
    assert len(e0) == 5 and all(b > a for a, b in zip(e0, e0[1:]))
    assert max(r["max_abs_dw"] for r in out["rows"] if r["order"] == 12) < 1e-6


def test_subdivision_and_disagreement_run():
    sub = studies.subdivision(grid=128)
    leaves = [r["leaves"] for r in sub["rows"]]
    assert leaves == sorted(leaves) and all(r["max_abs_dw"] < 1e-6 for r in sub["rows"])
    dis = studies.disagreement(grid=128)
    rows = {(r["order"], r["beta"]): r for r in dis["rows"]}
    assert rows[12, 3.0]["disagreements"] == 0
    assert rows[0, 2.0]["disagreements"] >= rows[2, 2.0]["disagreements"]
    assert sum(rows[0, 2.0]["hist"]) == rows[0, 2.0]["disagreements"]


def test_far_tol_study_trends():
    out = studies.far_tol(grid=128)
    rows = {r["far_tol"]: r for r in out["rows"]}
    budgets = sorted(t for t in rows if t > 0)
    # a looser budget accepts clusters sooner: fewer node visits, larger error
    visits = [rows[t]["node_visits"] for t in budgets]
    assert visits == sorted(visits, reverse=True)
    assert rows[1e-8]["max_abs_dw"] < 1e-6 and rows[1e-8]["node_visits"] < rows[0.0]["node_visits"]
