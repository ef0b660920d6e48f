"""The oracle reproduces its frozen regression fixtures (tests/golden/).
Not a pin (see tests/golden/make_oracle_fixtures.py): any change to the
oracle's arithmetic must be justified and the fixtures rewritten."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_oracle_fixtures as F  # noqa: E402


@pytest.mark.parametrize("name,kind,geom,q", list(F.cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_oracle_matches_fixture(oracle, name, kind, geom, q):
    data = np.loadtxt(os.path.join(HERE, "golden", f"oracle_{name}.txt"))
    assert np.array_equal(data[:, :-1], q)
    w = oracle.gwn2d(geom, q) if kind == "2d" else oracle.gwn3d(geom, q)
    assert np.abs(w - data[:, -1]).max() <= 1e-13
