"""The C ABI from a plain C program (paper_2605_19200_amd/examples/circle.c,
built by the package's build step): the unit circle as rational arcs and as
an extracted NURBS curve, queried on the GPU against the exact winding
number (1 inside, 0 outside)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "paper_2605_19200_amd", "examples", "circle")


def test_c_client_circle():
    if not os.path.exists(EXAMPLE):
        pytest.skip("examples/circle is built by __graft_entry__.build()")
    r = subprocess.run([EXAMPLE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "circle: ok" in r.stdout
    assert r.stdout.count("wrong containment flags = 0") == 2
