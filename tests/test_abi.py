"""The C-ABI library loads, exports every symbol declared in include/gwn.h,
and validates its inputs on the host (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from paper_2605_19200_amd import gwn as G
from paper_2605_19200_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gwn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gwn_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = G.lib()
    syms = declared_symbols()
    assert "gwn_query" in syms and "gwn_build2d" in syms
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(G.EXPORTED) == syms


def test_default_params():
    p = G.gwn_default_params()
    assert p.beta == 2.0 and p.taylor_order == 2 and p.max_diag_frac == 0.1 and p.gl_nodes == 10
    assert p.leaf_far == 1 and p.wave_accept == 0


def host_params(**kw):
    return G.gwn_default_params(device=-1, **kw)


def test_host_only_build_and_query_rejected():
    curves, q = W.config1()
    h = G.gwn_build2d(curves, host_params())
    s = G.gwn_inspect(h, G.GWN_I_SUMMARY)[0]
    assert s[0] == 2 and s[1] == 64 and s[2] >= 64 and s[3] == 2 * s[2] - 1
    st = G.lib().gwn_query(h, None, 0, None, None, None)
    assert st == G.GWN_EINVAL and "host-only" in G.gwn_last_error()
    G.gwn_free(h)


@pytest.mark.parametrize("bad", ["degree", "weight", "nan", "offset", "beta"])
def test_invalid_inputs(bad):
    p = [np.array([[0, 0], [1, 0], [1, 1.0]]), np.array([1.0, 0.5, 1.0])]
    params = host_params()
    if bad == "weight":
        p[1] = np.array([1.0, 0.0, 1.0])
    if bad == "nan":
        p[0] = np.array([[0, 0], [np.nan, 0], [1, 1.0]])
    c = W.Curves2D.from_list([tuple(p)])
    if bad == "degree":
        c.degree[0] = 4
    if bad == "offset":
        c.cp_offset[1] = 2
    if bad == "beta":
        params.beta = 1.5
    with pytest.raises(G.GwnError) as ei:
        G.gwn_build2d(c, params)
    assert ei.value.status == G.GWN_EINVAL
    assert G.gwn_last_error()


def test_empty_model():
    c = W.Curves2D.from_list([])
    h = G.gwn_build2d(c, host_params())
    assert G.gwn_inspect(h, G.GWN_I_SUMMARY)[0][2] == 0
    G.gwn_free(h)


def test_set_params_validation():
    curves, _ = W.config1()
    h = G.gwn_build2d(curves, host_params())
    p = G.gwn_get_params(h)
    p.taylor_order = 17
    with pytest.raises(G.GwnError):
        G.gwn_set_params(h, p)
    p.taylor_order = 1
    p.leaf_far = 2
    with pytest.raises(G.GwnError):
        G.gwn_set_params(h, p)
    p.leaf_far = 0
    p.beta = 8.0
    G.gwn_set_params(h, p)
    assert G.gwn_get_params(h).leaf_far == 0
    assert G.gwn_get_params(h).beta == 8.0 and G.gwn_get_params(h).taylor_order == 1
    G.gwn_free(h)


def test_header_is_plain_c(tmp_path):
    """include/gwn.h compiles as C99 on its own (no C++ or HIP types)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "t.c"
    src.write_text('#include "gwn.h"\nint main(void) { gwn_params p; gwn_default_params(&p); return p.gl_nodes == 10 ? 0 : 1; }\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-I",
                        os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr



def test_query_arguments_checked_before_any_launch():
    """The binding refuses every malformed tensor before the library is
    called: wrong dtype, wrong shape or dimension, a strided view, outputs
    of the wrong length or type, host tensors, short segment tables and
    mixed 2D / 3D batches (all raise ValueError, no launch)."""
    import torch
    curves, _ = W.config1()
    h = G.gwn_build2d(curves, host_params())
    n = 10
    good = torch.zeros((n, 2), dtype=torch.float64)
    out = torch.zeros(n, dtype=torch.float64)
    ins = torch.zeros(n, dtype=torch.uint8)
    cases = [
        (good.float(), out, ins, "float64"),
        (torch.zeros((n, 3), dtype=torch.float64), out, ins, "shape"),
        (torch.zeros(2 * n, dtype=torch.float64), out, ins, "[n, 2]"),
        (torch.zeros((n, 4), dtype=torch.float64)[:, ::2], out, ins, "contiguous"),
        (good, torch.zeros(n - 1, dtype=torch.float64), ins, "shape"),
        (good, out.float(), ins, "float64"),
        (good, out, torch.zeros(n, dtype=torch.int32), "uint8"),
        (good, out, torch.zeros(n + 1, dtype=torch.uint8), "shape"),
        (good, out, ins, "GPU"),
        (np.zeros((n, 2)), out, ins, "tensor"),
    ]
    for pts, o, i, msg in cases:
        for fn in (G.gwn_query, G.gwn_query_noalloc):
            with pytest.raises(ValueError, match=msg):
                fn(h, pts, o, i)
    with pytest.raises(ValueError, match="counters"):
        G.gwn_query_counters(h, good, torch.zeros(3, dtype=torch.int64))
    with pytest.raises(ValueError, match="n_seg"):
        G.gwn_query_batch([h, h], np.array([0, n]), good, out, ins)
    with pytest.raises(ValueError, match="non-decreasing"):
        G.gwn_query_batch([h, h], np.array([0, 6, 4]), good, out, ins)
    with pytest.raises(ValueError, match="shape"):
        G.gwn_query_batch([h, h], np.array([0, 4, 12]), good, out, ins)
    P = W.Patches3D.from_list([(cp, w, []) for cp, w in W.bodies(0, [("sphere", (0, 0, 0), 1.0)], disp=0.0)][:4])
    h3 = G.gwn_build3d(P, host_params())
    with pytest.raises(ValueError, match="one dimension"):
        G.gwn_query_batch([h, h3], np.array([0, 4, 8]), good, out, ins)
    with pytest.raises(ValueError, match="shape"):
        G.gwn_query(h3, good, out, ins)
    G.gwn_free(h)
    G.gwn_free(h3)


def test_overflow_count_semantics_documented():
    """The device overflow count is never reset; the header states that
    each overflowing call is reported once, by a later call."""
    src = open(os.path.join(ROOT, "include", "gwn.h")).read()
    assert "reported once" in src
