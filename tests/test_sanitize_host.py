"""Host code under AddressSanitizer and UBSan, on the CPU: the engine's host
builders (tree, 2D and 3D subdivision with trim clipping, NURBS extraction,
the budgeted far test) and the oracle, each compiled with
-fsanitize=address,undefined into a small driver and run on a case file of
seeded workloads (star loop, overlapping polygons, NURBS curves, bodies
and CAD patches with holes).  Any sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2605_19200_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2605_19200_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _arr(f, a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype).reshape(-1)
    f.write(np.int64(a.size).tobytes())
    f.write(a.tobytes())


@pytest.fixture(scope="module")
def case(tmp_path_factory):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    C = W.star_loop(1, 64).concat(W.overlapping_polygons(4))
    rng = W.Rng(91, "sanitize-nurbs")
    nurbs = []
    for p in (1, 2, 3):
        n = p + 4
        pts = np.stack([np.cos(np.linspace(0, 5, n)), np.sin(np.linspace(0, 5, n))], 1) + rng.uniform((n, 2), 0, .1)
        inner = np.sort(rng.uniform(n - p - 1, 0.1, 0.9))
        nurbs.append((p, pts, rng.uniform(n, 0.5, 2.0), np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])))
    N = W.Nurbs2D.from_list(nurbs)
    P3, _ = W.config3(grid=0)
    P4 = W.cad_assembly(4, n_bodies=2)
    P = P3.subset(np.arange(0, P3.n, 16)).concat(P4.subset(np.arange(0, P4.n, 4)))
    from tests.test_nurbs3d import nurbs_cube
    S3 = nurbs_cube(W.Rng(94, "sanitize-nurbs3d"))
    q2 = W.bbox_queries_uniform(W.Rng(92, "sanitize-q2"), *C.bbox(), 24)
    q3 = W.bbox_queries_uniform(W.Rng(93, "sanitize-q3"), *P.bbox(), 6)
    path = str(tmp_path_factory.mktemp("san") / "case.bin")
    with open(path, "wb") as f:
        _arr(f, C.degree, np.int32), _arr(f, C.cp_offset, np.int64), _arr(f, C.cp_xy, np.float64)
        _arr(f, C.cp_w, np.float64)
        _arr(f, N.degree, np.int32), _arr(f, N.cp_offset, np.int64), _arr(f, N.cp_xy, np.float64)
        _arr(f, N.cp_w, np.float64), _arr(f, N.knot_offset, np.int64), _arr(f, N.knots, np.float64)
        _arr(f, P.cp_xyz, np.float64), _arr(f, P.cp_w, np.float64), _arr(f, P.trim_offset, np.int64)
        _arr(f, P.trim_degree, np.int32), _arr(f, P.trim_cp_offset, np.int64)
        _arr(f, P.trim_cp_uv, np.float64), _arr(f, P.trim_cp_w, np.float64)
        _arr(f, q2, np.float64), _arr(f, q3, np.float64)
        S, T = S3, S3.trims
        for a, dt in ((S.degree_u, np.int32), (S.degree_v, np.int32), (S.n_u, np.int32), (S.n_v, np.int32),
                      (S.cp_offset, np.int64), (S.cp_xyz, np.float64), (S.cp_w, np.float64),
                      (S.knot_u_offset, np.int64), (S.knots_u, np.float64), (S.knot_v_offset, np.int64),
                      (S.knots_v, np.float64), (S.trim_offset, np.int64), (T.degree, np.int32),
                      (T.cp_offset, np.int64), (T.cp_xy, np.float64), (T.cp_w, np.float64),
                      (T.knot_offset, np.int64), (T.knots, np.float64)):
            _arr(f, a, dt)
    return path, C, P, q2, q3


def test_host_builders_sanitized(case, tmp_path):
    path = case[0]
    exe = str(tmp_path / "host")
    srcs = [os.path.join(CSRC, s) for s in ("tree.cpp", "build2d.cpp", "build3d.cpp", "trimclip.cpp", "nurbs.cpp")]
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-pthread", "-I", CSRC, os.path.join(HERE, "sanitize_host.cpp"),
                           *srcs, "-o", exe])
    r = subprocess.run([exe, path], capture_output=True, text=True, env=ENV, timeout=900)
    print(r.stdout)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.splitlines()
    assert sum(ln.startswith("2d ") for ln in lines) == 4 and sum(ln.startswith("3d ") for ln in lines) == 2
    assert any(ln.startswith("nurbs: ") and "segments" in ln for ln in lines)
    assert any(ln.startswith("nurbs3d: ") and "patches" in ln for ln in lines)


def test_oracle_sanitized(case, tmp_path, oracle):
    path, C, P, q2, q3 = case
    exe = str(tmp_path / "oracle")
    subprocess.check_call(["gcc", "-std=c11", *SAN, os.path.join(ROOT, "oracle", "gwn_oracle.c"),
                           os.path.join(HERE, "sanitize_oracle.c"), "-lm", "-o", exe])
    r = subprocess.run([exe, path], capture_output=True, text=True, env=ENV, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.splitlines()
    assert lines[0] == "unconverged2d 0" and lines[1] == "unconverged3d 0"
    got = np.array([float(x) for x in lines[2:]])
    ref = np.concatenate([oracle.gwn2d(C, q2, eps_on=1e-12), oracle.gwn3d(P, q3, eps_on=1e-12)])
    assert np.allclose(got, ref, rtol=0, atol=1e-12)
