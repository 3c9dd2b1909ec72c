"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Two executables are built with gcc/g++ ``-fsanitize=address,undefined`` from
the sources in tests/sanitize/: one drives the oracle and the graph
generators over small graphs (degenerate ones included) and checks their
mutual promises; the other drives the library's pure host code -- the
block-table checker and the host-thread per-task count of the hybrid
execution -- over block tables built here from the oracle's oriented graph by
the layout's definitions.  Any out-of-bounds access, use after free, leak or
undefined operation aborts the run; the host count is also compared task by
task with the oracle's per-task counts (the two share no code: they meet only
in this test)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import graphgen
import oracle

from test_layout_cpu import reference_tables, tables_np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitize")
    od, hd = str(d / "oracle_driver"), str(d / "host_driver")
    subprocess.check_call(["gcc", "-std=c11", *SAN, "-fopenmp", "-o", od,
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "graphgen", "graphgen.c"),
                           "-lm"])
    csrc = os.path.join(ROOT, "paper_2009_12457_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", csrc, "-I", os.path.join(ROOT, "include"), "-o", hd,
                           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                           os.path.join(csrc, "cpu_count.cpp")])
    return od, hd


def _run(cmd):
    out = subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert "Sanitizer" not in out.stderr and "runtime error" not in out.stderr, out.stderr[-4000:]
    return out.stdout


def test_oracle_and_generators_clean(drivers):
    out = _run([drivers[0]])
    assert out.strip().splitlines()[-1] == "oracle driver: all checks passed"
    # the graphs the driver builds, with the triangle counts the Python side of
    # the oracle finds for the same edge lists
    lines = dict(l.split(" ", 1) for l in out.strip().splitlines()[:-1])
    assert lines["triangle"].endswith("triangles=1")
    assert lines["single"].endswith("triangles=0") and lines["empty7"].endswith("triangles=0")


def _write_tables(path, t):
    with open(path, "wb") as f:
        np.array([t["n"], t["m"], t["p"], t["rT"]], np.int64).tofile(f)
        for k in ("cuts", "orow", "ocol", "botp", "bot", "acp", "acol", "aoff", "icolb"):
            a = np.ascontiguousarray(t[k])
            np.array([a.size], np.int64).tofile(f)
            a.tofile(f)


@pytest.mark.parametrize("name,p,T", [("er2000", 4, 32), ("rmat10", 7, 8), ("rmat10", 16, -1), ("rmat11", 3, 0),
                                      ("rmat10", 1, 1 << 30), ("rmat10", 31, 1 << 30)])
def test_host_count_and_checker_clean(drivers, tmp_path, name, p, T):
    g = graphgen.workload(name)
    t = tables_np(reference_tables(g, p, T))
    path = str(tmp_path / "tables.bin")
    _write_tables(path, t)
    out = _run([drivers[1], path]).strip().splitlines()
    assert out[0] == "tables: ok", out[0]
    ntask = p * (p + 1) * (p + 2) // 6
    rows = [l.split() for l in out[1:1 + ntask]]
    got = np.array([int(r[3]) for r in rows], np.uint64)
    assert [tuple(map(int, r[:3])) for r in rows] == [(i, j, k) for i in range(p) for j in range(i, p)
                                                      for k in range(j, p)]
    og = oracle.OracleGraph.from_graph(g)
    want_tot, want_per, _ = og.tasks(p, og.cuts(p))
    assert np.array_equal(got, want_per) and int(got.sum()) == want_tot
    rejected = out[1 + ntask:]
    assert rejected and all(not l.endswith(": ok") for l in rejected), rejected
