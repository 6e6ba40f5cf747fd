"""The persistent kernels' work queues, built by the library's own host code for
random batches and checked without a GPU by `queue_check.cpp`: runs partition
the tiles, queues partition the runs, every tile of every generation appears
exactly once, table-form strips cover each packet exactly, and a generation's
tiles share one queue."""
import os
import shutil
import subprocess

import pytest

import paper_1909_02871_amd as gf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_queue_invariants(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    gf.lib()                                  # the library is built
    libdir = os.path.dirname(gf.LIB_PATH)
    exe = str(tmp_path / "queue_check")
    cmd = [hipcc, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1909_02871_amd", "csrc"), os.path.join(ROOT, "tests", "queue_check.cpp"),
           "-L", libdir, "-lgfnc", "-Wl,-rpath," + libdir, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "queue checks ok" in r.stdout
