"""The library's host planning (csrc/plan.cpp: column offsets and their lookup, negligible-
block windows, cluster trees and block partition) built for the CPU with the address and
undefined-behaviour sanitizers (g++; no GPU code involved) and run on ring geometries of
the workloads' kind -- single cells of several sizes, odd and tiny ones, and a multi-cell
set -- by tests/plan_check.cpp, which also checks the plans' invariants."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import fbc_workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2105_08798_amd", "csrc")


def _write_sets(path, sets):
    with open(path, "wb") as fp:
        np.asarray([len(sets)], dtype=np.int32).tofile(fp)
        for cells in sets:
            np.asarray([len(cells)], dtype=np.int32).tofile(fp)
            for ci, cb in cells:
                np.asarray([len(ci), len(cb)], dtype=np.int32).tofile(fp)
                np.ascontiguousarray(ci, dtype=np.int32).tofile(fp)
                np.ascontiguousarray(cb, dtype=np.int32).tofile(fp)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(CSRC, "plan.cpp"),
           os.path.join(HERE, "plan_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    sets = []
    for n_i, n_b in ((1, 1), (7, 11), (96, 192), (300, 301), (640, 1280)):
        ci, cb = W.ring_columns(n_i, n_b)
        sets.append([(ci, cb)])
    sets.append([W.ring_columns(n_i, n_b) for n_i, n_b in ((40, 80), (13, 30), (200, 400))])
    geo = str(tmp_path / "geometry.bin")
    _write_sets(geo, sets)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, geo], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
