"""The library's host code (csrc/basis.cpp, csrc/hostla.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: built with g++ (host only, no GPU code), run over the cells of the
workloads (the tiny, mid, learned and large cells, two uneven cells and the grid-limit sizes), with
the basis sizes checked against the oracle's sphere, and over random matrices for the Jacobi
eigensolvers of the Davidson iterations."""
import os
import shutil
import subprocess

import pytest

from oracle import fft_grid, sphere_miller

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2607_14025_amd", "csrc")


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    from synth.cells import LARGE, LEARNED, MID, TINY, batched_specs
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "sanitize_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(HERE, "host", "sanitize_driver.cpp"),
           os.path.join(CSRC, "basis.cpp"), os.path.join(CSRC, "hostla.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    b = sorted(batched_specs(), key=lambda c: c.L)
    cells = [(c.L, c.ecut, c.n_atoms, 0) for c in (TINY, MID, LEARNED, LARGE, b[0], b[-1])]
    cells += [(4.0, 5.0, 1, 9), (8.0, 6.0, 3, 0)]
    inp = "".join(f"{L} {e} {n} {f}\n" for L, e, n, f in cells)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("cell")]
    assert len(lines) == len(cells)
    for (L, e, n, f), ln in zip(cells, lines):
        assert "npw" in ln, ln
        npw = int(ln.split(" npw ")[1].split()[0])
        N = int(ln.split(" N ")[1].split()[0])
        assert npw == len(sphere_miller(L, e))
        assert N == (f if f else fft_grid(L, e))
    assert sum(ln.startswith("jacobi") for ln in r.stdout.splitlines()) == 6
