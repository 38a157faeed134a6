"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from synth.cells import TINY, MID, batched_specs, miller_sorted
from oracle import sphere_miller

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stern.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "workload_sizes.json")

stern = pytest.importorskip("paper_2607_14025_amd.stern")


def _lib_or_skip():
    if not os.path.exists(stern.LIB_PATH):
        pytest.skip("libstern.so not built")
    return stern.lib()


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    decl = set(re.findall(r"^(?:int|void|const char\*)\s+(stern_[a-z0-9_]+)\s*\(", open(HEADER).read(), re.M))
    assert decl, "no declarations parsed"
    assert decl == set(stern.EXPORTED)
    for name in decl:
        assert hasattr(L, name), name


def test_basis_sizes_match_workloads():
    _lib_or_skip()
    g = json.load(open(GOLDEN))
    for c in g["cells"][:2]:
        npw, N, mil = stern.basis_info(c["L"], c["ecut"])
        assert (npw, N) == (c["npw"], c["grid"])


def test_canonical_order_matches_generator_and_oracle():
    _lib_or_skip()
    for L, e in [(TINY.L, TINY.ecut), (13.37, 20.0)]:
        npw, N, mil = stern.basis_info(L, e)
        assert np.array_equal(mil, miller_sorted(L, e))
        assert np.array_equal(mil, sphere_miller(L, e))
    for sp in batched_specs()[:3]:
        npw, N, mil = stern.basis_info(sp.L, sp.ecut)
        assert N in (32, 36, 48, 54)


def test_invalid_arguments_rejected():
    _lib_or_skip()
    with pytest.raises(stern.SternError) as e:
        stern.basis_info(-1.0, 10.0)
    assert e.value.code == -1
    with pytest.raises(stern.SternError):
        stern.basis_info(10.0, 10.0, fft_n=12)  # too small for the 4 Ecut sphere
    with pytest.raises(stern.SternError):
        # 4 nmax + 1 = 9 holds the differences of sphere points, but the 4 Ecut sphere of
        # V_loc reaches |n| = 5, which a 9-point grid would alias
        stern.basis_info(10.0, 2.5, fft_n=9)
    assert stern.basis_info(10.0, 2.0, fft_n=9)[1] == 9
    L = stern.lib()
    assert L.stern_basis_info(None, None, None, None) == -1
    assert b"NULL" in L.stern_last_error()
    rc = L.stern_apply_chi0(None, 1, None, None, None, None)
    assert rc == -1
    L.stern_free(None)  # NULL-safe
