"""Kernel variants and the autotuner through the C ABI: every variant the tuner can
pick gives results within the parity bounds, and its cache round-trips."""
import numpy as np
import pytest

from oracle import OracleCell, apply_chi0
from oracle.sternheimer import rel_l2
from synth.cells import CellSpec, place_atoms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tuned_tiny(tiny_system):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System
    t = tiny_system
    s = System(t["spec"].L, t["spec"].ecut, t["gs"]["pos"])
    s.set_occupied(t["gs"]["psi"], t["eps"])
    ref = apply_chi0(t["cell"], t["psi"], t["eps"], t["dv"][:3], tol=1e-12)
    yield {**t, "sys": s, "ref": ref, "dv": t["dv"][:3]}
    s.close()


def test_tunable_round_trip_and_errors(tuned_tiny):
    from paper_2607_14025_amd import SternError
    from paper_2607_14025_amd.stern import TUNE_PLANE64, TUNE_GEMM16_WG
    s = tuned_tiny["sys"]
    old = s.tunable(TUNE_PLANE64)
    assert s.tunable(TUNE_PLANE64, 0) == 0 and s.tunable(TUNE_PLANE64) == 0
    s.tunable(TUNE_PLANE64, old)
    assert s.tunable(TUNE_GEMM16_WG, 256) == 256
    s.tunable(TUNE_GEMM16_WG, 0)
    from paper_2607_14025_amd.stern import TUNE_GEMM16_EXPAND
    for which, value in ((7, 0), (TUNE_PLANE64, 3), (TUNE_GEMM16_WG, 1 << 20), (TUNE_GEMM16_EXPAND, 3)):
        with pytest.raises(SternError) as e:
            s.tunable(which, value)
        assert e.value.code == -1


@pytest.mark.parametrize("L,ecut,natoms", [(10.0, 10.0, 8), (12.5, 20.0, 9), (20.0, 25.0, 7)])
def test_plane_variants_match_oracle(L, ecut, natoms, tiny_system):
    """(H - shift) c through both yz-plane kernels, FP64, against the oracle."""
    from paper_2607_14025_amd import System
    from paper_2607_14025_amd.stern import TUNE_PLANE64
    spec = CellSpec(f"variants_{L}", 7, L, ecut, natoms, 4, 1)
    pos = place_atoms(spec)
    cell = OracleCell(L, ecut, pos)
    s = System(L, ecut, pos)
    rng = np.random.default_rng(5)
    c = rng.standard_normal((3, cell.npw)) + 1j * rng.standard_normal((3, cell.npw))
    shift = np.array([0.2, -0.7, 1.1])
    ref = cell.h_apply(c) - shift[:, None] * c
    for v in (0, 1, 2):
        s.tunable(TUNE_PLANE64, v)
        out = s.apply_h(c, shift)
        assert (np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)).max() < 1e-13, v
    s.close()


def test_every_variant_keeps_parity(tuned_tiny):
    from paper_2607_14025_amd import STERN_MIXED
    from paper_2607_14025_amd.stern import (TUNE_PLANE64, TUNE_PLANE32, TUNE_GEMM64_WG, TUNE_GEMM16_WG,
                                            TUNE_GEMM16_EXPAND)
    t = tuned_tiny
    s = t["sys"]
    for p64, p32, g64, g16, ex in ((0, 0, 256, 128, 0), (1, 1, 4096, 2048, 1), (2, 2, 0, 0, 2), (1, 0, 0, 0, 2)):
        s.tunable(TUNE_PLANE64, p64)
        s.tunable(TUNE_PLANE32, p32)
        s.tunable(TUNE_GEMM64_WG, g64)
        s.tunable(TUNE_GEMM16_WG, g16)
        s.tunable(TUNE_GEMM16_EXPAND, ex)
        dn, info = s.apply_chi0(t["dv"], tol=1e-10)
        assert info["n_converged"] == 48 and rel_l2(dn, t["ref"]["dn"]).max() < 1e-9
        dm, info = s.apply_chi0(t["dv"], tol=1e-10, precision=STERN_MIXED)
        assert info["n_converged"] == 48 and rel_l2(dm, t["ref"]["dn"]).max() < 1e-6
    # the expand tiles differ only in how outputs are spread over workgroups: each output
    # takes the same products in the same order, so the mixed path is bitwise the same
    out = []
    for ex in (0, 1, 2):
        s.tunable(TUNE_GEMM16_EXPAND, ex)
        out.append(s.apply_chi0(t["dv"], tol=1e-10, precision=STERN_MIXED)[0])
    assert all(np.array_equal(out[0], o) for o in out[1:])


def test_autotune_and_cache(tuned_tiny, tmp_path):
    from paper_2607_14025_amd import STERN_MIXED
    t = tuned_tiny
    s = t["sys"]
    cache = tmp_path / "tune.txt"
    n, chosen = s.autotune(n_vec=64, cache_path=str(cache))
    assert n >= 16
    assert chosen["plane64"] in (0, 1, 2) and chosen["plane32"] in (0, 1, 2)
    assert chosen["gemm64_wg"] in (256, 384, 512, 768, 1024, 2048, 4096)
    assert chosen["gemm16_wg"] in (128, 192, 256, 384, 512, 1024, 2048)
    assert chosen["gemm16_expand"] in (0, 1, 2)
    assert len(cache.read_text().splitlines()) == 5
    n2, chosen2 = s.autotune(n_vec=64, cache_path=str(cache))
    assert n2 == 0 and chosen2 == chosen
    dn, info = s.apply_chi0(t["dv"], tol=1e-10)
    assert info["n_converged"] == 48 and rel_l2(dn, t["ref"]["dn"]).max() < 1e-9
    dm, info = s.apply_chi0(t["dv"], tol=1e-10, precision=STERN_MIXED)
    assert info["n_converged"] == 48 and rel_l2(dm, t["ref"]["dn"]).max() < 1e-6
