"""GPU parity of the HIP path against the CPU oracle, called through the C ABI."""
import numpy as np
import pytest

from oracle import OracleCell, apply_chi0, project
from oracle.sternheimer import rel_l2, chi0_matrix
from synth.cells import CellSpec, TINY, place_atoms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _system(spec, pos, torch_cuda):
    from paper_2607_14025_amd import System
    return System(spec.L, spec.ecut, pos, spec.vloc_amp, spec.vloc_sigma, spec.kb_D, spec.kb_width)


@pytest.fixture(scope="module")
def tiny_gpu(tiny_system, torch_cuda):
    t = tiny_system
    sys_ = _system(t["spec"], t["gs"]["pos"], torch_cuda)
    assert sys_.n_pw == t["cell"].npw and sys_.fft_n == t["cell"].N
    sys_.set_occupied(t["gs"]["psi"], t["eps"])
    ref = apply_chi0(t["cell"], t["psi"], t["eps"], t["dv"], tol=1e-12)
    yield dict(sys=sys_, ref=ref, **t)
    sys_.close()


def _rand(rng, n, npw):
    return rng.standard_normal((n, npw)) + 1j * rng.standard_normal((n, npw))


@pytest.mark.parametrize("L,ecut,natoms", [(10.0, 10.0, 8), (11.0, 20.0, 6), (12.5, 20.0, 9), (15.0, 20.0, 12),
                                           (17.5, 20.0, 5), (20.0, 25.0, 7)])
def test_h_apply_matches_oracle(L, ecut, natoms, torch_cuda):
    """(H - shift) c through the pruned FFT, V_loc and KB kernels, grids 24 to 72."""
    spec = CellSpec(f"happly_{L}", 7, L, ecut, natoms, 4, 1)
    pos = place_atoms(spec)
    cell = OracleCell(L, ecut, pos)
    s = _system(spec, pos, torch_cuda)
    assert s.fft_n == cell.N
    rng = np.random.default_rng(11)
    c = _rand(rng, 3, cell.npw)
    shift = np.array([0.3, -1.2, 0.0])
    out = s.apply_h(c, shift)
    ref = cell.h_apply(c) - shift[:, None] * c
    err = np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)
    s.close()
    assert err.max() < 1e-13, err


def test_pc_matches_oracle(tiny_gpu):
    t = tiny_gpu
    rng = np.random.default_rng(3)
    y = _rand(rng, 5, t["cell"].npw)
    out = t["sys"].apply_pc(y)
    ref = project(t["psi"], y)
    assert np.max(np.linalg.norm(out - ref, axis=1) / np.linalg.norm(y, axis=1)) < 1e-14


def test_chi0_tiny_matches_oracle(tiny_gpu):
    t = tiny_gpu
    pairs = [(0, 0), (15, 0), (7, 3), (3, 7)]
    dn, info = t["sys"].apply_chi0(t["dv"], tol=1e-12, samples=pairs)
    assert info["rc"] == 0 and info["n_converged"] == info["n_solves"] == 128
    assert info["max_true_resid"] <= 1e-12
    assert rel_l2(dn, t["ref"]["dn"]).max() < 1e-9
    for k, (v, i) in enumerate(pairs):
        ref = t["ref"]["x"][t["ref"]["pairs"].index((v, i))]
        assert np.linalg.norm(info["samples"][k] - ref) / np.linalg.norm(ref) < 1e-9


def test_chi0_tiny_at_workload_tolerance(tiny_gpu):
    """At the tiny workload's CG tolerance (1e-10) dn still meets 1e-9 against the 1e-12 oracle."""
    t = tiny_gpu
    dn, info = t["sys"].apply_chi0(t["dv"], tol=1e-10)
    assert info["n_converged"] == 128
    assert rel_l2(dn, t["ref"]["dn"]).max() < 1e-9
    M = chi0_matrix(t["cell"], t["dv"], dn)
    assert np.linalg.norm(M - M.T) / np.linalg.norm(M) < 1e-9
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).max() <= 1e-9 * np.linalg.norm(M)
    assert np.abs(dn.sum(axis=(1, 2, 3))).max() < 1e-10 * np.abs(dn).sum(axis=(1, 2, 3)).max()


def test_batching_band_ranges_and_determinism(tiny_gpu):
    t = tiny_gpu
    s = t["sys"]
    full, _ = s.apply_chi0(t["dv"], tol=1e-12)
    again, _ = s.apply_chi0(t["dv"], tol=1e-12)
    assert np.array_equal(full, again)
    small, info = s.apply_chi0(t["dv"], tol=1e-12, max_batch=16, check_every=3)
    assert rel_l2(small, full).max() < 1e-11
    lo, _ = s.apply_chi0(t["dv"][:2], tol=1e-12, band_range=(0, 7))
    hi, _ = s.apply_chi0(t["dv"][:2], tol=1e-12, band_range=(7, 16))
    assert rel_l2(lo + hi, full[:2]).max() < 1e-11


def test_device_pointers_match_host(tiny_gpu, torch_cuda):
    torch = torch_cuda
    t = tiny_gpu
    dv = torch.from_numpy(t["dv"][:3]).cuda()
    dn, info = t["sys"].apply_chi0(dv, tol=1e-12)
    torch.cuda.synchronize()
    host, _ = t["sys"].apply_chi0(t["dv"][:3], tol=1e-12)
    assert np.array_equal(dn.cpu().numpy(), host)


def test_error_paths(tiny_system, torch_cuda):
    from paper_2607_14025_amd import System, SternError
    t = tiny_system
    s = System(t["spec"].L, t["spec"].ecut, t["gs"]["pos"])
    with pytest.raises(SternError) as e:
        s.apply_chi0(t["dv"][:1])
    assert e.value.code == -2
    s.set_occupied(t["gs"]["psi"], t["eps"])
    with pytest.raises(SternError) as e:
        s.apply_chi0(t["dv"][:1], band_range=(5, 3))
    assert e.value.code == -1
    _, info = s.apply_chi0(t["dv"][:1], tol=1e-12, max_iter=2)
    assert info["rc"] == 1 and info["n_converged"] < info["n_solves"]
    s.close()


def test_chi0_tiny_mixed_precision(tiny_gpu):
    """FP32 FFTs + split-BF16 MFMA GEMMs inside FP64 defect correction: dn within 1e-6 of the oracle,
    every solve accepted by the FP64 true residual."""
    from paper_2607_14025_amd import STERN_MIXED
    t = tiny_gpu
    pairs = [(0, 0), (15, 7)]
    dn, info = t["sys"].apply_chi0(t["dv"], tol=1e-10, precision=STERN_MIXED, samples=pairs)
    assert info["n_converged"] == 128 and info["max_true_resid"] <= 1e-10
    assert rel_l2(dn, t["ref"]["dn"]).max() < 1e-6
    for k, pr in enumerate(pairs):
        ref = t["ref"]["x"][t["ref"]["pairs"].index(pr)]
        assert np.linalg.norm(info["samples"][k] - ref) / np.linalg.norm(ref) < 1e-7


def test_mixed_fallback_path(tiny_gpu):
    """With one defect-correction step and a loose inner tolerance the unconverged solves
    are re-solved by FP64 PCG from zero and still meet the tolerance."""
    from paper_2607_14025_amd import STERN_MIXED
    t = tiny_gpu
    dn, info = t["sys"].apply_chi0(t["dv"][:2], tol=1e-10, precision=STERN_MIXED, max_outer=1, inner_tol=1e-2)
    assert info["n_fallback"] > 0
    assert info["n_converged"] == 32
    assert rel_l2(dn, t["ref"]["dn"][:2]).max() < 1e-6


@pytest.mark.parametrize("op", ["projected", "shifted"])
def test_mixed_inner_operators(tiny_gpu, op):
    """Both inner operators of the mixed solve give accepted solutions within the mixed
    bound of the oracle."""
    import paper_2607_14025_amd as P
    t = tiny_gpu
    code = {"projected": P.STERN_INNER_PROJECTED, "shifted": P.STERN_INNER_SHIFTED}[op]
    dn, info = t["sys"].apply_chi0(t["dv"], tol=1e-10, precision=P.STERN_MIXED, inner_op=code)
    assert info["n_converged"] == 128 and info["max_true_resid"] <= 1e-10 and info["n_fallback"] == 0
    assert rel_l2(dn, t["ref"]["dn"]).max() < 1e-6


def test_bad_inner_operator_is_refused(tiny_gpu):
    from paper_2607_14025_amd import STERN_MIXED, SternError
    with pytest.raises(SternError):
        tiny_gpu["sys"].apply_chi0(tiny_gpu["dv"][:1], tol=1e-10, precision=STERN_MIXED, inner_op=2)

def test_mixed_without_atoms(torch_cuda):
    """Free electrons (no atoms, V = 0, the top band a degenerate shell): no KB GEMMs run,
    and both inner operators meet the oracle."""
    import paper_2607_14025_amd as P
    from synth.cells import random_dv
    from synth.ground import ground_state
    spec = CellSpec("free_L10_10Ry", 7, 10.0, 10.0, 0, 7, 4)
    gs = ground_state(spec)
    cell = OracleCell(spec.L, spec.ecut, gs["pos"])
    _, _, dv = random_dv(spec)
    ref = apply_chi0(cell, cell.take(gs["psi"], gs["miller"]), gs["eps"], dv, tol=1e-12)
    s = _system(spec, gs["pos"], torch_cuda)
    s.set_occupied(gs["psi"], gs["eps"])
    try:
        for op in (P.STERN_INNER_PROJECTED, P.STERN_INNER_SHIFTED):
            dn, info = s.apply_chi0(dv, tol=1e-10, precision=P.STERN_MIXED, inner_op=op)
            assert info["n_converged"] == 28 and info["max_true_resid"] <= 1e-10
            assert rel_l2(dn, ref["dn"]).max() < 1e-6
    finally:
        s.close()


def test_degenerate_fields(tiny_gpu):
    """Fields the method maps to zero, mixed into one call with ordinary ones: an all-zero
    field (b = 0: dn exactly 0, nothing to solve) and a constant field (P_c annihilates
    c psi_v, and chi0 . const = 0); the ordinary fields still meet the oracle. Empty
    inputs are refused."""
    import paper_2607_14025_amd as P
    t = tiny_gpu
    s = t["sys"]
    dv = np.concatenate([np.zeros_like(t["dv"][:1]), t["dv"][:2], np.full_like(t["dv"][:1], 0.7)])
    for prec, bound in ((P.STERN_FP64, 1e-9), (P.STERN_MIXED, 1e-6)):
        dn, info = s.apply_chi0(dv, tol=1e-10, precision=prec)
        assert info["n_converged"] == info["n_solves"] == 4 * 16
        assert np.isfinite(dn).all()
        assert np.all(dn[0] == 0.0)
        assert np.all(dn[3] == 0.0)  # every P_c (c psi_v) cut to zero: x = 0
        assert info["max_true_resid"] <= 1e-10
        assert rel_l2(dn[1:3], t["ref"]["dn"][:2]).max() < bound
    with pytest.raises(P.SternError) as e:
        s.apply_chi0(t["dv"][:0])
    assert e.value.code == -1
    with pytest.raises(P.SternError) as e:
        s.apply_chi0(t["dv"][:1], band_range=(3, 3))
    assert e.value.code == -1
