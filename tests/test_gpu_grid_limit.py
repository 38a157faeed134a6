"""Grids at the limit the compact plane kernels rely on.

Those kernels skip, without a test, the y and z ranges strictly between [0, m] and
[N - m, N) with m = floor((N - 1) / 4), which holds every sphere index when
N >= 4 nmax + 1. On grids with nmax = m (N = 9, 27, 81 with nmax = 2, 6, 20) the
outermost active index is m itself, so a skipped range off by one would drop live data.
Each grid also holds the 4 Ecut sphere of V_loc, as the basis requires. Checked against
the oracle: the FP64 H apply of every plane variant, and the FP64 and mixed chi0 paths on
the 27^3 cell (L = 10 bohr, 16 Ry, its default grid)."""
import numpy as np
import pytest

from oracle import OracleCell, apply_chi0
from oracle.sternheimer import rel_l2
from synth.cells import CellSpec, place_atoms, random_dv

pytestmark = pytest.mark.gpu

CASES = [(10.0, 2.0, 9, 2), (10.0, 16.0, 27, 6), (20.0, 41.0, 81, 20)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("L,ecut,N,nmax", CASES)
def test_h_apply_at_the_grid_limit(L, ecut, N, nmax, torch_cuda):
    from paper_2607_14025_amd import System
    from paper_2607_14025_amd.stern import TUNE_PLANE64
    spec = CellSpec(f"limit_{N}", 7, L, ecut, 8, 4, 1)
    pos = place_atoms(spec)
    cell = OracleCell(L, ecut, pos, N=N)
    assert int(np.abs(cell.miller).max()) == nmax == (N - 1) // 4
    s = System(L, ecut, pos, fft_n=N)
    assert s.fft_n == N and s.n_pw == cell.npw
    rng = np.random.default_rng(23)
    c = rng.standard_normal((3, cell.npw)) + 1j * rng.standard_normal((3, cell.npw))
    shift = np.array([0.4, -0.9, 0.0])
    ref = cell.h_apply(c) - shift[:, None] * c
    for v in (0, 1, 2):
        s.tunable(TUNE_PLANE64, v)
        out = s.apply_h(c, shift)
        assert (np.linalg.norm(out - ref, axis=1) / np.linalg.norm(ref, axis=1)).max() < 1e-13, v
    s.close()


def test_chi0_at_the_grid_limit(torch_cuda):
    """16 bands x 2 fields on the 27^3 cell (nmax = 6 = (27 - 1) / 4): both precisions, and
    the FP32 plane kernel variants, against the oracle's dn."""
    from paper_2607_14025_amd import System, STERN_FP64, STERN_MIXED
    from paper_2607_14025_amd.stern import TUNE_PLANE32
    from synth.ground import ground_state
    spec = CellSpec("limit_27_chi0", 7, 10.0, 16.0, 8, 16, 2)
    gs = ground_state(spec)
    sp = gs["spec"]
    cell = OracleCell(sp.L, sp.ecut, gs["pos"])
    assert cell.N == 27 and int(np.abs(cell.miller).max()) == 6
    _, _, dv = random_dv(sp)
    psi = cell.take(gs["psi"], gs["miller"])
    ref = apply_chi0(cell, psi, gs["eps"], dv, tol=1e-12)
    s = System(sp.L, sp.ecut, gs["pos"], sp.vloc_amp, sp.vloc_sigma, sp.kb_D, sp.kb_width)
    s.set_occupied(gs["psi"], gs["eps"])
    dn, info = s.apply_chi0(dv, tol=1e-10, precision=STERN_FP64)
    assert info["n_converged"] == 32 and rel_l2(dn, ref["dn"]).max() < 1e-9
    for v in (0, 1, 2):
        s.tunable(TUNE_PLANE32, v)
        dm, info = s.apply_chi0(dv, tol=1e-10, precision=STERN_MIXED)
        assert info["n_converged"] == 32 and rel_l2(dm, ref["dn"]).max() < 1e-6, v
    s.close()
