"""PDEP block Davidson on chi-bar0 = v^{1/2} chi0 v^{1/2} through the C ABI (stern_pdep_davidson),
against the dense reference built from the sum over all empty states (tiny model cell) and the
discrete Lindhard closed form (free electrons)."""
import math

import numpy as np
import pytest

from oracle import OracleCell
from oracle.pdep import chibar0_dense, coords_from_coefficients, free_electron_eigs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dense_tiny(tiny_system):
    M, reps = chibar0_dense(tiny_system["cell"], 16, 2.5)
    return 0.5 * (M + M.T), reps


def _system(tiny_system):
    from paper_2607_14025_amd import System
    sp, gs = tiny_system["spec"], tiny_system["gs"]
    s = System(sp.L, sp.ecut, gs["pos"])
    s.set_occupied(gs["psi"], gs["eps"])
    return s


def test_davidson_matches_dense_chibar0(tiny_system, dense_tiny):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    M, reps = dense_tiny
    ref = np.linalg.eigvalsh(M)
    s = _system(tiny_system)
    n = 8
    eig, vec, info = s.pdep_davidson(n, tol=1e-7, block=8, max_basis=40, chi0_tol=1e-11, seed=3)
    s.close()
    print("pdep:", {k: v for k, v in info.items() if k != "miller"}, "eig", eig, "ref", ref[:n])
    assert info["n_converged"] == n and info["basis_dim"] == 80
    assert np.all(eig < 0)
    assert np.abs(eig - ref[:n]).max() <= 1e-8 * np.abs(ref).max()
    # eigenpotentials: unit norm, Hermitian, and eigenvectors of the dense matrix
    u = coords_from_coefficients(vec, info["miller"], reps)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-12)
    r = np.linalg.norm(u @ M - eig[:, None] * u, axis=1) / np.abs(eig)
    assert r.max() <= 1e-6, r
    mil = info["miller"]
    key = {tuple(m): k for k, m in enumerate(mil.tolist())}
    neg = np.array([key[(-a, -b, -c)] for a, b, c in mil.tolist()])
    assert np.allclose(vec[:, neg], vec.conj(), atol=1e-14)


def test_davidson_free_electrons_match_lindhard():
    """No wells, no projectors, a closed shell of 7 plane waves: the eigenvalues are the discrete
    Lindhard sums, (4 pi / |q|^2)(-2 S(q) / Omega), each twice."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System
    from paper_2607_14025_amd.stern import basis_info
    L, ecut = 10.0, 10.0
    npw, N, mil = basis_info(L, ecut)
    n2 = (mil.astype(np.int64) ** 2).sum(axis=1)
    occ = np.flatnonzero(n2 <= 1)
    assert len(occ) == 7
    psi = np.zeros((7, npw), dtype=np.complex128)
    psi[np.arange(7), occ] = 1.0
    eps = 0.5 * (2 * math.pi / L) ** 2 * n2[occ].astype(float)
    s = System(L, ecut, np.zeros((0, 3)))
    s.set_occupied(psi, eps)
    eig, vec, info = s.pdep_davidson(6, tol=1e-8, block=6, chi0_tol=1e-12, seed=1)
    s.close()
    ref = free_electron_eigs(OracleCell(L, ecut, np.zeros((0, 3))), 7, ecut / 4)
    print("free electrons:", eig, ref[:6])
    assert info["n_converged"] == 6
    assert np.abs(eig - ref[:6]).max() <= 1e-9 * np.abs(ref).max()


def test_davidson_with_mixed_precision_chi0(tiny_system, dense_tiny):
    """The chi0 applies in mixed precision (FP64 true residual 1e-9): eigenvalues within 1e-7."""
    from paper_2607_14025_amd import STERN_MIXED
    M, _ = dense_tiny
    ref = np.linalg.eigvalsh(M)
    s = _system(tiny_system)
    eig, _, info = s.pdep_davidson(4, tol=1e-6, chi0_tol=1e-9, precision=STERN_MIXED, seed=5)
    s.close()
    assert info["n_converged"] == 4
    assert np.abs(eig - ref[:4]).max() <= 1e-7 * np.abs(ref).max()


def test_davidson_refuses_bad_requests(tiny_system):
    from paper_2607_14025_amd.stern import SternError
    s = _system(tiny_system)
    with pytest.raises(SternError):
        s.pdep_davidson(0)
    with pytest.raises(SternError):
        s.pdep_davidson(81)            # more than the 80 potentials of the basis
    with pytest.raises(SternError):
        s.pdep_davidson(2, ecut_pot=20.0)  # beyond the wave-function cutoff
    s.close()
