"""Pins of the oracle's density response at imaginary frequency (CPU only)."""
import numpy as np
import pytest

from oracle import OracleCell, sum_over_states
from oracle.frequency import dense_shifted_solve, lindhard_dn_iu, shifted_residual, sum_over_states_iu
from oracle.sternheimer import chi0_matrix, delta_n, rhs


@pytest.fixture(scope="module")
def tiny_sos(tiny_system):
    t = tiny_system
    n_occ = t["spec"].n_occ
    return {u: sum_over_states_iu(t["cell"], n_occ, t["dv"][:3], u) for u in (0.0, 0.3, 1.5)}


def test_zero_frequency_is_the_static_response(tiny_system, tiny_sos):
    t = tiny_system
    occ, eo, xs, dn = sum_over_states(t["cell"], t["spec"].n_occ, t["dv"][:3])
    _, _, xs0, dn0 = tiny_sos[0.0]
    assert np.max(np.abs(xs0 - xs)) <= 1e-13 * np.max(np.abs(xs))
    assert np.max(np.abs(dn0 - dn)) <= 1e-13 * np.max(np.abs(dn))


@pytest.mark.parametrize("u", [0.3, 1.5])
def test_sum_over_states_equals_dense_shifted_solve(tiny_system, tiny_sos, u):
    """Eigen-sum and dense linear solve are independent routes to the same x."""
    t = tiny_system
    occ, eo, xs, _ = tiny_sos[u]
    pairs = [(0, 0), (5, 1), (t["spec"].n_occ - 1, 2)]
    b = rhs(t["cell"], occ, t["dv"], [v for v, _ in pairs], [i for _, i in pairs])
    x = dense_shifted_solve(t["cell"], occ, eo[[v for v, _ in pairs]], b, u)
    for k, (v, i) in enumerate(pairs):
        assert np.linalg.norm(x[k] - xs[i, v]) <= 1e-10 * np.linalg.norm(xs[i, v])
    # the FFT-based operator agrees with the dense one on that solution
    assert np.max(shifted_residual(t["cell"], occ, eo[[v for v, _ in pairs]], b, x, u)) <= 1e-10


def test_response_symmetric_negative_and_decreasing_in_u(tiny_system, tiny_sos):
    t = tiny_system
    mats = {u: chi0_matrix(t["cell"], t["dv"][:3], tiny_sos[u][3]) for u in (0.0, 0.3, 1.5)}
    norms = []
    for u, M in mats.items():
        assert np.max(np.abs(M - M.T)) <= 1e-10 * np.max(np.abs(M))
        assert np.max(np.linalg.eigvalsh(0.5 * (M + M.T))) <= 1e-12 * np.max(np.abs(M))
        norms.append(np.linalg.norm(M))
    assert norms[0] > norms[1] > norms[2]


@pytest.mark.parametrize("n_occ,qn,u", [(7, (1, 0, 0), 0.1), (7, (1, 1, 0), 2.0), (19, (2, 1, 0), 0.7)])
def test_free_electron_lindhard_at_imaginary_frequency(n_occ, qn, u):
    """Closed form against the dense shifted solve (a route that never diagonalises)."""
    cell = OracleCell(8.0, 12.0, np.zeros((0, 3)), amp=0.0, D=0.0)
    order = np.argsort(cell.g2, kind="stable")
    psi = np.zeros((n_occ, cell.npw), dtype=np.complex128)
    psi[np.arange(n_occ), order[:n_occ]] = 1.0
    eps = 0.5 * cell.g2[order[:n_occ]]
    N = cell.N
    j = np.arange(N) * cell.L / N
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    q = np.array(qn) * cell.b
    dv = (2.0 * np.cos(q[0] * X + q[1] * Y + q[2] * Z))[None]
    bands = list(range(n_occ))
    b = rhs(cell, psi, dv, bands, [0] * n_occ)
    x = dense_shifted_solve(cell, psi, eps, b, u)
    dn = delta_n(cell, psi, x, bands, [0] * n_occ, 1)
    ref = lindhard_dn_iu(cell, n_occ, qn, u)
    assert np.max(np.abs(dn[0] - ref)) <= 1e-11 * np.max(np.abs(ref))
