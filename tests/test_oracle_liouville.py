"""Pins of the oracle's TDDFT Liouville superoperator (Tamm-Dancoff, Hartree kernel), CPU only:
free-electron closed forms written out by hand, the transition-basis matrix from a full
diagonalisation against the grid route, Hermiticity, positivity and the gap bound, and the
residual of a dense Z-vector solve."""
import math

import numpy as np
import pytest

from oracle import OracleCell
from oracle.liouville import casida_tda, free_electron_tda, liouville_apply, liouville_residual

MICRO_L, MICRO_ECUT, MICRO_OCC = 8.0, 6.0, 4


def micro_positions():
    return np.random.default_rng(7).uniform(0.0, MICRO_L, size=(3, 3))


@pytest.fixture(scope="module")
def micro():
    cell = OracleCell(MICRO_L, MICRO_ECUT, micro_positions())
    L, occ, eo, emp, ee = casida_tda(cell, MICRO_OCC)
    return dict(cell=cell, L=L, occ=occ, eo=eo, emp=emp, ee=ee)


def free_cell():
    return OracleCell(MICRO_L, MICRO_ECUT, np.zeros((0, 3)), amp=0.0, D=0.0)


def unit_rows(cell, idx):
    psi = np.zeros((len(idx), cell.npw), dtype=np.complex128)
    psi[np.arange(len(idx)), idx] = 1.0
    return psi


def test_one_plane_wave_closed_form():
    """One occupied state G = 0: every transition to G is its own eigenvector with
    w = |G|^2 / 2 + 8 pi / (Omega |G|^2)."""
    cell = free_cell()
    psi = unit_rows(cell, [0])                       # miller[0] = (0, 0, 0)
    assert np.all(cell.miller[0] == 0)
    cs = [1, 7, 20, cell.npw - 1]
    A = np.zeros((len(cs), 1, cell.npw), dtype=np.complex128)
    for k, c in enumerate(cs):
        A[k, 0, c] = 1.0
    out = liouville_apply(cell, psi, np.zeros(1), A)
    for k, c in enumerate(cs):
        w = 0.5 * cell.g2[c] + 8.0 * math.pi / (cell.omega * cell.g2[c])
        ref = np.zeros(cell.npw, dtype=np.complex128)
        ref[c] = w
        assert np.max(np.abs(out[k, 0] - ref)) <= 1e-12 * w


def test_closed_shell_matches_the_hand_written_matrix():
    """Seven occupied plane waves (G = 0 and its six neighbours), transitions to a set of empty
    plane waves: grid route against the matrix written out from momentum conservation."""
    cell = free_cell()
    order = np.argsort(cell.g2, kind="stable")
    occ_idx = list(order[:7])
    emp_idx = list(order[7:40])
    psi = unit_rows(cell, occ_idx)
    eps = 0.5 * cell.g2[occ_idx]
    ref = free_electron_tda(cell, occ_idx, emp_idx)
    n_t = len(occ_idx) * len(emp_idx)
    A = np.zeros((n_t, len(occ_idx), cell.npw), dtype=np.complex128)
    for t in range(n_t):
        v, c = divmod(t, len(emp_idx))
        A[t, v, emp_idx[c]] = 1.0
    out = liouville_apply(cell, psi, eps, A)
    got = out[:, :, emp_idx].reshape(n_t, n_t).T       # got[b, a] = <B_b | L A_a>
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.count_nonzero(np.abs(ref - np.diag(np.diag(ref))) > 0) > 0  # the kernel couples transitions


def test_model_cell_grid_route_matches_transition_matrix(micro):
    cell, L = micro["cell"], micro["L"]
    occ, emp = micro["occ"], micro["emp"]
    n_emp = emp.shape[0]
    rng = np.random.default_rng(3)
    cols = rng.choice(L.shape[0], size=6, replace=False)
    A = np.zeros((len(cols), MICRO_OCC, cell.npw), dtype=np.complex128)
    for k, t in enumerate(cols):
        v, c = divmod(int(t), n_emp)
        A[k, v] = emp[c]
    out = liouville_apply(cell, occ, micro["eo"], A)
    for k, t in enumerate(cols):
        col = (out[k] @ emp.conj().T).reshape(-1)      # <psi_c'| (L A)_v'> in transition order
        assert np.max(np.abs(col - L[:, t])) <= 1e-11 * np.max(np.abs(L))


def test_hermitian_positive_and_above_the_gap(micro):
    L = micro["L"]
    assert np.max(np.abs(L - L.conj().T)) <= 1e-12 * np.max(np.abs(L))
    w = np.linalg.eigvalsh(L)
    gap = micro["ee"].min() - micro["eo"].max()
    assert gap > 0
    assert w.min() >= gap * (1.0 - 1e-12)                 # K1e is positive semidefinite
    d = np.diag(L).real - (micro["ee"][None, :] - micro["eo"][:, None]).reshape(-1)
    assert d.min() >= -1e-14 and d.max() > 1e-3             # and not zero on this cell


def test_dense_solution_has_zero_residual(micro):
    """Z-vector system L z = b solved in the transition basis, measured by the grid route."""
    cell, L, occ, emp = micro["cell"], micro["L"], micro["occ"], micro["emp"]
    rng = np.random.default_rng(11)
    y = rng.standard_normal(L.shape[0]) + 1j * rng.standard_normal(L.shape[0])
    z_t = np.linalg.solve(L, y)
    n_emp = emp.shape[0]
    b = (y.reshape(MICRO_OCC, n_emp) @ emp)[None]
    z = (z_t.reshape(MICRO_OCC, n_emp) @ emp)[None]
    assert liouville_residual(cell, occ, micro["eo"], b, z)[0] <= 1e-11


def test_occupied_components_of_the_input_are_removed(micro):
    """L acts on P_c A: adding occupied components to A changes nothing."""
    cell, occ, emp = micro["cell"], micro["occ"], micro["emp"]
    rng = np.random.default_rng(5)
    A = (rng.standard_normal((2, MICRO_OCC, emp.shape[0])) @ emp).astype(np.complex128)
    extra = rng.standard_normal((2, MICRO_OCC, MICRO_OCC)) @ occ
    a = liouville_apply(cell, occ, micro["eo"], A)
    b = liouville_apply(cell, occ, micro["eo"], A + extra)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


ALPHA = 0.25


def test_closed_shell_with_exchange_matches_the_hand_written_matrix():
    """The direct term of bare exchange: grid route against momentum conservation written out."""
    cell = free_cell()
    order = np.argsort(cell.g2, kind="stable")
    occ_idx = list(order[:7])
    emp_idx = list(order[7:40])
    psi = unit_rows(cell, occ_idx)
    eps = 0.5 * cell.g2[occ_idx]
    ref = free_electron_tda(cell, occ_idx, emp_idx, ALPHA)
    assert np.abs(ref - free_electron_tda(cell, occ_idx, emp_idx)).max() > 1e-3   # the term is there
    n_t = len(occ_idx) * len(emp_idx)
    A = np.zeros((n_t, len(occ_idx), cell.npw), dtype=np.complex128)
    for t in range(n_t):
        v, c = divmod(t, len(emp_idx))
        A[t, v, emp_idx[c]] = 1.0
    out = liouville_apply(cell, psi, eps, A, ALPHA)
    got = out[:, :, emp_idx].reshape(n_t, n_t).T
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_model_cell_with_exchange_grid_route_matches_transition_matrix(micro):
    cell, occ, emp = micro["cell"], micro["occ"], micro["emp"]
    L, _, _, _, _ = casida_tda(cell, MICRO_OCC, ALPHA)
    assert np.max(np.abs(L - L.conj().T)) <= 1e-12 * np.max(np.abs(L))
    assert np.abs(L - micro["L"]).max() > 1e-4
    n_emp = emp.shape[0]
    cols = np.random.default_rng(4).choice(L.shape[0], size=6, replace=False)
    A = np.zeros((len(cols), MICRO_OCC, cell.npw), dtype=np.complex128)
    for k, t in enumerate(cols):
        v, c = divmod(int(t), n_emp)
        A[k, v] = emp[c]
    out = liouville_apply(cell, occ, micro["eo"], A, ALPHA)
    for k, t in enumerate(cols):
        col = (out[k] @ emp.conj().T).reshape(-1)
        assert np.max(np.abs(col - L[:, t])) <= 1e-11 * np.max(np.abs(L))


def test_lanczos_chain_reproduces_moments_and_the_low_energy_spectrum(micro):
    """k steps of the chain reproduce the moments <d|L^j|d>, j < 2k, exactly (those of its tridiagonal
    matrix); its continued fraction equals the eigen-sum where the chain has converged (the bottom of
    the spectrum), and the eigen-sum integrates to ||d||^2."""
    from oracle.liouville import lanczos_chain, spectrum_exact, spectrum_from_chain
    L = micro["L"]
    d = np.random.default_rng(2).standard_normal(L.shape[0]).astype(np.complex128)
    k = 8
    a, b, n2 = lanczos_chain(L, d, k)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    v, e1 = d.copy(), np.eye(k)[0]
    t = e1.copy()
    for j in range(2 * k):
        mom = np.vdot(d, v).real
        assert abs(n2 * t[0] - mom) <= 1e-9 * abs(mom), j
        v = L @ v
        t = T @ t
    a, b, n2 = lanczos_chain(L, d, 60)
    om = np.linspace(0.0, 0.25, 101)
    eta = 0.02
    s_ch = spectrum_from_chain(a, b, n2, om, eta)
    s_ex = spectrum_exact(L, d, om, eta)
    assert np.abs(s_ch - s_ex).max() <= 1e-8 * np.abs(s_ex).max()
    wide = np.linspace(-200.0, 200.0, 400001)
    total = np.trapezoid(spectrum_exact(L, d, wide, 0.5), wide)
    assert abs(total - n2) <= 5e-3 * n2


@pytest.fixture(scope="module")
def screening(micro):
    """W - v from the dense chi-bar0 of the micro cell (potentials |G|^2 < Ecut / 4)."""
    from oracle.closed_form import sum_over_states
    from oracle.liouville import screening_from_chibar0
    from oracle.pdep import basis_fields, potential_reps, vhalf
    cell = micro["cell"]
    reps = potential_reps(cell.L, cell.ecut / 4.0)
    f = basis_fields(cell, reps)
    vh = vhalf(cell, reps)
    _, _, _, dn = sum_over_states(cell, MICRO_OCC, vh[:, None, None, None] * f)
    m = len(vh)
    M = (f.reshape(m, -1) @ dn.reshape(m, -1).T) / cell.N ** 3 * vh[:, None]
    w, c = screening_from_chibar0(cell, M, f, vh)
    return dict(M=M, f=f, vh=vh, w=w, c=c)


def test_screening_equals_the_inverse_dielectric_matrix(micro, screening):
    """sum_a w_a c_a <w_a, .> from the eigenpairs = v^{1/2} ((1 - M)^{-1} - 1) v^{1/2} by a dense solve,
    on the real basis functions (no eigen-decomposition on this side)."""
    cell = micro["cell"]
    M, f, vh, w, c = (screening[k] for k in ("M", "f", "vh", "w", "c"))
    m = len(vh)
    N3 = cell.N ** 3
    proj = np.einsum("axyz,jxyz->ja", w, f) / N3
    got = np.einsum("ja,a,ka->jk", proj, c, proj)                       # <f_j, dW f_k>_N
    Ms = 0.5 * (M + M.T)
    ref = vh[:, None] * (np.linalg.solve(np.eye(m) - Ms, np.eye(m)) - np.eye(m)) * vh[None, :]
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(c <= 0.0) and np.all(c > -1.0)                        # screening lowers W


def test_screened_grid_route_matches_transition_matrix(micro, screening):
    """BSE's W (alpha = 1 plus the screening): grid route against the transition-basis matrix."""
    from oracle.liouville import screened_grid
    cell, occ, emp = micro["cell"], micro["occ"], micro["emp"]
    scr = (screening["w"], screening["c"])
    L, _, _, _, _ = casida_tda(cell, MICRO_OCC, 1.0, scr)
    L1, _, _, _, _ = casida_tda(cell, MICRO_OCC, 1.0)
    assert np.max(np.abs(L - L.conj().T)) <= 1e-12 * np.max(np.abs(L))
    assert np.abs(L - L1).max() > 1e-4                                   # the screening changes L
    n_emp = emp.shape[0]
    cols = np.random.default_rng(6).choice(L.shape[0], size=6, replace=False)
    A = np.zeros((len(cols), MICRO_OCC, cell.npw), dtype=np.complex128)
    for k, t in enumerate(cols):
        v, c = divmod(int(t), n_emp)
        A[k, v] = emp[c]
    out = liouville_apply(cell, occ, micro["eo"], A, 1.0, scr)
    for k, t in enumerate(cols):
        col = (out[k] @ emp.conj().T).reshape(-1)
        assert np.max(np.abs(col - L[:, t])) <= 1e-11 * np.max(np.abs(L))
    # no screening weight: the bare-exchange route
    rho = np.random.default_rng(1).standard_normal((2, cell.N, cell.N, cell.N)).astype(np.complex128)
    zero = (screening["w"], np.zeros_like(screening["c"]))
    assert np.abs(screened_grid(cell, rho, 0.3, zero) - screened_grid(cell, rho, 0.3, None)).max() <= 1e-15
