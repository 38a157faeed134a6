"""TDDFT Liouville superoperator through the C ABI (stern_liouville_apply, stern_liouville_solve,
stern_liouville_davidson) against the oracle: the grid route on the tiny cell, the transition-basis
matrix of a full diagonalisation on a micro cell, the free-electron closed form, the Z-vector solve
against the oracle's residual and a dense solve, and the Davidson excitation energies against the
dense spectrum, a degenerate free-electron shell and the oracle's operator."""
import math

import numpy as np
import pytest

from oracle import OracleCell
from oracle.liouville import casida_tda, liouville_apply, liouville_residual

pytestmark = pytest.mark.gpu

MICRO_L, MICRO_ECUT, MICRO_OCC = 8.0, 6.0, 4


def _system(*args, **kw):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System
    return System(*args, **kw)


@pytest.fixture(scope="module")
def tiny_sys(tiny_system):
    sp, gs = tiny_system["spec"], tiny_system["gs"]
    s = _system(sp.L, sp.ecut, gs["pos"])
    s.set_occupied(gs["psi"], gs["eps"])
    yield s
    s.close()


@pytest.fixture(scope="module")
def micro():
    pos = np.random.default_rng(7).uniform(0.0, MICRO_L, size=(3, 3))
    cell = OracleCell(MICRO_L, MICRO_ECUT, pos)
    L, occ, eo, emp, ee = casida_tda(cell, MICRO_OCC)
    s = _system(MICRO_L, MICRO_ECUT, pos)
    mil = s.miller()
    s.set_occupied(cell.give(occ, mil), eo)
    yield dict(cell=cell, L=L, occ=occ, eo=eo, emp=emp, sys=s, mil=mil)
    s.close()


def _to_oracle(cell, rows, mil):
    n_e, nb, npw = rows.shape
    return cell.take(rows.reshape(-1, npw), mil).reshape(n_e, nb, npw)


def _to_lib(cell, rows, mil):
    n_e, nb, npw = rows.shape
    return cell.give(rows.reshape(-1, npw), mil).reshape(n_e, nb, npw)


def test_apply_matches_oracle_on_the_tiny_cell(tiny_system, tiny_sys):
    """Random excitations with occupied components (the apply projects them out first)."""
    t = tiny_system
    cell, mil = t["cell"], t["gs"]["miller"]
    nb, npw = tiny_sys.n_occ, tiny_sys.n_pw
    rng = np.random.default_rng(21)
    a = rng.standard_normal((3, nb, npw)) + 1j * rng.standard_normal((3, nb, npw))
    print(f"case: tiny cell, 3 excitations x {nb} bands, grid {tiny_sys.fft_n}", flush=True)
    out = tiny_sys.liouville_apply(a)
    ref = liouville_apply(cell, t["psi"], t["eps"], _to_oracle(cell, a, mil))
    got = _to_oracle(cell, out, mil)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  max rel error {err:.2e}")
    assert err <= 1e-12


def test_apply_matches_the_transition_matrix(micro):
    cell, L, emp, s, mil = micro["cell"], micro["L"], micro["emp"], micro["sys"], micro["mil"]
    n_emp = emp.shape[0]
    cols = np.random.default_rng(3).choice(L.shape[0], size=8, replace=False)
    A = np.zeros((len(cols), MICRO_OCC, cell.npw), dtype=np.complex128)
    for k, t in enumerate(cols):
        v, c = divmod(int(t), n_emp)
        A[k, v] = emp[c]
    print(f"case: micro cell, grid {s.fft_n}, {MICRO_OCC} bands, {n_emp} empty states", flush=True)
    out = _to_oracle(cell, s.liouville_apply(_to_lib(cell, A, mil)), mil)
    for k, t in enumerate(cols):
        col = (out[k] @ emp.conj().T).reshape(-1)
        assert np.abs(col - L[:, t]).max() <= 1e-11 * np.abs(L).max()


def test_free_electron_closed_form():
    """One occupied plane wave G = 0: L A = (|G|^2/2 + 8 pi / (Omega |G|^2)) A for A = e^{i G.r}."""
    cell = OracleCell(MICRO_L, MICRO_ECUT, np.zeros((0, 3)), amp=0.0, D=0.0)
    s = _system(MICRO_L, MICRO_ECUT, np.zeros((0, 3)), vloc_amp=0.0, kb_D=0.0)
    mil = s.miller()
    psi = np.zeros((1, cell.npw), dtype=np.complex128)
    psi[0, 0] = 1.0                                     # oracle index 0 is G = 0
    s.set_occupied(cell.give(psi, mil), np.zeros(1))
    cs = [1, 7, 20, cell.npw - 1]
    A = np.zeros((len(cs), 1, cell.npw), dtype=np.complex128)
    for k, c in enumerate(cs):
        A[k, 0, c] = 1.0
    out = _to_oracle(cell, s.liouville_apply(_to_lib(cell, A, mil)), mil)
    s.close()
    for k, c in enumerate(cs):
        w = 0.5 * cell.g2[c] + 8.0 * math.pi / (cell.omega * cell.g2[c])
        ref = np.zeros(cell.npw, dtype=np.complex128)
        ref[c] = w
        assert np.abs(out[k, 0] - ref).max() <= 1e-12 * w


def test_solve_meets_the_oracle_residual(tiny_system, tiny_sys):
    t = tiny_system
    cell, mil = t["cell"], t["gs"]["miller"]
    nb, npw = tiny_sys.n_occ, tiny_sys.n_pw
    rng = np.random.default_rng(8)
    b = rng.standard_normal((2, nb, npw)) + 1j * rng.standard_normal((2, nb, npw))
    print("case: tiny cell, 2 Z-vector systems", flush=True)
    z, it, res, rc = tiny_sys.liouville_solve(b, tol=1e-11)
    print(f"  iterations {it}, true residuals {res}")
    assert rc == 0 and (res <= 1e-11).all()
    bo = _to_oracle(cell, tiny_sys.apply_pc(b.reshape(-1, npw)).reshape(b.shape), mil)
    ro = liouville_residual(cell, t["psi"], t["eps"], bo, _to_oracle(cell, z, mil))
    print(f"  oracle residuals {ro}")
    assert (ro <= 2e-11).all()


def test_solve_matches_a_dense_solve(micro):
    cell, L, emp, s, mil = micro["cell"], micro["L"], micro["emp"], micro["sys"], micro["mil"]
    n_emp = emp.shape[0]
    rng = np.random.default_rng(13)
    y = rng.standard_normal((2, L.shape[0])) + 1j * rng.standard_normal((2, L.shape[0]))
    b = np.stack([(yy.reshape(MICRO_OCC, n_emp) @ emp) for yy in y])
    zref = np.stack([(np.linalg.solve(L, yy).reshape(MICRO_OCC, n_emp) @ emp) for yy in y])
    z, it, res, rc = s.liouville_solve(_to_lib(cell, b, mil), tol=1e-12)
    print(f"micro cell: iterations {it}, true residuals {res}")
    assert rc == 0
    zo = _to_oracle(cell, z, mil)
    for e in range(2):
        assert np.linalg.norm(zo[e] - zref[e]) <= 1e-10 * np.linalg.norm(zref[e])


def test_rejects_bad_requests(tiny_system):
    sp, gs = tiny_system["spec"], tiny_system["gs"]
    s = _system(sp.L, sp.ecut, gs["pos"])
    with pytest.raises(RuntimeError):  # before set_occupied
        from paper_2607_14025_amd.stern import lib
        import ctypes as C
        a = np.zeros((1, 2, s.n_pw), dtype=np.complex128)
        from paper_2607_14025_amd.stern import _check, STERN_MEM_HOST
        _check(lib().stern_liouville_apply(s._h, 1, C.c_void_p(a.ctypes.data), C.c_void_p(a.ctypes.data),
                                           STERN_MEM_HOST))
    s.set_occupied(gs["psi"], gs["eps"])
    with pytest.raises(ValueError):
        s.liouville_apply(np.zeros((1, s.n_occ + 1, s.n_pw), dtype=np.complex128))
    s.close()


def test_davidson_matches_the_dense_spectrum(micro):
    cell, L, s, mil = micro["cell"], micro["L"], micro["sys"], micro["mil"]
    ref = np.linalg.eigvalsh(L)
    n = 5
    print(f"case: micro cell Davidson, {n} lowest of {L.shape[0]} excitations", flush=True)
    w, vec, info = s.liouville_davidson(n, tol=1e-9, seed=3)
    print("  w", w, "ref", ref[:n], info)
    assert info["rc"] == 0
    assert np.abs(w - ref[:n]).max() <= 1e-10 * ref[n - 1]
    xo = _to_oracle(cell, vec, mil)
    lx = liouville_apply(cell, micro["occ"], micro["eo"], xo)
    for k in range(n):
        assert np.linalg.norm(lx[k] - w[k] * xo[k]) <= 1e-8 * w[k]


def test_davidson_free_electron_degenerate_shell():
    """One occupied plane wave: the six transitions to the first shell |G| = 2 pi / L share
    w = |G|^2 / 2 + 8 pi / (Omega |G|^2), below the next shell's."""
    cell = OracleCell(MICRO_L, MICRO_ECUT, np.zeros((0, 3)), amp=0.0, D=0.0)
    s = _system(MICRO_L, MICRO_ECUT, np.zeros((0, 3)), vloc_amp=0.0, kb_D=0.0)
    psi = np.zeros((1, cell.npw), dtype=np.complex128)
    psi[0, 0] = 1.0
    s.set_occupied(cell.give(psi, s.miller()), np.zeros(1))
    w, _, info = s.liouville_davidson(6, tol=1e-10, seed=1)
    s.close()
    g2 = cell.b ** 2
    ref = 0.5 * g2 + 8.0 * math.pi / (cell.omega * g2)
    print("free-electron shell", w, "closed form", ref, info)
    assert info["rc"] == 0
    assert np.abs(w - ref).max() <= 1e-12 * ref


def test_davidson_pairs_satisfy_the_oracle_operator(tiny_system, tiny_sys):
    t = tiny_system
    cell, mil = t["cell"], t["gs"]["miller"]
    n = 4
    print(f"case: tiny cell Davidson, {n} lowest", flush=True)
    w, vec, info = tiny_sys.liouville_davidson(n, tol=1e-8, block=4, seed=2)
    print("  w", w, info)
    assert info["rc"] == 0
    gap = t["eps"][tiny_sys.n_occ - 1]
    xo = _to_oracle(cell, vec, mil)
    lx = liouville_apply(cell, t["psi"], t["eps"], xo)
    for k in range(n):
        assert np.linalg.norm(lx[k] - w[k] * xo[k]) <= 2e-8 * w[k]
        assert abs(np.linalg.norm(xo[k]) - 1.0) <= 1e-10
    assert np.all(np.diff(w) >= -1e-12) and w[0] > 0


ALPHA = 0.25


def test_exchange_apply_matches_oracle_on_the_tiny_cell(tiny_system):
    t = tiny_system
    sp, gs = t["spec"], t["gs"]
    cell, mil = t["cell"], gs["miller"]
    s = _system(sp.L, sp.ecut, gs["pos"])
    s.set_occupied(gs["psi"], gs["eps"])
    s.liouville_set_kernel(ALPHA)
    nb, npw = s.n_occ, s.n_pw
    rng = np.random.default_rng(22)
    a = rng.standard_normal((2, nb, npw)) + 1j * rng.standard_normal((2, nb, npw))
    print(f"case: tiny cell with alpha_x = {ALPHA}, 2 excitations", flush=True)
    out = _to_oracle(cell, s.liouville_apply(a), mil)
    ref = liouville_apply(cell, t["psi"], t["eps"], _to_oracle(cell, a, mil), ALPHA)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"  max rel error {err:.2e}")
    assert err <= 1e-12
    z, it, res, rc = s.liouville_solve(a, tol=1e-10)
    bo = _to_oracle(cell, s.apply_pc(a.reshape(-1, npw)).reshape(a.shape), mil)
    ro = liouville_residual(cell, t["psi"], t["eps"], bo, _to_oracle(cell, z, mil), ALPHA)
    print(f"  Z-vector iterations {it}, oracle residuals {ro}")
    assert rc == 0 and (ro <= 2e-10).all()
    with pytest.raises(RuntimeError):
        s.liouville_set_kernel(1.5)
    s.close()


def test_exchange_davidson_matches_the_dense_spectrum():
    pos = np.random.default_rng(7).uniform(0.0, MICRO_L, size=(3, 3))
    cell = OracleCell(MICRO_L, MICRO_ECUT, pos)
    L, occ, eo, emp, _ = casida_tda(cell, MICRO_OCC, ALPHA)
    s = _system(MICRO_L, MICRO_ECUT, pos)
    mil = s.miller()
    s.set_occupied(cell.give(occ, mil), eo)
    s.liouville_set_kernel(ALPHA)
    n_emp = emp.shape[0]
    cols = np.random.default_rng(9).choice(L.shape[0], size=6, replace=False)
    A = np.zeros((len(cols), MICRO_OCC, cell.npw), dtype=np.complex128)
    for k, t in enumerate(cols):
        v, c = divmod(int(t), n_emp)
        A[k, v] = emp[c]
    out = _to_oracle(cell, s.liouville_apply(_to_lib(cell, A, mil)), mil)
    for k, t in enumerate(cols):
        assert np.abs((out[k] @ emp.conj().T).reshape(-1) - L[:, t]).max() <= 1e-11 * np.abs(L).max()
    ref = np.linalg.eigvalsh(L)
    w, _, info = s.liouville_davidson(5, tol=1e-9, seed=3)
    s.close()
    print("micro cell with exchange: w", w, "ref", ref[:5], info)
    assert info["rc"] == 0
    assert np.abs(w - ref[:5]).max() <= 1e-10 * ref[4]


def test_lanczos_chain_matches_the_dense_chain(micro):
    """The GPU chain from P_c dV psi_v against the same recurrence on the transition-basis matrix, and
    its continued fraction against the eigen-sum at the bottom of the spectrum."""
    from oracle.liouville import lanczos_chain, spectrum_exact
    from oracle.sternheimer import rhs
    cell, L, occ, emp, s = micro["cell"], micro["L"], micro["occ"], micro["emp"], micro["sys"]
    N = cell.N
    dv = np.random.default_rng(17).standard_normal((N, N, N))
    k = 12
    print(f"case: micro cell Lanczos, {k} steps", flush=True)
    a, b, n2 = s.liouville_lanczos(dv, k)
    bt = rhs(cell, occ, dv[None], list(range(MICRO_OCC)), [0] * MICRO_OCC)
    d = (bt @ emp.conj().T).reshape(-1)
    ao, bo, n2o = lanczos_chain(L, d, k)
    print("  alpha", a[:4], ao[:4], "beta", b[:4], bo[:4])
    assert abs(n2 - n2o) <= 1e-12 * n2o
    assert np.abs(a - ao).max() <= 1e-9 * np.abs(ao).max()
    assert np.abs(b - bo).max() <= 1e-9 * np.abs(bo).max()
    a60, b60, n2 = s.liouville_lanczos(dv, 60)
    om = np.linspace(0.0, 0.25, 101)
    sp = s.lanczos_spectrum(a60, b60, n2, om, 0.02)
    ex = spectrum_exact(L, d, om, 0.02)
    print(f"  spectrum max rel difference {np.abs(sp - ex).max() / np.abs(ex).max():.2e}")
    assert np.abs(sp - ex).max() <= 1e-6 * np.abs(ex).max()


def test_bse_screened_direct_term_matches_the_dense_matrix(micro):
    """BSE's W = v + sum_a w_a c_a w_a^T (w_a, c_a from the oracle's dense chi-bar0 of the micro cell)
    with alpha = 1: apply against the transition-basis matrix, Davidson against its spectrum."""
    from oracle.closed_form import sum_over_states
    from oracle.liouville import screening_from_chibar0
    from oracle.pdep import basis_fields, potential_reps, vhalf
    cell, occ, emp, s, mil = micro["cell"], micro["occ"], micro["emp"], micro["sys"], micro["mil"]
    reps = potential_reps(cell.L, cell.ecut / 4.0)
    f = basis_fields(cell, reps)
    vh = vhalf(cell, reps)
    _, _, _, dn = sum_over_states(cell, MICRO_OCC, vh[:, None, None, None] * f)
    m = len(vh)
    M = (f.reshape(m, -1) @ dn.reshape(m, -1).T) / cell.N ** 3 * vh[:, None]
    w, c = screening_from_chibar0(cell, M, f, vh)
    L, _, _, _, _ = casida_tda(cell, MICRO_OCC, 1.0, (w, c))
    print(f"case: micro cell BSE, {m} screening potentials", flush=True)
    s.liouville_set_kernel(1.0)
    s.liouville_set_screening(w, c)
    try:
        n_emp = emp.shape[0]
        cols = np.random.default_rng(12).choice(L.shape[0], size=6, replace=False)
        A = np.zeros((len(cols), MICRO_OCC, cell.npw), dtype=np.complex128)
        for k, t in enumerate(cols):
            v, cc = divmod(int(t), n_emp)
            A[k, v] = emp[cc]
        out = _to_oracle(cell, s.liouville_apply(_to_lib(cell, A, mil)), mil)
        for k, t in enumerate(cols):
            assert np.abs((out[k] @ emp.conj().T).reshape(-1) - L[:, t]).max() <= 1e-11 * np.abs(L).max()
        ref = np.linalg.eigvalsh(L)
        wv, _, info = s.liouville_davidson(5, tol=1e-9, seed=3)
        print("  w", wv, "ref", ref[:5], info)
        assert info["rc"] == 0
        assert np.abs(wv - ref[:5]).max() <= 1e-10 * ref[4]
    finally:
        s.liouville_set_kernel(0.0)
        s.liouville_set_screening(None)


def test_pdep_eigenpotentials_feed_the_bse_screening(micro):
    """PDEP eigenpairs from the library (stern_pdep_davidson) -> grid potentials (stern_pdep_potentials,
    against the same sum done by numpy) -> BSE screening; the apply equals the oracle's with the same
    potentials and weights."""
    cell, occ, s, mil = micro["cell"], micro["occ"], micro["sys"], micro["mil"]
    n = 6
    eig, vec, info = s.pdep_davidson(n, tol=1e-8, chi0_tol=1e-11, seed=4)
    print("case: micro cell PDEP -> screening; eigenvalues", eig, flush=True)
    assert info["n_converged"] == n
    w = s.pdep_potentials(vec)
    gm = s.pdep_basis()
    idx = cell.index_of(gm)
    vh = np.sqrt(4.0 * np.pi) / (cell.b * np.sqrt(np.sum(gm.astype(np.float64) ** 2, axis=1)))
    coef = np.zeros((n, cell.npw), dtype=np.complex128)
    coef[:, idx] = vh[None, :] * vec
    w_np = cell.to_grid(coef)
    assert np.abs(w_np.imag).max() <= 1e-13 * np.abs(w_np.real).max()
    assert np.abs(w - w_np.real).max() <= 1e-12 * np.abs(w_np.real).max()
    c = eig / (1.0 - eig)
    s.liouville_set_kernel(1.0)
    s.liouville_set_screening(w, c)
    try:
        rng = np.random.default_rng(31)
        a = rng.standard_normal((2, MICRO_OCC, cell.npw)) + 1j * rng.standard_normal((2, MICRO_OCC, cell.npw))
        out = _to_oracle(cell, s.liouville_apply(_to_lib(cell, a, mil)), mil)
        ref = liouville_apply(cell, occ, micro["eo"], a, 1.0, (w_np.real, c))
        err = np.abs(out - ref).max() / np.abs(ref).max()
        print(f"  BSE apply with the PDEP screening: max rel error {err:.2e}")
        assert err <= 1e-12
    finally:
        s.liouville_set_kernel(0.0)
        s.liouville_set_screening(None)
