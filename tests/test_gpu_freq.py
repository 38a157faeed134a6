"""Response at imaginary frequency i u through the C ABI (stern_opts.omega_imag): conjugate
orthogonal CG on the shifted Sternheimer systems, against the oracle's sum over all empty states
(tiny cell), the static response as u -> 0, the oracle's shifted residual on an uneven cell, and
the PDEP eigenvalues of chi-bar0(i u) against the dense matrix."""
import numpy as np
import pytest

from oracle import OracleCell
from oracle.frequency import shifted_residual, sum_over_states_iu
from oracle.pdep import basis_fields, potential_reps, vhalf
from oracle.sternheimer import rel_l2, rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny_sys(tiny_system):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System
    sp, gs = tiny_system["spec"], tiny_system["gs"]
    s = System(sp.L, sp.ecut, gs["pos"])
    s.set_occupied(gs["psi"], gs["eps"])
    yield s
    s.close()


@pytest.mark.parametrize("u", [0.05, 0.5, 5.0])
def test_dn_matches_sum_over_states(tiny_system, tiny_sys, u):
    t = tiny_system
    dv = t["dv"]
    print(f"case: tiny cell, u = {u}, {dv.shape[0]} fields", flush=True)
    dn, info = tiny_sys.apply_chi0(dv, tol=1e-12, omega_imag=u)
    assert info["n_converged"] == info["n_solves"] == dv.shape[0] * t["spec"].n_occ
    _, _, _, ref = sum_over_states_iu(t["cell"], t["spec"].n_occ, dv, u)
    err = rel_l2(dn, ref).max()
    print(f"  dn rel L2 {err:.2e}, mean iterations {info['total_iters'] / info['n_solves']:.1f}")
    assert err <= 1e-9


def test_small_u_is_the_static_response(tiny_system, tiny_sys):
    dv = tiny_system["dv"][:2]
    d0, _ = tiny_sys.apply_chi0(dv, tol=1e-12)
    du, _ = tiny_sys.apply_chi0(dv, tol=1e-12, omega_imag=1e-7)
    assert rel_l2(du, d0).max() <= 1e-8


def test_rejects_unsupported_requests(tiny_system, tiny_sys):
    from paper_2607_14025_amd import STERN_MIXED
    dv = tiny_system["dv"][:1]
    with pytest.raises(RuntimeError):
        tiny_sys.apply_chi0(dv, omega_imag=0.5, precision=STERN_MIXED)
    with pytest.raises(RuntimeError):
        tiny_sys.apply_chi0(dv, omega_imag=-1.0)


def test_uneven_cell_solutions_satisfy_the_oracle_shifted_system():
    """A batched-config cell (36^3 grid): sampled x against the oracle's FFT operator."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System
    from synth.cells import batched_specs, random_dv
    from synth.inputs import load_ground_state
    sp = sorted(batched_specs(), key=lambda c: c.L)[1]
    gs = load_ground_state(sp)
    s = System(sp.L, sp.ecut, gs["pos"], sp.vloc_amp, sp.vloc_sigma, sp.kb_D, sp.kb_width)
    s.set_occupied(gs["psi"], gs["eps"])
    _, _, dv = random_dv(gs["spec"], n_pert=2, N=gs["N"])
    nb = s.n_occ
    pairs = [(0, 0), (nb // 2, 1), (nb - 1, 0)]
    u = 0.8
    print(f"case: uneven cell {sp.name}, grid {s.fft_n}, {nb} bands, u = {u}", flush=True)
    dn, info = s.apply_chi0(dv, tol=1e-10, omega_imag=u, samples=pairs)
    s.close()
    assert info["n_converged"] == info["n_solves"]
    cell = OracleCell(gs["spec"].L, gs["spec"].ecut, gs["pos"])
    psi = cell.take(gs["psi"], gs["miller"])
    b = rhs(cell, psi, dv, [v for v, _ in pairs], [i for _, i in pairs])
    x = cell.take(info["samples"], gs["miller"])
    res = shifted_residual(cell, psi, gs["eps"][[v for v, _ in pairs]], b, x, u)
    print("  oracle residuals", res)
    assert res.max() <= 1e-9


def test_pdep_eigenvalues_at_imaginary_frequency(tiny_system, tiny_sys):
    """chi-bar0(i u) = v^{1/2} chi0(i u) v^{1/2}: Davidson through the ABI against the dense matrix
    built from the oracle's sum over states at i u."""
    t = tiny_system
    cell, u, ecut_pot = t["cell"], 0.4, 2.5
    reps = potential_reps(cell.L, ecut_pot)
    f = basis_fields(cell, reps)
    vh = vhalf(cell, reps)
    _, _, _, dn = sum_over_states_iu(cell, t["spec"].n_occ, vh[:, None, None, None] * f, u)
    m = len(vh)
    M = (f.reshape(m, -1) @ dn.reshape(m, -1).T) / cell.N ** 3 * vh[:, None]
    ref = np.linalg.eigvalsh(0.5 * (M + M.T))
    n = 6
    eig, vec, info = tiny_sys.pdep_davidson(n, tol=1e-7, block=6, max_basis=36, chi0_tol=1e-11, seed=5, omega_imag=u)
    print("pdep(i u):", eig, "ref", ref[:n])
    assert info["n_converged"] == n
    assert np.abs(eig - ref[:n]).max() <= 1e-8 * np.abs(ref).max()
