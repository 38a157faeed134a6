"""Pins of the oracle's Sternheimer solve and density response (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import OracleCell, apply_chi0, band_kinetic, finite_field_dn, lindhard_dn, sum_over_states, teter
from oracle.sternheimer import chi0_matrix, rel_l2


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def tiny_ref(tiny_system):
    t = tiny_system
    occ, eo, xs, dn_sos = sum_over_states(t["cell"], t["spec"].n_occ, t["dv"])
    out = apply_chi0(t["cell"], t["psi"], t["eps"], t["dv"], tol=1e-12)
    return dict(occ=occ, eo=eo, xs=xs, dn_sos=dn_sos, out=out)


def test_teter_limits():
    """K(0) = 1, K ~ 27 / (16 y^4) for large y, strictly between 0 and 1 elsewhere."""
    assert teter(np.array([0.0]))[0] == 1.0
    y = np.array([1e3, 1e4])
    assert np.allclose(teter(y) * 16 * y ** 4 / (8 * y ** 3), 1.0, rtol=1e-2)
    z = np.linspace(1e-3, 50, 1000)
    k = teter(z)
    assert np.all((k > 0) & (k < 1)) and np.all(np.diff(k) < 0)


def test_teter_exact_values():
    """The preconditioner at fractions of y where the published formula was evaluated exactly
    (tests/golden/teter_exact.json): a wrong coefficient in any power of y fails here."""
    pts = json.load(open(os.path.join(GOLDEN, "teter_exact.json")))["points"]
    y = np.array([p["y_num"] / p["y_den"] for p in pts])
    want = np.array([p["K_num"] / p["K_den"] for p in pts])
    assert np.allclose(teter(y), want, rtol=1e-15, atol=0)


def test_band_kinetic_and_its_floor():
    """T_v of single plane waves is |G|^2 / 2 exactly; the G = 0 wave (T = 0) and a band
    below the floor take the kinetic energy of the smallest nonzero G, (2 pi / L)^2 / 2."""
    L = 10.0
    cell = OracleCell(L, 10.0, np.zeros((0, 3)))
    b2h = 0.5 * (2.0 * math.pi / L) ** 2
    mil = [tuple(m) for m in cell.miller.tolist()]
    psi = np.zeros((5, cell.npw), dtype=np.complex128)
    psi[0, mil.index((0, 0, 0))] = 1.0                       # T = 0 -> floor
    psi[1, mil.index((1, 0, 0))] = 1j                        # T = b^2/2 (the floor itself)
    psi[2, mil.index((2, 0, 0))] = -1.0                      # T = 4 b^2/2
    psi[3, mil.index((1, 1, 1))] = np.exp(0.3j)              # T = 3 b^2/2
    psi[4, mil.index((0, 0, 0))] = math.sqrt(0.9)            # T = 0.1 b^2/2, below the floor
    psi[4, mil.index((0, 1, 0))] = math.sqrt(0.1)
    t = band_kinetic(cell, psi)
    assert np.allclose(t, b2h * np.array([1.0, 1.0, 4.0, 3.0, 1.0]), rtol=1e-14, atol=0)


def test_pcg_dn_equals_sum_over_states(tiny_system, tiny_ref):
    out = tiny_ref["out"]
    assert out["resid"].max() <= 1e-12
    assert rel_l2(out["dn"], tiny_ref["dn_sos"]).max() < 1e-11


def test_pcg_x_equals_sum_over_states_per_solve(tiny_system):
    """With the dense eigenvectors as input, every solution vector matches the explicit sum."""
    t = tiny_system
    occ, eo, xs, _ = sum_over_states(t["cell"], t["spec"].n_occ, t["dv"][:2])
    out = apply_chi0(t["cell"], occ, eo, t["dv"][:2], tol=1e-12)
    for k, (v, i) in enumerate(out["pairs"]):
        ref = xs[i, v]
        err = np.linalg.norm(out["x"][k] - ref) / np.linalg.norm(ref)
        assert err < 1e-10, (v, i, err)


def test_dn_equals_finite_field_density_derivative(tiny_system, tiny_ref):
    """Factor 4 (spin x c.c.) and sign: d rho / d lambda of H + lambda dV equals chi0 dV."""
    t = tiny_system
    for i in (0, 3):
        ff = finite_field_dn(t["cell"], t["spec"].n_occ, t["dv"][i])
        dn = tiny_ref["out"]["dn"][i]
        assert np.linalg.norm(ff - dn) / np.linalg.norm(dn) < 1e-9


@pytest.mark.parametrize("n_occ,qn", [(1, (1, 0, 0)), (7, (1, 0, 0)), (7, (1, 1, 0)), (19, (2, 1, 0)), (27, (1, 1, 1))])
def test_free_electron_lindhard(n_occ, qn):
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
    out = apply_chi0(cell, psi, eps, dv, tol=1e-13)
    ref = lindhard_dn(cell, n_occ, qn)
    assert np.max(np.abs(out["dn"][0] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_chi0_hermitian_and_negative_semidefinite(tiny_system, tiny_ref):
    M = chi0_matrix(tiny_system["cell"], tiny_system["dv"], tiny_ref["out"]["dn"])
    nrm = np.linalg.norm(M)
    assert np.linalg.norm(M - M.T) / nrm < 1e-11
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).max() <= 1e-12 * nrm


def test_charge_conserved_and_constant_annihilated(tiny_system, tiny_ref):
    t = tiny_system
    dn = tiny_ref["out"]["dn"]
    assert np.max(np.abs(dn.sum(axis=(1, 2, 3)))) <= 1e-13 * np.abs(dn).sum(axis=(1, 2, 3)).max()
    const = np.full((1,) + t["dv"].shape[1:], 0.7)
    out = apply_chi0(t["cell"], t["psi"], t["eps"], const, tol=1e-12)
    # P_c (c psi_v) = 0: every right-hand side is zero, so x = 0 with no iteration
    assert np.all(out["dn"] == 0.0) and np.all(out["iters"] == 0) and np.all(out["resid"] == 0.0)


def test_rhs_cut_keeps_small_resolvable_fields(tiny_system):
    """b is linear in dV: a constant plus 1e-6 of a field gives 1e-6 of that field's b, so the
    zero cut for b at the projection's rounding level leaves a small but resolvable b alone."""
    from oracle.sternheimer import rhs
    t = tiny_system
    n = t["spec"].n_occ
    bands, perts = list(range(n)), [0] * n
    b = rhs(t["cell"], t["psi"], t["dv"], bands, perts)
    mix = 0.7 + 1e-6 * t["dv"][:1]
    bm = rhs(t["cell"], t["psi"], mix, bands, perts)
    assert np.all(np.linalg.norm(bm, axis=1) > 0)
    assert np.max(np.linalg.norm(bm - 1e-6 * b, axis=1) / np.linalg.norm(1e-6 * b, axis=1)) < 1e-8


def test_linearity_and_phase_gauge(tiny_system, tiny_ref):
    t = tiny_system
    a, b = 0.3, -1.7
    comb = (a * t["dv"][1] + b * t["dv"][2])[None]
    theta = np.linspace(0.1, 2.0, t["psi"].shape[0])
    psi_g = t["psi"] * np.exp(1j * theta)[:, None]
    out = apply_chi0(t["cell"], psi_g, t["eps"], comb, tol=1e-12)
    ref = a * tiny_ref["out"]["dn"][1] + b * tiny_ref["out"]["dn"][2]
    assert np.linalg.norm(out["dn"][0] - ref) / np.linalg.norm(ref) < 1e-10


def test_translation_covariance(tiny_system, tiny_ref):
    """Shifting atoms and fields by a grid vector shifts dn; psi_G -> psi_G exp(-i G.t) stays an eigenvector."""
    t = tiny_system
    cell = t["cell"]
    shift = np.array([3, 0, 5])
    tv = shift * cell.L / cell.N
    cell2 = OracleCell(cell.L, cell.ecut, (t["gs"]["pos"] + tv) % cell.L)
    psi2 = t["psi"] * np.exp(-1j * (cell.gvec @ tv))[None, :]
    res = cell2.h_apply(psi2) - t["eps"][:, None] * psi2
    assert np.max(np.linalg.norm(res, axis=1)) < 1e-12
    dv2 = np.roll(t["dv"][:2], shift=tuple(shift), axis=(1, 2, 3))
    out = apply_chi0(cell2, psi2, t["eps"], dv2, tol=1e-12)
    ref = np.roll(tiny_ref["out"]["dn"][:2], shift=tuple(shift), axis=(1, 2, 3))
    assert rel_l2(out["dn"], ref).max() < 1e-10


def test_axis_permutation_covariance(tiny_system, tiny_ref):
    """Swapping x and y in positions, fields and coefficients swaps the axes of dn."""
    t = tiny_system
    cell = t["cell"]
    cell2 = OracleCell(cell.L, cell.ecut, t["gs"]["pos"][:, [1, 0, 2]])
    m2 = cell.miller[:, [1, 0, 2]]
    psi2 = cell2.take(t["psi"], m2)
    dv2 = np.transpose(t["dv"][:2], (0, 2, 1, 3))
    out = apply_chi0(cell2, psi2, t["eps"], dv2, tol=1e-12)
    ref = np.transpose(tiny_ref["out"]["dn"][:2], (0, 2, 1, 3))
    assert rel_l2(out["dn"], ref).max() < 1e-10


def test_band_subsets_sum_to_full(tiny_system, tiny_ref):
    t = tiny_system
    n = t["psi"].shape[0]
    lo = apply_chi0(t["cell"], t["psi"], t["eps"], t["dv"][:1], tol=1e-12, bands=range(0, n // 2))
    hi = apply_chi0(t["cell"], t["psi"], t["eps"], t["dv"][:1], tol=1e-12, bands=range(n // 2, n))
    ref = tiny_ref["out"]["dn"][:1]
    assert rel_l2(lo["dn"] + hi["dn"], ref).max() < 1e-11
