"""Pins of the oracle's basis, model and input generator against independent facts."""
import json
import math
import os

import numpy as np
import pytest

from oracle import OracleCell, fft_grid, sphere_miller, project
from synth.cells import TINY, batched_specs, fft_size, miller_sorted, place_atoms, random_dv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "workload_sizes.json")


def _brute_count(L, ecut):
    """Lattice points with |n|^2 <= ecut L^2 / 4pi^2, counted column by column."""
    r2 = ecut * L * L / (4.0 * math.pi ** 2)
    nm = int(math.isqrt(int(r2)))
    total = 0
    for a in range(-nm, nm + 1):
        for b in range(-nm, nm + 1):
            rest = r2 - a * a - b * b
            if rest < 0:
                continue
            c = math.isqrt(int(math.floor(rest)))
            total += 2 * c + 1
    return total


def test_sphere_counts_and_grids_match_workloads():
    g = json.load(open(GOLDEN))
    for c in g["cells"]:
        assert fft_grid(c["L"], c["ecut"]) == c["grid"]
        assert fft_size(c["L"], c["ecut"]) == c["grid"]
        n = _brute_count(c["L"], c["ecut"])
        assert n == c["npw"]
        if c["npw"] < 40000:
            assert len(sphere_miller(c["L"], c["ecut"])) == n
            assert len(miller_sorted(c["L"], c["ecut"])) == n


def test_batched_grids_in_range():
    lo, hi = json.load(open(GOLDEN))["batched_grid_range"]
    for sp in batched_specs():
        n = fft_grid(sp.L, sp.ecut)
        assert lo <= n <= hi
        assert n == fft_size(sp.L, sp.ecut)


def test_no_lattice_point_on_sphere_surface():
    for L, e in [(10, 10), (20, 25), (24, 30), (32, 30)]:
        r2 = e * L * L / (4 * math.pi ** 2)
        assert abs(r2 - round(r2)) > 1e-6


def test_grid_alias_free():
    """N exceeds 4 R + 1: G - G' - q never wraps for wave-function G, G' and |q|^2 <= 4 Ecut."""
    for L, e in [(10, 10), (20, 25), (24, 30), (32, 30), (13.7, 20)]:
        R = math.sqrt(e) * L / (2 * math.pi)
        assert fft_grid(L, e) > 4 * R + 1


def test_vloc_grid_equals_real_space_gaussian_sum():
    """V(r_j) from the truncated Fourier series equals the periodic Gaussian sum in real space."""
    pos = place_atoms(TINY)
    cell = OracleCell(TINY.L, TINY.ecut, pos)
    L, N = cell.L, cell.N
    rng = np.random.default_rng(5)
    pts = rng.integers(0, N, size=(40, 3))
    for j in pts:
        r = j * L / N
        val = 0.0
        for R in pos:
            d = r - R
            for m in np.array(np.meshgrid([-2, -1, 0, 1, 2], [-2, -1, 0, 1, 2], [-2, -1, 0, 1, 2])).reshape(3, -1).T:
                dd = d + L * m
                val += cell.amp * math.exp(-float(dd @ dd) / (2 * cell.sigma ** 2))
        assert abs(cell.v_r[tuple(j)] - val) < 1e-7


def test_kb_projector_is_unit_gaussian_at_atom():
    """At a cutoff where the Gaussian is fully resolved, beta_a(r) = (2 pi)^-3/2 exp(-|r-R_a|^2/2)."""
    pos = np.array([[2.5, 7.0, 4.0]])
    cell = OracleCell(10.0, 80.0, pos)
    f = cell.to_grid(cell.beta)[0] / math.sqrt(cell.omega)   # Omega^-1/2 sum beta(G) e^{iGr}
    assert np.max(np.abs(f.imag)) < 1e-12
    L, N = cell.L, cell.N
    j = np.arange(N) * L / N
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    ref = np.zeros_like(X)
    for mx in (-1, 0, 1):
        for my in (-1, 0, 1):
            for mz in (-1, 0, 1):
                d2 = (X - pos[0, 0] - L * mx) ** 2 + (Y - pos[0, 1] - L * my) ** 2 + (Z - pos[0, 2] - L * mz) ** 2
                ref += np.exp(-d2 / 2)
    ref *= (2 * math.pi) ** -1.5
    assert np.max(np.abs(f.real - ref)) < 1e-10


def test_h_apply_equals_dense(tiny_system):
    cell = tiny_system["cell"]
    H = cell.h_dense()
    assert np.max(np.abs(H - H.conj().T)) < 1e-14
    rng = np.random.default_rng(1)
    c = rng.standard_normal((5, cell.npw)) + 1j * rng.standard_normal((5, cell.npw))
    assert np.max(np.abs(cell.h_apply(c) - (H @ c.T).T)) < 1e-12 * np.max(np.abs(c))


def test_ground_state_is_eigenbasis_of_oracle_h(tiny_system):
    cell, psi, eps = tiny_system["cell"], tiny_system["psi"], tiny_system["eps"]
    res = cell.h_apply(psi) - eps[:, None] * psi
    assert np.max(np.linalg.norm(res, axis=1)) < 1e-12
    assert np.max(np.abs(psi @ psi.conj().T - np.eye(psi.shape[0]))) < 1e-13
    e_all = np.linalg.eigvalsh(cell.h_dense())
    assert np.max(np.abs(e_all[: psi.shape[0]] - eps)) < 1e-12
    assert tiny_system["gs"]["gap"] > 1e-4


def test_projector_idempotent(tiny_system):
    cell, psi = tiny_system["cell"], tiny_system["psi"]
    rng = np.random.default_rng(2)
    y = rng.standard_normal((4, cell.npw)) + 1j * rng.standard_normal((4, cell.npw))
    py = project(psi, y)
    assert np.max(np.linalg.norm(project(psi, py) - py, axis=1) / np.linalg.norm(y, axis=1)) < 1e-13
    assert np.max(np.abs(py @ psi.conj().T)) < 1e-13


def test_perturbations_real_band_limited_unit(tiny_system):
    cell, dv = tiny_system["cell"], tiny_system["dv"]
    N = cell.N
    F = np.fft.fftn(dv, axes=(1, 2, 3)) / N ** 3
    n = np.fft.fftfreq(N, 1.0 / N).astype(int)
    NX, NY, NZ = np.meshgrid(n, n, n, indexing="ij")
    g2 = (NX ** 2 + NY ** 2 + NZ ** 2) * (2 * math.pi / cell.L) ** 2
    outside = g2 >= cell.ecut / 4
    assert np.max(np.abs(F[:, outside])) < 1e-15
    assert np.allclose(np.sum(np.abs(F) ** 2, axis=(1, 2, 3)), 1.0, atol=1e-13)
    # a real field has Hermitian-symmetric coefficients
    Fm = F[:, (-np.arange(N)) % N][:, :, (-np.arange(N)) % N][:, :, :, (-np.arange(N)) % N]
    assert np.max(np.abs(F - Fm.conj())) < 1e-15


def test_atoms_respect_minimum_separation():
    for sp in [TINY] + batched_specs()[:4]:
        pos = place_atoms(sp)
        d = pos[:, None, :] - pos[None, :, :]
        d -= sp.L * np.round(d / sp.L)
        r = np.sqrt(np.sum(d ** 2, axis=-1)) + np.eye(len(pos)) * 1e9
        assert r.min() >= sp.min_sep
        assert np.all((pos >= 0) & (pos < sp.L))


def test_inputs_are_seeded():
    a = random_dv(TINY, n_pert=2)[2]
    b = random_dv(TINY, n_pert=2)[2]
    assert np.array_equal(a, b)
    assert np.array_equal(place_atoms(TINY), place_atoms(TINY))
