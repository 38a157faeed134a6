"""Pins of the dense chi-bar0 reference (oracle/pdep.py), CPU only: for free electrons the sum over
all empty states and the discrete Lindhard closed form give the same eigenvalues; for the tiny
model cell the matrix is symmetric and negative semidefinite and its columns equal the projected
Teter-PCG oracle's."""
import math

import numpy as np

from oracle import OracleCell, apply_chi0
from oracle.pdep import basis_fields, chibar0_dense, free_electron_eigs, potential_reps, vhalf


def test_free_electrons_sum_over_states_equals_lindhard():
    cell = OracleCell(10.0, 10.0, np.zeros((0, 3)))
    M, reps = chibar0_dense(cell, 7, 2.5)
    lam = np.linalg.eigvalsh(0.5 * (M + M.T))
    ref = free_electron_eigs(cell, 7, 2.5)
    assert len(reps) == 40 and M.shape == (80, 80)
    assert np.abs(lam - ref).max() <= 1e-10 * np.abs(ref).max()
    # diagonal in the cos/sin basis: nothing off the diagonal
    off = M - np.diag(np.diag(M))
    assert np.abs(off).max() <= 1e-10 * np.abs(M).max()


def test_model_cell_matrix_symmetric_nsd_and_equal_to_pcg(tiny_system):
    t = tiny_system
    cell = t["cell"]
    M, reps = chibar0_dense(cell, 16, 2.5)
    nrm = np.linalg.norm(M)
    assert np.linalg.norm(M - M.T) <= 1e-12 * nrm
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).max() <= 1e-12 * nrm
    f = basis_fields(cell, reps)
    vh = vhalf(cell, reps)
    cols = [0, 7, 41]
    out = apply_chi0(cell, t["psi"], t["eps"], vh[cols, None, None, None] * f[cols], tol=1e-12)
    Mc = (f.reshape(len(vh), -1) @ out["dn"].reshape(len(cols), -1).T) / cell.N ** 3 * vh[:, None]
    assert np.abs(Mc - M[:, cols]).max() <= 1e-9 * np.abs(M).max()


def test_potential_reps_are_half_of_the_sphere():
    L, e = 10.0, 2.5
    reps = potential_reps(L, e)
    b = 2 * math.pi / L
    assert np.all(np.sum((reps * b) ** 2, axis=1) < e)
    s = {tuple(r) for r in reps.tolist()}
    assert not any(tuple(-r) in s for r in reps)
