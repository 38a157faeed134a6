"""Pins of the oracle's deflated Sternheimer solve (CPU only): with exact lowest empty states the
deflated solution equals the plain projected PCG's and the dense solve, with no empty states it is
the plain solve, and the slowest (near-gap) solves take fewer iterations."""
import numpy as np
import pytest

from oracle import band_kinetic, pcg_solve, rhs
from oracle.deflation import deflated_solve


@pytest.fixture(scope="module")
def states(tiny_system):
    t = tiny_system
    cell = t["cell"]
    e, U = np.linalg.eigh(cell.h_dense())
    n = t["spec"].n_occ
    psi = U.T[:n]
    return dict(cell=cell, psi=psi, eps=e[:n], emp=U.T[n:], eemp=e[n:], n=n, dv=t["dv"])


def test_deflated_solution_equals_the_plain_one(states):
    cell, psi, n = states["cell"], states["psi"], states["n"]
    bands = [n - 1, n - 2, 0, 7]
    b = rhs(cell, psi, states["dv"], bands, [0, 1, 2, 0])
    tk = band_kinetic(cell, psi)[bands]
    eps = states["eps"][bands]
    x0, it0, _ = pcg_solve(cell, psi, eps, tk, b, 1e-12)
    # dense reference: x = sum over all empty states
    coef = (b @ states["emp"].conj().T) / (states["eemp"][None, :] - eps[:, None])
    xd = coef @ states["emp"]
    for nE in (0, 8, 32):
        x, it, res = deflated_solve(cell, psi, eps, tk, b, states["emp"][:nE], states["eemp"][:nE], 1e-12)
        for k in range(len(bands)):
            assert np.linalg.norm(x[k] - xd[k]) <= 1e-10 * np.linalg.norm(xd[k])
        if nE == 0:
            assert np.array_equal(it, it0)
        print(f"empty states taken out {nE}: iterations {it.tolist()} (plain {it0.tolist()})")
    _, it8, _ = deflated_solve(cell, psi, eps, tk, b, states["emp"][:8], states["eemp"][:8], 1e-12)
    assert it8[0] < it0[0] and it8[1] < it0[1]   # the two bands next to the gap
