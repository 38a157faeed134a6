"""Dense symmetrised density response for the PDEP eigenproblem (TEST INFRASTRUCTURE ONLY).

Sec. II.A (eq. pdep) diagonalises the symmetrised irreducible response
chi-bar0 = v^{1/2} chi0 v^{1/2}, v^{1/2}(G) = sqrt(4 pi) / |G|, iteratively and
keeps its lowest eigenpairs (lambda_a, phi-bar_a). Here the plain definition:
the matrix of chi-bar0 in an orthonormal real basis of the band-limited
potentials, then all its eigenvalues by numpy.

Basis: for each half-space representative G (n_x > 0; or n_x = 0, n_y > 0; or
n_x = n_y = 0, n_z > 0) with |G|^2 < ecut_pot, G != 0 (the long-range G = 0 part
belongs to the separate term of eq. pdep), in the canonical order (|n|^2, then
n), the two functions f = sqrt(2) cos(G.r) and sqrt(2) sin(G.r). Their plane-wave
coefficients are (1, 1) / sqrt(2) and (-i, i) / sqrt(2) at (G, -G), so the basis is
orthonormal for sum_G conj(c_G) c'_G = (1 / N^3) sum_r f(r) f'(r), and

    M_ij = v^{1/2}(G_i) v^{1/2}(G_j) (1 / N^3) sum_r f_i(r) chi0[f_j](r).

chi0 comes from the explicit sum over all empty states (closed_form.sum_over_states),
so nothing iterative enters the matrix. For free electrons (no wells, no
projectors, a closed shell of plane waves) chi0 is diagonal in G and the
eigenvalues follow from the discrete Lindhard sum of closed_form.lindhard_dn.
"""
from __future__ import annotations

import math

import numpy as np

from .closed_form import sum_over_states, lindhard_dn
from .model import OracleCell, sphere_miller


def potential_reps(L: float, ecut_pot: float) -> np.ndarray:
    """Half-space representatives n (G = 2 pi n / L, G != 0, |G|^2 < ecut_pot), canonical order."""
    r2 = ecut_pot * L * L / (4.0 * math.pi ** 2)
    m = sphere_miller(L, ecut_pot)
    n2 = np.sum(m ** 2, axis=1)
    keep = (n2 < r2) & ((m[:, 0] > 0) | ((m[:, 0] == 0) & (m[:, 1] > 0)) |
                        ((m[:, 0] == 0) & (m[:, 1] == 0) & (m[:, 2] > 0)))
    return m[keep]


def basis_fields(cell: OracleCell, reps: np.ndarray) -> np.ndarray:
    """The real basis functions on the grid, [2 m, N, N, N] (cos then sin of each representative)."""
    N = cell.N
    j = np.arange(N) * (cell.L / N)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    out = np.empty((2 * len(reps), N, N, N))
    for k, n in enumerate(reps):
        ph = cell.b * (n[0] * X + n[1] * Y + n[2] * Z)
        out[2 * k] = math.sqrt(2.0) * np.cos(ph)
        out[2 * k + 1] = math.sqrt(2.0) * np.sin(ph)
    return out


def vhalf(cell: OracleCell, reps: np.ndarray) -> np.ndarray:
    """v^{1/2}(G) of each basis function, [2 m]."""
    g = np.sqrt(np.sum((reps * cell.b) ** 2, axis=1))
    return np.repeat(math.sqrt(4.0 * math.pi) / g, 2)


def chibar0_dense(cell: OracleCell, n_occ: int, ecut_pot: float):
    """(M [2m, 2m], reps): chi-bar0 in the real basis, chi0 from the sum over all empty states."""
    reps = potential_reps(cell.L, ecut_pot)
    f = basis_fields(cell, reps)
    vh = vhalf(cell, reps)
    _, _, _, dn = sum_over_states(cell, n_occ, vh[:, None, None, None] * f)
    n = len(vh)
    M = (f.reshape(n, -1) @ dn.reshape(n, -1).T) / cell.N ** 3 * vh[:, None]
    return M, reps


def free_electron_eigs(cell: OracleCell, n_occ: int, ecut_pot: float) -> np.ndarray:
    """Eigenvalues of chi-bar0 for free electrons, ascending: for each representative q,
    chi0 maps 2 cos(q.r) to -(4 / Omega) S(q) cos(q.r) (the Lindhard sum S of
    closed_form.lindhard_dn) and sin alike, so lambda(q) = (4 pi / |q|^2) (-2 S(q) / Omega),
    twice (cos and sin)."""
    reps = potential_reps(cell.L, ecut_pot)
    out = []
    for n in reps:
        dn = lindhard_dn(cell, n_occ, n)
        # dn = -(4 / Omega) S cos(q.r): read -(4/Omega) S off the grid value at r = 0
        amp = dn[0, 0, 0]
        q2 = float(np.sum((n * cell.b) ** 2))
        lam = (4.0 * math.pi / q2) * amp / 2.0
        out += [lam, lam]
    return np.sort(np.array(out))


def coords_from_coefficients(phi: np.ndarray, miller: np.ndarray, reps: np.ndarray) -> np.ndarray:
    """Real basis coordinates (a, b) of potentials given as complex coefficients phi [n, n_g] over the
    Miller list `miller` (both G and -G): c_G = (a - i b) / sqrt(2)."""
    key = {tuple(m): k for k, m in enumerate(np.asarray(miller).tolist())}
    idx = np.array([key[tuple(n)] for n in reps.tolist()])
    c = np.atleast_2d(phi)[:, idx]
    out = np.empty((c.shape[0], 2 * len(reps)))
    out[:, 0::2] = math.sqrt(2.0) * c.real
    out[:, 1::2] = -math.sqrt(2.0) * c.imag
    return out
