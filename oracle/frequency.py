"""Density response at imaginary frequency (TEST INFRASTRUCTURE ONLY).

Sec. II.A evaluates the self-energy at several frequencies (Lanczos chains,
full-frequency G0W0), which needs the density response beyond zero frequency;
the same Sternheimer machinery then solves shifted systems. At imaginary
frequency i u the Lehmann form of chi0 couples each occupied band v to every
empty state c through 1/(eps_v - eps_c + i u) and 1/(eps_v - eps_c - i u). For a
real field dV the two terms are complex conjugates of each other, so

    dn_i(r; i u) = 4 Re sum_v conj(psi_v(r)) x_{v,i}(r),
    (P_c (H - eps_v) P_c - i u) x_{v,i} = -P_c dV_i psi_v      on range(P_c),

the static Sternheimer equation with the complex shift -i u (u = 0 gives it
back). Three plain routes, pinned against each other and against closed forms:

* sum_over_states_iu: x_v = sum_c psi_c <psi_c|dV|psi_v> / (eps_v - eps_c + i u)
  over all empty states of a full diagonalisation;
* dense_shifted_solve: the dense system (P_c (H - eps_v - i u) P_c + P_v) x = b,
  which equals the projected one on range(P_c) and is nonsingular;
* lindhard_dn_iu: free electrons with closed shells and dV = 2 cos(q.r), where
  dn(r) = -(4/Omega) cos(q.r) sum_{s=+-} sum_{k occ} [k + s q empty, in the sphere]
          (e_t - e_k) / ((e_t - e_k)^2 + u^2),  t = k + s q.
shifted_residual measures a given solution under the oracle's own operator
(FFT-based H apply), for cells too large for the dense routes.
"""
from __future__ import annotations

import numpy as np

from .model import OracleCell
from .sternheimer import project


def sum_over_states_iu(cell: OracleCell, n_occ: int, dv_r: np.ndarray, u: float):
    """Dense route at imaginary frequency i u: returns (psi_occ, eps_occ, x [n_pert, n_occ, npw], dn)."""
    e, U = np.linalg.eigh(cell.h_dense())
    psi = U.T
    occ, emp = psi[:n_occ], psi[n_occ:]
    eo, ee = e[:n_occ], e[n_occ:]
    n_pert = dv_r.shape[0]
    xs = np.zeros((n_pert, n_occ, cell.npw), dtype=np.complex128)
    N = cell.N
    dn = np.zeros((n_pert, N, N, N))
    occ_r = cell.to_grid(occ)
    for i in range(n_pert):
        m = emp.conj() @ cell.potential_dense(dv_r[i]) @ occ.T   # <psi_c|dV|psi_v>  [n_emp, n_occ]
        coef = m / (eo[None, :] - ee[:, None] + 1j * u)
        xs[i] = (emp.T @ coef).T
        xr = cell.to_grid(xs[i])
        dn[i] = (4.0 / cell.omega) * np.sum(np.real(np.conj(occ_r) * xr), axis=0)
    return occ, eo, xs, dn


def dense_shifted_solve(cell: OracleCell, psi: np.ndarray, eps_s: np.ndarray, b: np.ndarray, u: float) -> np.ndarray:
    """x [S, npw] with (P_c (H - eps_s - i u) P_c + P_v) x = b row by row (b in range(P_c))."""
    H = cell.h_dense()
    Pv = psi.T @ psi.conj()           # sum_v |psi_v><psi_v| as a matrix acting on coefficient columns
    Pc = np.eye(cell.npw) - Pv
    out = np.empty_like(b)
    for k in range(b.shape[0]):
        M = Pc @ (H - (eps_s[k] + 1j * u) * np.eye(cell.npw)) @ Pc + Pv
        out[k] = np.linalg.solve(M, b[k])
    return out


def shifted_residual(cell: OracleCell, psi: np.ndarray, eps_s: np.ndarray, b: np.ndarray, x: np.ndarray,
                     u: float) -> np.ndarray:
    """||b - (P_c (H - eps_s) P_c - i u P_c) x|| / ||b|| per row, with the FFT-based H apply."""
    xp = project(psi, x)
    ax = project(psi, cell.h_apply(xp) - eps_s[:, None] * xp) - 1j * u * xp
    return np.linalg.norm(b - ax, axis=1) / np.linalg.norm(b, axis=1)


def lindhard_dn_iu(cell: OracleCell, n_occ: int, qn, u: float) -> np.ndarray:
    """Closed-form dn(i u) on the grid for free electrons and dV = 2 cos(q.r), q = (2 pi/L) qn.

    The occupied set is the n_occ lowest plane waves and must close a shell (then it is
    symmetric under k -> -k and the sin(q.r) parts of the two couplings cancel)."""
    g2 = cell.g2
    order = np.argsort(g2, kind="stable")
    if n_occ < cell.npw and np.isclose(g2[order[n_occ - 1]], g2[order[n_occ]]):
        raise ValueError("n_occ does not close a shell")
    occ = {tuple(cell.miller[k]) for k in order[:n_occ]}
    inside = {tuple(m) for m in cell.miller.tolist()}
    qn = np.asarray(qn)
    total = 0.0
    for k in occ:
        kk = np.array(k)
        for s in (1, -1):
            t = tuple(kk + s * qn)
            if t in inside and t not in occ:
                d = 0.5 * cell.b ** 2 * (float(np.dot(t, t)) - float(kk @ kk))
                total += d / (d * d + u * u)
    N = cell.N
    j = np.arange(N) * (cell.L / N)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    qv = qn * cell.b
    return -(4.0 / cell.omega) * np.cos(qv[0] * X + qv[1] * Y + qv[2] * Z) * total
