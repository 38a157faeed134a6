"""Closed forms that pin the oracle's Sternheimer path (TEST INFRASTRUCTURE ONLY).

* sum_over_states: the explicit sum over all empty states from full
  diagonalisation, x_v = -sum_{c > N_occ} psi_c <psi_c|dV|psi_v> / (eps_c - eps_v),
  i.e. the Adler-Wiser-type expression that Sec. II.A contrasts with the
  Sternheimer route (N_occ x N_empty x N_pw^2 cost).
* finite_field_dn: the central difference of rho(lambda) = 2 sum_v |psi_v(lambda)|^2
  (eq. rho with two electrons per band) for H + lambda dV, with one Richardson step.
* lindhard_dn: free electrons (V = 0, D = 0) with complete shells and
  dV = 2 cos(q.r); dn(r) = -(4/Omega) cos(q.r) sum_{s=+-} sum_{k occ}
  [k + s q empty and inside the sphere] / (|k + s q|^2/2 - |k|^2/2).
"""
from __future__ import annotations

import numpy as np

from .model import OracleCell


def sum_over_states(cell: OracleCell, n_occ: int, dv_r: np.ndarray):
    """Dense route: returns (psi_occ [n_occ, npw], eps [n_occ], x [n_pert, n_occ, npw], dn)."""
    e, U = np.linalg.eigh(cell.h_dense())
    psi = U.T  # rows
    occ, emp = psi[:n_occ], psi[n_occ:]
    eo, ee = e[:n_occ], e[n_occ:]
    n_pert = dv_r.shape[0]
    xs = np.zeros((n_pert, n_occ, cell.npw), dtype=np.complex128)
    N = cell.N
    dn = np.zeros((n_pert, N, N, N))
    occ_r = cell.to_grid(occ)
    for i in range(n_pert):
        Vm = cell.potential_dense(dv_r[i])
        m = emp.conj() @ Vm @ occ.T          # <psi_c|dV|psi_v>  [n_emp, n_occ]
        coef = -m / (ee[:, None] - eo[None, :])
        xs[i] = (emp.T @ coef).T
        xr = cell.to_grid(xs[i])
        dn[i] = (4.0 / cell.omega) * np.sum(np.real(np.conj(occ_r) * xr), axis=0)
    return occ, eo, xs, dn


def density(cell: OracleCell, psi: np.ndarray) -> np.ndarray:
    """rho(r) = (2 / Omega) sum_v |psi~_v(r)|^2 (two electrons per band)."""
    return (2.0 / cell.omega) * np.sum(np.abs(cell.to_grid(psi)) ** 2, axis=0)


def finite_field_dn(cell: OracleCell, n_occ: int, dv_r: np.ndarray, lam: float = 1e-4) -> np.ndarray:
    """d rho / d lambda at 0 for H + lambda dV, by central differences + Richardson."""
    H0 = cell.h_dense()
    Vm = cell.potential_dense(dv_r)

    def rho(l):
        e, U = np.linalg.eigh(H0 + l * Vm)
        return density(cell, U[:, :n_occ].T)

    def d(l):
        return (rho(l) - rho(-l)) / (2.0 * l)

    return (4.0 * d(lam / 2.0) - d(lam)) / 3.0


def lindhard_dn(cell: OracleCell, n_occ: int, qn) -> np.ndarray:
    """Closed-form dn on the grid for free electrons and dV = 2 cos(q.r), q = (2 pi/L) qn.

    The occupied set is the n_occ lowest plane waves, which must close a shell."""
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
                ek = 0.5 * cell.b ** 2 * float(kk @ kk)
                et = 0.5 * cell.b ** 2 * float(np.dot(t, t))
                total += 1.0 / (et - ek)
    N = cell.N
    j = np.arange(N) * (cell.L / N)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    qv = qn * cell.b
    cosq = np.cos(qv[0] * X + qv[1] * Y + qv[2] * Z)
    return -(4.0 / cell.omega) * cosq * total
