"""Deflated Sternheimer solve (TEST INFRASTRUCTURE ONLY).

The slowest solves of the static response are those of the bands next to the gap: the smallest
eigenvalue of P_c (H - eps_v) P_c on range(P_c) is eps_LUMO - eps_v. When the lowest empty states
psi_c, c in E, are known as eigenvectors of H (a ground-state code commonly returns a few above the
occupied ones), their part of the solution is exact in closed form and the iteration only has to
act on the rest:

    x = sum_{c in E} psi_c <psi_c|b> / (eps_c - eps_v) + x_perp,
    Q (H - eps_v) Q x_perp = Q b,   Q = P_c - sum_{c in E} |psi_c><psi_c|,

whose smallest eigenvalue is eps_{c_max + 1} - eps_v. This is the same projected PCG with the
empty states appended to the occupied ones in the projector; the sum splits exactly because H
leaves span(E) invariant.
"""
from __future__ import annotations

import numpy as np

from .model import OracleCell
from .sternheimer import pcg_solve, project


def deflated_solve(cell: OracleCell, psi: np.ndarray, eps_s: np.ndarray, tkin_s: np.ndarray, b: np.ndarray,
                   psi_e: np.ndarray, eps_e: np.ndarray, tol: float, max_iter: int = 1000):
    """x for the rows of b (b in range(P_c)) with the empty states psi_e [nE, npw] of energies eps_e
    taken out; returns (x, iterations of the remaining projected PCG, its true residual)."""
    coef = (b @ psi_e.conj().T) / (eps_e[None, :] - eps_s[:, None])
    x_e = coef @ psi_e
    ext = np.vstack([psi, psi_e]) if len(psi_e) else psi
    x_perp, iters, res = pcg_solve(cell, ext, eps_s, tkin_s, project(ext, b), tol, max_iter)
    return x_e + x_perp, iters, res
