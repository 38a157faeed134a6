"""Oracle Sternheimer solve and density response (TEST INFRASTRUCTURE ONLY).

Sec. II.A states that the density response is evaluated within DFPT by
solving the Sternheimer equation; the steps below are the standard DFPT
definitions that statement refers to, written out plainly:

  b_{v,i}  = -P_c [dV_i psi_v]            (product formed on the grid, exact);
             a b of norm <= 1e-12 ||dV_i psi_v|| is zero (reading: dV_i psi_v then
             lies in the occupied span, e.g. dV_i constant, and what the projection
             leaves is its rounding, which the projected operator cannot resolve)
  A_v      = P_c (H - eps_v) P_c          (SPD on range(P_c) when eps_v < eps_LUMO)
  solve A_v x = b by preconditioned CG from x = 0 with z = P_c (K_v o r), where
  K_v(G)   = (27 + 18y + 12y^2 + 8y^3) / (27 + 18y + 12y^2 + 8y^3 + 16y^4),
             y = (|G|^2 / 2) / T_v, T_v = <psi_v| -nabla^2/2 |psi_v>
             (Teter, Payne and Allan, Phys. Rev. B 40, 12255 (1989)),
             with T_v floored at the kinetic energy of the smallest nonzero G;
  stop when the FP64 true residual ||b - A x|| / ||b|| <= tol;
  dn_i(r)  = 4 Re sum_v conj(psi_v(r)) x_{v,i}(r)   (2 for spin x 2 for psi* dpsi + c.c.).
"""
from __future__ import annotations

import math

import numpy as np

from .model import OracleCell


def project(psi: np.ndarray, y: np.ndarray) -> np.ndarray:
    """P_c y = y - sum_v psi_v <psi_v|y> for rows y [nb, npw], psi [n_occ, npw]."""
    return y - (y @ psi.conj().T) @ psi


def teter(y: np.ndarray) -> np.ndarray:
    num = 27.0 + 18.0 * y + 12.0 * y ** 2 + 8.0 * y ** 3
    return num / (num + 16.0 * y ** 4)


def band_kinetic(cell: OracleCell, psi: np.ndarray) -> np.ndarray:
    """T_v = sum_G |G|^2/2 |c_vG|^2, floored at (2 pi / L)^2 / 2."""
    t = np.sum(0.5 * cell.g2[None, :] * np.abs(psi) ** 2, axis=1)
    return np.maximum(t, 0.5 * cell.b ** 2)


RHS_CUT = 1e-12


def rhs(cell: OracleCell, psi: np.ndarray, dv_r: np.ndarray, bands, perts) -> np.ndarray:
    """b for the pairs (bands[k], perts[k]): -P_c of the sphere part of dV_i psi_v, or zero
    when that is at most RHS_CUT of the unprojected product."""
    out = np.empty((len(bands), cell.npw), dtype=np.complex128)
    for k, (v, i) in enumerate(zip(bands, perts)):
        f = cell.from_grid(dv_r[i][None] * cell.to_grid(psi[v]))
        out[k] = -project(psi, f)[0]
        if np.linalg.norm(out[k]) <= RHS_CUT * np.linalg.norm(f):
            out[k] = 0.0
    return out


def _op(cell, psi, eps_s, p):
    """A_v p = P_c (H - eps_v) P_c p, row by row."""
    pp = project(psi, p)
    return project(psi, cell.h_apply(pp) - eps_s[:, None] * pp)


def _dot(a, b):
    return np.real(np.sum(np.conj(a) * b, axis=1))


def pcg_solve(cell: OracleCell, psi: np.ndarray, eps_s: np.ndarray, tkin_s: np.ndarray,
              b: np.ndarray, tol: float, max_iter: int = 1000):
    """Projected PCG for every row of b (independent solves, vectorised over rows).

    Returns (x [S, npw], iterations [S], true relative residual [S])."""
    S = b.shape[0]
    K = teter(0.5 * cell.g2[None, :] / tkin_s[:, None])
    x = np.zeros_like(b)
    r = b.copy()
    z = project(psi, K * r)
    p = z.copy()
    rz = _dot(r, z)
    bn = np.linalg.norm(b, axis=1)
    iters = np.zeros(S, dtype=np.int64)
    res = np.zeros(S)
    done = bn == 0.0
    for _ in range(max_iter):
        a = np.flatnonzero(~done)
        if a.size == 0:
            break
        q = _op(cell, psi, eps_s[a], p[a])
        alpha = rz[a] / _dot(p[a], q)
        x[a] += alpha[:, None] * p[a]
        r[a] -= alpha[:, None] * q
        iters[a] += 1
        small = np.linalg.norm(r[a], axis=1) <= tol * bn[a]
        if np.any(small):
            c = a[small]
            rt = b[c] - _op(cell, psi, eps_s[c], x[c])
            tr = np.linalg.norm(rt, axis=1) / bn[c]
            ok = tr <= tol
            done[c[ok]] = True
            res[c[ok]] = tr[ok]
            bad = c[~ok]
            if bad.size:  # restart from the true residual
                r[bad] = rt[~ok]
        go = np.flatnonzero(~done)
        go_new = np.intersect1d(go, a)
        if go_new.size == 0:
            continue
        restarted = np.isin(go_new, a[small]) if np.any(small) else np.zeros(go_new.size, bool)
        zn = project(psi, K[go_new] * r[go_new])
        rzn = _dot(r[go_new], zn)
        beta = np.where(restarted, 0.0, rzn / rz[go_new])
        p[go_new] = zn + beta[:, None] * p[go_new]
        rz[go_new] = rzn
    a = np.flatnonzero(~done)
    if a.size:
        rt = b[a] - _op(cell, psi, eps_s[a], x[a])
        res[a] = np.linalg.norm(rt, axis=1) / np.where(bn[a] > 0, bn[a], 1.0)
    return x, iters, res


def delta_n(cell: OracleCell, psi: np.ndarray, x: np.ndarray, bands, perts, n_pert: int) -> np.ndarray:
    """dn_i(r) = (4 / Omega) Re sum_v conj(psi~_v(r)) x~_{v,i}(r), summed in band order."""
    N = cell.N
    dn = np.zeros((n_pert, N, N, N))
    psi_r = {}
    for k, (v, i) in enumerate(zip(bands, perts)):
        if v not in psi_r:
            psi_r[v] = cell.to_grid(psi[v])[0]
        dn[i] += np.real(np.conj(psi_r[v]) * cell.to_grid(x[k])[0])
    return dn * (4.0 / cell.omega)


def apply_chi0(cell: OracleCell, psi: np.ndarray, eps: np.ndarray, dv_r: np.ndarray, tol: float,
               bands=None, perts=None, max_iter: int = 1000, batch: int = 64):
    """dn = chi0 dV for every field (or the listed perturbations), summed over the
    listed bands (default: all occupied). psi rows are in this cell's basis order.

    Returns dict(dn [n_pert, N, N, N], x [S, npw], pairs [(v, i)], iters, resid)."""
    n_occ = psi.shape[0]
    n_pert = dv_r.shape[0]
    bands = list(range(n_occ)) if bands is None else list(bands)
    perts = list(range(n_pert)) if perts is None else list(perts)
    pairs = [(v, i) for i in perts for v in bands]
    tk = band_kinetic(cell, psi)
    xs, its, rs = [], [], []
    for s in range(0, len(pairs), batch):
        chunk = pairs[s:s + batch]
        bv = [p[0] for p in chunk]
        bi = [p[1] for p in chunk]
        b = rhs(cell, psi, dv_r, bv, bi)
        x, it, res = pcg_solve(cell, psi, eps[bv], tk[bv], b, tol, max_iter)
        xs.append(x)
        its.append(it)
        rs.append(res)
    x = np.concatenate(xs)
    dn = delta_n(cell, psi, x, [p[0] for p in pairs], [p[1] for p in pairs], n_pert)
    return dict(dn=dn, x=x, pairs=pairs, iters=np.concatenate(its), resid=np.concatenate(rs))


def chi0_matrix(cell: OracleCell, dv_r: np.ndarray, dn: np.ndarray) -> np.ndarray:
    """M_ij = <dV_j | dn_i> = (Omega / N^3) sum_r dV_j(r) dn_i(r)."""
    n = dv_r.shape[0]
    return (cell.omega / cell.N ** 3) * (dn.reshape(n, -1) @ dv_r.reshape(n, -1).T)


def rel_l2(a: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-field relative L2 error over grid points."""
    a = a.reshape(a.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
