"""Ground-state stand-in: lowest Kohn-Sham-like eigenpairs of the model Hamiltonian.

The paper takes the occupied states from an external ground-state code (Sec. II,
workflow paragraph: pwscf supplies psi_i and eps_i, eq. ks). Here a synthetic
model replaces that code: H = -1/2 nabla^2 + sum_a A exp(-|r-R_a|^2 / 2 sigma^2)
+ D sum_a |beta_a><beta_a|, diagonalised densely for small bases and by a block
LOBPCG (Knyazev 2001) with the Teter-Payne-Allan preconditioner otherwise.

This is input preparation, written independently of both the oracle and the
GPU library; the oracle re-checks every eigen-residual with its own operator.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

from .cells import CellSpec, fft_size, miller_sorted, place_atoms, stream_rng, STREAM_EIG

_WORKERS = max(1, len(os.sched_getaffinity(0)))


class ModelH:
    """H for one cell in the canonical plane-wave order (miller_sorted)."""

    def __init__(self, spec: CellSpec, pos: np.ndarray, N: int | None = None):
        self.spec = spec
        self.pos = pos
        self.L = spec.L
        self.omega = spec.L ** 3
        self.N = fft_size(spec.L, spec.ecut) if N is None else N
        self.miller = miller_sorted(spec.L, spec.ecut)
        self.npw = len(self.miller)
        b = 2.0 * math.pi / spec.L
        g = self.miller * b
        self.g2 = np.einsum("ij,ij->i", g, g)
        N = self.N
        self.idx = (self.miller[:, 0] % N, self.miller[:, 1] % N, self.miller[:, 2] % N)
        # V(q) on the 4 Ecut sphere, placed at q mod N
        mq = miller_sorted(spec.L, 4.0 * spec.ecut)
        q = mq * b
        q2 = np.einsum("ij,ij->i", q, q)
        s = spec.vloc_sigma
        pref = spec.vloc_amp * (2.0 * math.pi * s * s) ** 1.5 / self.omega * np.exp(-0.5 * s * s * q2)
        vq = pref * np.exp(-1j * (q @ pos.T)).sum(axis=1)
        self.vq_box = np.zeros((N, N, N), dtype=np.complex128)
        self.vq_box[mq[:, 0] % N, mq[:, 1] % N, mq[:, 2] % N] = vq
        vr = sfft.ifftn(self.vq_box, workers=_WORKERS) * N ** 3
        self.v_r = vr.real.copy()
        w = spec.kb_width
        self.beta = (np.exp(-0.5 * w * w * self.g2)[None, :] * np.exp(-1j * (pos @ g.T))) / math.sqrt(self.omega)

    def apply(self, c: np.ndarray, chunk: int = 32) -> np.ndarray:
        """H c for rows c [nb, npw]."""
        out = np.empty_like(c)
        N = self.N
        for s in range(0, c.shape[0], chunk):
            blk = c[s:s + chunk]
            box = np.zeros((blk.shape[0], N, N, N), dtype=np.complex128)
            box[:, self.idx[0], self.idx[1], self.idx[2]] = blk
            f = sfft.ifftn(box, axes=(1, 2, 3), workers=_WORKERS, norm="forward")
            f *= self.v_r[None]
            f = sfft.fftn(f, axes=(1, 2, 3), workers=_WORKERS, norm="forward")
            out[s:s + chunk] = f[:, self.idx[0], self.idx[1], self.idx[2]]
        out += 0.5 * self.g2[None, :] * c
        out += self.spec.kb_D * ((c @ self.beta.conj().T) @ self.beta)
        return out

    def dense(self) -> np.ndarray:
        N = self.N
        m = self.miller
        d = (m[:, None, :] - m[None, :, :]) % N
        h = self.vq_box[d[..., 0], d[..., 1], d[..., 2]]
        h[np.diag_indices(self.npw)] += 0.5 * self.g2
        h += self.spec.kb_D * (self.beta.T @ self.beta.conj())
        return h


def _teter(y):
    num = 27.0 + y * (18.0 + y * (12.0 + 8.0 * y))
    return num / (num + 16.0 * y ** 4)


def _svqb(V, HV, drop=1e-13):
    S = V.conj().T @ V
    d = 1.0 / np.sqrt(np.real(np.diag(S)))
    S = d[:, None] * S * d[None, :]
    th, U = np.linalg.eigh(0.5 * (S + S.conj().T))
    keep = th > drop * th.max()
    T = (d[:, None] * U[:, keep]) / np.sqrt(th[keep])[None, :]
    return V @ T, (HV @ T if HV is not None else None)


def lobpcg(H: ModelH, nb: int, nconv: int, tol: float, rng, maxit: int = 600, verbose=False):
    """Lowest nb eigenpairs of H (columns); stops when the lowest nconv have
    ||H x - theta x|| < tol. Returns (theta, X [npw, nb], residual norms)."""
    npw = H.npw
    kin = 0.5 * H.g2
    X = (rng.standard_normal((npw, nb)) + 1j * rng.standard_normal((npw, nb))) / (1.0 + kin)[:, None]
    X, _ = _svqb(X, None)
    X, _ = _svqb(X, None)
    HX = H.apply(X.T).T
    A = X.conj().T @ HX
    th, C = np.linalg.eigh(0.5 * (A + A.conj().T))
    X, HX = X @ C, HX @ C
    P = HP = None
    floor = 0.5 * (2.0 * math.pi / H.L) ** 2
    rn = None
    for it in range(maxit):
        if it and it % 25 == 0:
            HX = H.apply(X.T).T
        R = HX - X * th[None, :]
        rn = np.linalg.norm(R, axis=0)
        if verbose and it % 10 == 0:
            print(f"  lobpcg it {it}: max res (wanted) {rn[:nconv].max():.2e}", flush=True)
        if np.all(rn[:nconv] < tol):
            break
        act = rn > 0.1 * tol
        Tk = np.maximum(np.real(np.sum(np.abs(X[:, act]) ** 2 * kin[:, None], axis=0)), floor)
        W = R[:, act] * _teter(kin[:, None] / Tk[None, :])
        for _ in range(2):
            W -= X @ (X.conj().T @ W)
        HW = H.apply(W.T).T
        if P is not None:
            Z, HZ = np.concatenate([W, P], axis=1), np.concatenate([HW, HP], axis=1)
        else:
            Z, HZ = W, HW
        for _ in range(2):
            cf = X.conj().T @ Z
            Z = Z - X @ cf
            HZ = HZ - HX @ cf
        Z, HZ = _svqb(Z, HZ)
        Z, HZ = _svqb(Z, HZ)
        Q = np.concatenate([X, Z], axis=1)
        HQ = np.concatenate([HX, HZ], axis=1)
        A = Q.conj().T @ HQ
        th_all, C = np.linalg.eigh(0.5 * (A + A.conj().T))
        C = C[:, :nb]
        th = th_all[:nb]
        Cx, Cz = C[:nb], C[nb:]
        newX = X @ Cx + Z @ Cz
        newHX = HX @ Cx + HZ @ Cz
        act2 = rn > tol
        P = Z @ Cz[:, act2]
        HP = HZ @ Cz[:, act2]
        if P.shape[1] == 0:
            P = HP = None
        X, HX = newX, newHX
        # keep X orthonormal in FP64 over many iterations
        if it % 10 == 9:
            X, HX = _svqb(X, HX)
            A = X.conj().T @ HX
            th, C = np.linalg.eigh(0.5 * (A + A.conj().T))
            X, HX = X @ C, HX @ C
    HX = H.apply(X.T).T
    A = X.conj().T @ HX
    th, C = np.linalg.eigh(0.5 * (A + A.conj().T))
    X, HX = X @ C, HX @ C
    rn = np.linalg.norm(HX - X * th[None, :], axis=0)
    return th, X, rn


def ground_state(spec: CellSpec, dense_limit: int = 3000, tol: float = 2e-10, verbose=False, max_reseed: int = 8):
    """Occupied eigenpairs of one cell (re-seeding on a HOMO-LUMO gap < 1e-4 Ha).

    Returns dict(spec, pos, miller, psi [n_occ, npw] complex rows, eps [n_occ],
    eps_lumo, gap, resid [n_occ])."""
    for k in range(max_reseed):
        sp = spec.with_system(spec.system_id + 1000 * k)
        pos = place_atoms(sp)
        H = ModelH(sp, pos)
        if H.npw <= dense_limit:
            e, U = np.linalg.eigh(H.dense())
            eps = e[:sp.n_occ + 1]
            X = U[:, :sp.n_occ + 1]
            res = np.linalg.norm(H.apply(X.T).T - X * eps[None, :], axis=0)
        else:
            nb = sp.n_occ + max(8, sp.n_occ // 8)
            rng = stream_rng(sp.config_id, sp.system_id, STREAM_EIG)
            eps, X, res = lobpcg(H, nb, sp.n_occ + 1, tol, rng, verbose=verbose)
            eps, X, res = eps[:sp.n_occ + 1], X[:, :sp.n_occ + 1], res[:sp.n_occ + 1]
        gap = eps[sp.n_occ] - eps[sp.n_occ - 1]
        if gap >= 1e-4:
            psi = np.ascontiguousarray(X[:, :sp.n_occ].T)
            return dict(spec=sp, pos=pos, miller=H.miller, psi=psi, eps=eps[:sp.n_occ].copy(),
                        eps_lumo=float(eps[sp.n_occ]), gap=float(gap), resid=res[:sp.n_occ].copy(), N=H.N)
        if verbose:
            print(f"  gap {gap:.2e} < 1e-4 Ha, reseeding", flush=True)
    raise RuntimeError("no cell with a usable gap")
