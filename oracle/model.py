"""Oracle model: plane-wave basis, local potential, KB projectors, H (TEST INFRASTRUCTURE ONLY).

Conventions (Hartree atomic units; the paper's workflow, Sec. II, takes the
Hamiltonian from a plane-wave ground-state code and fixes none of these):
  * cubic cell of edge L, Omega = L^3, Gamma point, G = (2 pi / L) n,
    basis |G|^2 <= Ecut with Ecut in Ry (so |G|^2 is in bohr^-2);
  * psi(r) = Omega^(-1/2) sum_G c_G exp(i G.r); the grid is r_j = L j / N;
  * V(q) = A (2 pi s^2)^(3/2) / Omega exp(-s^2 |q|^2 / 2) sum_a exp(-i q.R_a),
    the Fourier series of the periodic sum of A exp(-|r-R_a|^2 / 2 s^2);
    <G|V|G'> = V(G - G'), and on the grid V(r_j) = sum_{|q|^2 <= 4 Ecut} V(q) e^{i q.r_j};
  * beta_a(G) = Omega^(-1/2) exp(-w^2 |G|^2 / 2) exp(-i G.R_a), H_KB = D sum_a |beta_a><beta_a|.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

WORKERS = max(1, len(os.sched_getaffinity(0)))


def fft_grid(L: float, ecut: float) -> int:
    """Smallest N = 2^a 3^b with N >= 2 (floor(2 sqrt(Ecut) L / 2 pi) + 1) + 1.

    The grid then holds the 4 Ecut sphere without aliasing, so every product
    formed on it below is exact in the basis."""
    nmax = int(math.floor(2.0 * math.sqrt(ecut) * L / (2.0 * math.pi)))
    need = 2 * (nmax + 1) + 1
    n = need
    while True:
        m = n
        while m % 2 == 0:
            m //= 2
        while m % 3 == 0:
            m //= 3
        if m == 1:
            return n
        n += 1


def sphere_miller(L: float, ecut: float) -> np.ndarray:
    """All n in Z^3 with (2 pi / L)^2 |n|^2 <= ecut; oracle's own order (|n|^2, then n)."""
    r2 = ecut * L * L / (4.0 * math.pi * math.pi)
    nm = int(math.floor(math.sqrt(r2)))
    pts = []
    for a in range(-nm, nm + 1):
        for b in range(-nm, nm + 1):
            for c in range(-nm, nm + 1):
                if a * a + b * b + c * c <= r2:
                    pts.append((a * a + b * b + c * c, a, b, c))
    pts.sort()
    return np.array([p[1:] for p in pts], dtype=np.int64).reshape(-1, 3)


class OracleCell:
    """Basis and Hamiltonian of one cell."""

    def __init__(self, L, ecut, pos, amp=-2.0, sigma=1.0, D=1.0, width=1.0, N=None):
        self.L = float(L)
        self.ecut = float(ecut)
        self.pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        self.amp, self.sigma, self.D, self.width = float(amp), float(sigma), float(D), float(width)
        self.omega = self.L ** 3
        self.N = fft_grid(L, ecut) if N is None else int(N)
        self.miller = sphere_miller(L, ecut)
        self.npw = len(self.miller)
        self.b = 2.0 * math.pi / self.L
        self.gvec = self.miller * self.b
        self.g2 = np.sum(self.gvec ** 2, axis=1)
        N = self.N
        self.ix = self.miller[:, 0] % N
        self.iy = self.miller[:, 1] % N
        self.iz = self.miller[:, 2] % N
        self.v_r = self._vloc_grid()
        self.beta = self._kb_beta()

    # -- local potential -------------------------------------------------
    def vloc_q(self, qvec: np.ndarray) -> np.ndarray:
        q2 = np.sum(qvec ** 2, axis=1)
        s = self.sigma
        pref = self.amp * (2.0 * math.pi * s * s) ** 1.5 / self.omega * np.exp(-0.5 * s * s * q2)
        phase = np.exp(-1j * (qvec @ self.pos.T))
        return pref * phase.sum(axis=1)

    def _vloc_grid(self) -> np.ndarray:
        N = self.N
        mq = sphere_miller(self.L, 4.0 * self.ecut)
        box = np.zeros((N, N, N), dtype=np.complex128)
        box[mq[:, 0] % N, mq[:, 1] % N, mq[:, 2] % N] = self.vloc_q(mq * self.b)
        v = sfft.ifftn(box, workers=WORKERS, norm="forward")  # sum_q V(q) e^{i q r_j}
        return np.ascontiguousarray(v.real)

    def _kb_beta(self) -> np.ndarray:
        w = self.width
        radial = np.exp(-0.5 * w * w * self.g2) / math.sqrt(self.omega)
        return radial[None, :] * np.exp(-1j * (self.pos @ self.gvec.T))

    # -- grid transforms ---------------------------------------------------
    def to_grid(self, c: np.ndarray) -> np.ndarray:
        """rows c [nb, npw] -> f(r_j) = sum_G c_G exp(i G.r_j), shape [nb, N, N, N]."""
        c = np.atleast_2d(c)
        N = self.N
        box = np.zeros((c.shape[0], N, N, N), dtype=np.complex128)
        box[:, self.ix, self.iy, self.iz] = c
        return sfft.ifftn(box, axes=(1, 2, 3), workers=WORKERS, norm="forward")

    def from_grid(self, f: np.ndarray) -> np.ndarray:
        """f [nb, N, N, N] -> coefficients (1/N^3) sum_j exp(-i G.r_j) f(r_j) on the sphere."""
        F = sfft.fftn(f, axes=(1, 2, 3), workers=WORKERS, norm="forward")
        return F[:, self.ix, self.iy, self.iz]

    # -- Hamiltonian -------------------------------------------------------
    def h_apply(self, c: np.ndarray, chunk: int = 16) -> np.ndarray:
        """H c for rows c [nb, npw]: kinetic + local (via the grid) + KB."""
        c = np.atleast_2d(c)
        out = np.empty_like(c)
        for s in range(0, c.shape[0], chunk):
            blk = c[s:s + chunk]
            out[s:s + chunk] = self.from_grid(self.v_r[None] * self.to_grid(blk))
        out += 0.5 * self.g2[None, :] * c
        out += self.D * ((c @ self.beta.conj().T) @ self.beta)
        return out

    def h_dense(self) -> np.ndarray:
        """Dense H_GG' = 1/2 |G|^2 delta + V(G - G') + D sum_a beta_a(G) conj beta_a(G')."""
        dq = (self.miller[:, None, :] - self.miller[None, :, :]).reshape(-1, 3) * self.b
        h = self.vloc_q(dq).reshape(self.npw, self.npw)
        h[np.diag_indices(self.npw)] += 0.5 * self.g2
        h += self.D * (self.beta.T @ self.beta.conj())
        return h

    def potential_dense(self, f_r: np.ndarray) -> np.ndarray:
        """Dense matrix <G|f|G'> = f(G - G') of a real band-limited grid field f."""
        N = self.N
        fq = sfft.fftn(f_r, workers=WORKERS, norm="forward")
        d = (self.miller[:, None, :] - self.miller[None, :, :]) % N
        return fq[d[..., 0], d[..., 1], d[..., 2]]

    # -- mapping foreign coefficient arrays onto this basis ------------------
    def index_of(self, miller: np.ndarray) -> np.ndarray:
        """Position in this basis of each Miller triple (raises if one is missing)."""
        key = {tuple(m): k for k, m in enumerate(self.miller.tolist())}
        return np.array([key[tuple(m)] for m in np.asarray(miller).tolist()], dtype=np.int64)

    def take(self, c: np.ndarray, miller: np.ndarray) -> np.ndarray:
        """Reorder rows given in the order `miller` into this basis' order."""
        pos = self.index_of(miller)
        if len(pos) != self.npw:
            raise ValueError("basis size mismatch")
        out = np.zeros((np.atleast_2d(c).shape[0], self.npw), dtype=np.complex128)
        out[:, pos] = np.atleast_2d(c)
        return out

    def give(self, c: np.ndarray, miller: np.ndarray) -> np.ndarray:
        """Inverse of take: rows in this basis -> rows in the order `miller`."""
        return np.atleast_2d(c)[:, self.index_of(miller)]
