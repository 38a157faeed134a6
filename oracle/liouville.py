"""Liouville superoperator of TDDFT in the Tamm-Dancoff approximation (TEST INFRASTRUCTURE ONLY).

Sec. II.C.1, eq. bse_tddft: the excitation energies w_s solve (D + K1e - K1d) A_s = w_s A_s over
auxiliary orbitals A_s = {a_{s,v}}, one per occupied band, with Delta gamma_s = sum_v |a_{s,v}><psi_v|.
The paper names the three terms (D: electron-hole energy differences; K1e, K1d: exchange and direct
electron-hole interaction) but not their formulas. The reading here is closed-shell singlet
excitations with the Hartree kernel: the model Hamiltonian carries no exchange-correlation
functional, so K1d = 0, as in TDDFT with a semilocal functional, and

    (D A)_v   = P_c (H - eps_v) a_v,
    (K1e A)_v = 2 P_c [ V[rho_A] psi_v ],   rho_A(r) = sum_v' conj(psi_v'(r)) a_v'(r),
    V[rho](r) = int rho(r') / |r - r'| dr' = sum_{q != 0} (4 pi / |q|^2) rho(q) e^{i q.r},

rho(q) = Omega^-1 int rho e^{-i q.r}, on the A with a_v in range(P_c) (inputs are projected first).
rho_A is band-limited to the 4 Ecut sphere, which the grid holds exactly, so the grid route has no
aliasing. <B|K1e A> = 2 Omega sum_{q != 0} (4 pi / |q|^2) conj(rho_B(q)) rho_A(q): the operator is
Hermitian in <A|B> = sum_v <a_v|b_v>, and positive definite when the gap is open.

Hybrid functionals add the direct term with a fraction alpha of bare exchange, built from the
Coulomb integrals of occupied pairs (eq. tau_u):

    (K1d A)_v = alpha P_c sum_v' tau_{v'v}(r) a_v'(r),   tau_{v'v} = V[conj(psi_v') psi_v],

so that L = D + K1e - K1d. <B|K1d A> = alpha sum_{v,v'} int conj(b_v) tau_{v'v} a_v' is Hermitian, as
tau_{vv'} = conj(tau_{v'v}); for plane-wave states it couples transitions with the same momentum
transfer by alpha 4 pi / (Omega |k_v - k_v'|^2) (v != v'; q = 0 omitted, as in V).

BSE replaces the bare interaction of the direct term by the screened W of eq. tau. With the PDEP
eigenpairs of chi-bar0 (Sec. II.A, eq. pdep), W = v + sum_a (v^{1/2} phi_a) lambda_a / (1 - lambda_a)
(v^{1/2} phi_a)^T on the span of the phi_a. Here the direct term takes the interaction
alpha v + sum_a w_a c_a w_a^T for real grid potentials w_a and weights c_a, acting as
V_W[rho](r) = alpha V[rho](r) + sum_a w_a(r) c_a <w_a, rho>, <f, g> = N^-3 sum_j f(r_j) g(r_j);
screening_from_chibar0 builds w_a = v^{1/2} g_a and c_a = lambda_a / (1 - lambda_a) from the dense
chi-bar0 of oracle/pdep.py (g_a its eigenfunctions, normalised to a unit cell average of g_a^2),
and alpha = 1 with them is BSE's W.

Routes, pinned against each other and against closed forms:
* liouville_apply: the grid route above (FFTs of the oracle cell);
* casida_tda: the matrix in the transition basis {a_v' = delta_vv' psi_c} from a full
  diagonalisation, L_{vc,v'c'} = (eps_c - eps_v) delta + 2 Omega sum_q (4 pi/|q|^2) conj(rho_vc(q)) rho_v'c'(q)
  with rho_vc = conj(psi_v) psi_c;
* free_electron_tda: for plane-wave occupied and empty states k, the same matrix written out by
  hand: (|k_c|^2 - |k_v|^2)/2 on the diagonal plus 8 pi / (Omega |q|^2) between transitions with the
  same momentum transfer q = k_c - k_v.
liouville_residual measures a solution of L z = b under liouville_apply, for the Z-vector solve.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

from .model import OracleCell, sphere_miller, WORKERS
from .sternheimer import project


def coulomb_q(cell: OracleCell):
    """Miller indices [n_q, 3] of the 4 Ecut sphere without q = 0, and 4 pi / |q|^2 on them."""
    mq = sphere_miller(cell.L, 4.0 * cell.ecut)
    mq = mq[np.any(mq != 0, axis=1)]
    q2 = np.sum((mq * cell.b) ** 2, axis=1)
    return mq, 4.0 * math.pi / q2


def hartree_grid(cell: OracleCell, rho_r: np.ndarray) -> np.ndarray:
    """V[rho](r_j) for complex band-limited densities rho_r [n, N, N, N]."""
    N = cell.N
    mq, vq = coulomb_q(cell)
    ix, iy, iz = (mq[:, 0] % N, mq[:, 1] % N, mq[:, 2] % N)
    rq = sfft.fftn(rho_r, axes=(1, 2, 3), workers=WORKERS, norm="forward")  # rho(q)
    box = np.zeros_like(rq)
    box[:, ix, iy, iz] = vq[None, :] * rq[:, ix, iy, iz]
    return sfft.ifftn(box, axes=(1, 2, 3), workers=WORKERS, norm="forward")  # sum_q V(q) e^{i q r}


def screened_grid(cell: OracleCell, rho_r: np.ndarray, alpha_x: float, screen) -> np.ndarray:
    """alpha V[rho] + sum_a w_a c_a <w_a, rho> for densities rho_r [n, N, N, N]; screen = (w [m, N, N, N], c [m])."""
    out = alpha_x * hartree_grid(cell, rho_r) if alpha_x != 0.0 else np.zeros_like(rho_r)
    if screen is not None:
        w, c = screen
        N3 = cell.N ** 3
        proj = np.einsum("axyz,nxyz->na", w, rho_r) / N3          # <w_a, rho_n>
        out = out + np.einsum("axyz,na->nxyz", w, proj * c[None, :])
    return out


def screening_from_chibar0(cell: OracleCell, M: np.ndarray, fields: np.ndarray, vh: np.ndarray):
    """(w [2m, N, N, N], c [2m]) of W - v from the dense chi-bar0 M in the real basis fields [2m, N, N, N]
    with v^{1/2} vh [2m] (oracle/pdep.py): w_a = sum_j U_ja vh_j f_j, c_a = lambda_a / (1 - lambda_a)."""
    lam, U = np.linalg.eigh(0.5 * (M + M.T))
    w = np.einsum("ja,jxyz->axyz", U * vh[:, None], fields)
    return w, lam / (1.0 - lam)


def liouville_apply(cell: OracleCell, psi: np.ndarray, eps: np.ndarray, A: np.ndarray,
                    alpha_x: float = 0.0, screen=None) -> np.ndarray:
    """(D + K1e - K1d) A for A [n_exc, n_occ, npw] (oracle order); psi [n_occ, npw], eps [n_occ];
    K1d with the interaction alpha_x v + sum_a w_a c_a w_a^T (screen = (w, c) or None)."""
    A = np.asarray(A, dtype=np.complex128)
    n_exc, n_occ, npw = A.shape
    Ap = project(psi, A.reshape(-1, npw)).reshape(n_exc, n_occ, npw)
    out = np.empty_like(Ap)
    psi_r = cell.to_grid(psi)                                    # psi~_v(r) = sqrt(Omega) psi_v(r)
    tau = None
    if alpha_x != 0.0 or screen is not None:                     # tau[v', v] = V_W[conj(psi_v') psi_v]
        tau = np.stack([screened_grid(cell, np.conj(psi_r) * psi_r[v][None] / cell.omega, alpha_x, screen)
                        for v in range(n_occ)], 1)
    for e in range(n_exc):
        d = cell.h_apply(Ap[e]) - eps[:, None] * Ap[e]
        a_r = cell.to_grid(Ap[e])
        rho = np.sum(np.conj(psi_r) * a_r, axis=0)[None] / cell.omega
        v = hartree_grid(cell, rho)[0]
        k = 2.0 * cell.from_grid(v[None] * psi_r)
        if tau is not None:
            k -= cell.from_grid(np.einsum("wvxyz,wxyz->vxyz", tau, a_r))
        out[e] = project(psi, d + k)
    return out


def liouville_residual(cell: OracleCell, psi: np.ndarray, eps: np.ndarray, b: np.ndarray, z: np.ndarray,
                       alpha_x: float = 0.0, screen=None) -> np.ndarray:
    """||b - L z|| / ||b|| per excitation (norms over all bands)."""
    r = b - liouville_apply(cell, psi, eps, z, alpha_x, screen)
    n = b.shape[0]
    return np.linalg.norm(r.reshape(n, -1), axis=1) / np.linalg.norm(b.reshape(n, -1), axis=1)


def casida_tda(cell: OracleCell, n_occ: int, alpha_x: float = 0.0, screen=None):
    """Dense L in the transition basis t = v * n_emp + c from a full diagonalisation of H, with the
    direct term of the interaction alpha_x v + sum_a w_a c_a w_a^T:
    L_{vc,v'c'} -= alpha_x Omega sum_q (4 pi/|q|^2) conj(rho_{c'c}(q)) rho_{v'v}(q)
                   + Omega sum_a c_a <w_a, rho_{cc'}> <w_a, rho_{v'v}>.
    Returns (L [n_occ n_emp, n_occ n_emp], occupied psi, eps_occ, empty psi, eps_emp)."""
    e, U = np.linalg.eigh(cell.h_dense())
    psi = U.T
    occ, emp = psi[:n_occ], psi[n_occ:]
    eo, ee = e[:n_occ], e[n_occ:]
    n_emp = emp.shape[0]
    N = cell.N
    mq, vq = coulomb_q(cell)
    ix, iy, iz = (mq[:, 0] % N, mq[:, 1] % N, mq[:, 2] % N)
    occ_r = cell.to_grid(occ)
    emp_r = cell.to_grid(emp)
    rho_q = np.empty((n_occ, n_emp, len(vq)), dtype=np.complex128)
    for v in range(n_occ):
        rv = np.conj(occ_r[v])[None] * emp_r / cell.omega        # rho_vc(r), physical normalisation
        rq = sfft.fftn(rv, axes=(1, 2, 3), workers=WORKERS, norm="forward")
        rho_q[v] = rq[:, ix, iy, iz]
    R = rho_q.reshape(n_occ * n_emp, -1)
    L = 2.0 * cell.omega * (R.conj() * vq[None, :]) @ R.T
    L[np.diag_indices_from(L)] += (ee[None, :] - eo[:, None]).reshape(-1)
    if alpha_x != 0.0 or screen is not None:
        def pair_q(a_r, b_r):                                   # rho_ab(q) for rho_ab = conj(a) b
            out = np.empty((a_r.shape[0], b_r.shape[0], len(vq)), dtype=np.complex128)
            for i in range(a_r.shape[0]):
                rq = sfft.fftn(np.conj(a_r[i])[None] * b_r / cell.omega, axes=(1, 2, 3), workers=WORKERS,
                               norm="forward")
                out[i] = rq[:, ix, iy, iz]
            return out
        Rvv = pair_q(occ_r, occ_r)                              # [v', v, q]
        Rcc = pair_q(emp_r, emp_r)                              # [c', c, q]
        # K1d[(v,c),(v',c')] = Omega sum_q conj(rho_{c'c}(q)) w(q) rho_{v'v}(q)
        K = alpha_x * cell.omega * np.einsum("dcq,q,wvq->vcwd", Rcc.conj(), vq, Rvv, optimize=True)
        if screen is not None:
            w, cw = screen
            wq = sfft.fftn(w, axes=(1, 2, 3), workers=WORKERS, norm="forward")[:, ix, iy, iz]  # w_a(q)
            pc = np.einsum("aq,cdq->acd", wq.conj(), Rcc)                            # <w_a, rho_{cc'}>
            pv = np.einsum("aq,wvq->awv", wq.conj(), Rvv)                            # <w_a, rho_{v'v}>
            K += cell.omega * np.einsum("a,acd,awv->vcwd", cw, pc, pv, optimize=True)
        L -= K.reshape(n_occ * n_emp, n_occ * n_emp)
    return L, occ, eo, emp, ee


def free_electron_tda(cell: OracleCell, occ_idx, emp_idx, alpha_x: float = 0.0) -> np.ndarray:
    """Hand-written L for plane-wave states (basis indices of the oracle cell): transitions
    t = (occ_idx[v], emp_idx[c]) in the order v * len(emp_idx) + c."""
    k = cell.miller
    trans = [(v, c) for v in occ_idx for c in emp_idx]
    L = np.zeros((len(trans), len(trans)))
    for a, (v, c) in enumerate(trans):
        qa = k[c] - k[v]
        L[a, a] = 0.5 * (cell.g2[c] - cell.g2[v])
        for b, (w, d) in enumerate(trans):
            if np.array_equal(k[d] - k[w], qa):
                L[a, b] += 8.0 * math.pi / (cell.omega * float(np.sum((qa * cell.b) ** 2)))
                if w != v:
                    dk = k[v] - k[w]
                    L[a, b] -= alpha_x * 4.0 * math.pi / (cell.omega * float(np.sum((dk * cell.b) ** 2)))
    return L


def lanczos_chain(Lmat: np.ndarray, d: np.ndarray, n_steps: int):
    """Hermitian Lanczos on a dense matrix from d: alpha [n], beta [n] (beta[k] couples steps k and
    k+1) and ||d||^2; plain three-term recurrence, no reorthogonalisation, in the order it is written:
    q_0 = d/||d||, w = L q_k - beta_{k-1} q_{k-1}, alpha_k = <q_k|w>, w -= alpha_k q_k,
    beta_k = ||w||, q_{k+1} = w / beta_k."""
    nrm2 = float(np.vdot(d, d).real)
    q_prev = np.zeros_like(d)
    q = d / np.sqrt(nrm2)
    alpha, beta = np.zeros(n_steps), np.zeros(n_steps)
    b_prev = 0.0
    for k in range(n_steps):
        w = Lmat @ q - b_prev * q_prev
        alpha[k] = np.vdot(q, w).real
        w = w - alpha[k] * q
        beta[k] = np.linalg.norm(w)
        q_prev, q, b_prev = q, w / beta[k], beta[k]
    return alpha, beta, nrm2


def spectrum_from_chain(alpha, beta, nrm2, omega, eta):
    """-Im <d|(w + i eta - L)^{-1}|d> / pi from a Lanczos chain, by the continued fraction
    nrm2 / (z - a_0 - b_0^2 / (z - a_1 - b_1^2 / ...)), z = w + i eta, closed after the last step."""
    z = np.asarray(omega, dtype=np.float64) + 1j * eta
    g = np.zeros_like(z)
    for k in range(len(alpha) - 1, -1, -1):
        tail = beta[k] ** 2 * g if k < len(alpha) - 1 else 0.0
        g = 1.0 / (z - alpha[k] - tail)
    return -(nrm2 * g).imag / np.pi


def spectrum_exact(Lmat: np.ndarray, d: np.ndarray, omega, eta):
    """-Im <d|(w + i eta - L)^{-1}|d> / pi from the eigenpairs of the dense L."""
    w, U = np.linalg.eigh(Lmat)
    amp = np.abs(U.conj().T @ d) ** 2
    z = np.asarray(omega, dtype=np.float64)[:, None] + 1j * eta
    return -(amp[None, :] / (z - w[None, :])).sum(axis=1).imag / np.pi
