"""Seeded synthetic cells: atom positions, perturbation fields, workload shapes.

This module only draws random numbers and lays them out; it holds none of the
Sternheimer arithmetic. It is shared by the CPU oracle, the tests and the
benchmark so that every side reads bit-identical inputs.

Model (the paper fixes none of it; see the Sternheimer paragraph of Sec. II.A,
which only states that the density response is obtained from Sternheimer
solves): a cubic cell of edge L (bohr), Gamma point, complex plane waves with
|G|^2 <= Ecut (Ecut in Ry, i.e. bohr^-2), Gaussian wells as local potential and
one s-type Kleinman-Bylander projector per atom.

Random streams: numpy default_rng(SeedSequence([config_id, system_id, stream]))
with stream 0 = atoms, 1 = perturbations, 2 = eigensolver start vectors.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

STREAM_ATOMS = 0
STREAM_DV = 1
STREAM_EIG = 2


@dataclass(frozen=True)
class CellSpec:
    """One synthetic system and the size of one chi0 apply on it."""
    name: str
    config_id: int
    L: float            # cubic cell edge, bohr
    ecut: float         # plane-wave cutoff, Ry (|G|^2 <= ecut in bohr^-2)
    n_atoms: int
    n_occ: int
    n_pert: int
    system_id: int = 0
    vloc_amp: float = -2.0    # Ha, depth of each Gaussian well
    vloc_sigma: float = 1.0   # bohr
    kb_D: float = 1.0         # Ha, KB coupling
    kb_width: float = 1.0     # beta(G) = exp(-width^2 |G|^2 / 2)
    min_sep: float = 1.5      # bohr, minimum-image atom separation

    def with_system(self, system_id: int) -> "CellSpec":
        return replace(self, system_id=system_id)


# The five workloads (cell edge, cutoff, atoms, bands, perturbations).
TINY = CellSpec("tiny_L10_8at_10Ry", 0, 10.0, 10.0, 8, 16, 8)
MID = CellSpec("mid_L20_64at_25Ry", 1, 20.0, 25.0, 64, 128, 64)
LEARNED = CellSpec("learned_L24_128at_30Ry", 3, 24.0, 30.0, 128, 256, 128)
LARGE = CellSpec("large_L32_512at_30Ry", 4, 32.0, 30.0, 512, 1024, 32)
# The large cell's box, cutoff and atoms (128^3 grid, ~91k PWs, 512 KB projectors) with
# 32 occupied bands and 4 fields: its ground state takes minutes on the host, where the
# 1024-band one takes hours.
LARGE_GRID = CellSpec("large_grid_L32_512at_30Ry", 4, 32.0, 30.0, 512, 32, 4)
# A 108^3 grid (radices 12 x 9), the other size whose FP64 plane exceeds LDS.
GRID108 = CellSpec("grid108_L24_64at_38Ry", 5, 24.0, 38.0, 64, 16, 4)


def batched_specs(n_systems: int = 32) -> list[CellSpec]:
    """Uneven cells: L ~ U[10, 18], atoms ~ U{8..48}, N_occ = 2 atoms, 20 Ry, 16 fields."""
    rng = stream_rng(2, 0, 3)
    out = []
    for s in range(n_systems):
        L = float(rng.uniform(10.0, 18.0))
        na = int(rng.integers(8, 49))
        out.append(CellSpec(f"batched_{s}", 2, L, 20.0, na, 2 * na, 16, system_id=s))
    return out


def stream_rng(config_id: int, system_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([config_id, system_id, stream]))


def place_atoms(spec: CellSpec) -> np.ndarray:
    """Sequential rejection sampling of U[0,L)^3 with minimum-image distance >= min_sep."""
    rng = stream_rng(spec.config_id, spec.system_id, STREAM_ATOMS)
    L = spec.L
    pos = np.zeros((spec.n_atoms, 3))
    n = 0
    tries = 0
    while n < spec.n_atoms:
        tries += 1
        if tries > 1000000:
            raise RuntimeError("atom placement failed")
        cand = rng.uniform(0.0, L, size=3)
        if n:
            d = pos[:n] - cand
            d -= L * np.round(d / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < spec.min_sep ** 2:
                continue
        pos[n] = cand
        n += 1
    return pos


def fft_size(L: float, ecut: float) -> int:
    """Smallest 2^a 3^b >= 2 (floor(2 sqrt(ecut) L / 2pi) + 1) + 1 (holds the 4 Ecut sphere)."""
    need = 2 * (int(math.floor(2.0 * math.sqrt(ecut) * L / (2.0 * math.pi))) + 1) + 1
    best = None
    p2 = 1
    while p2 <= 4 * need:
        p = p2
        while p <= 4 * need:
            if p >= need and (best is None or p < best):
                best = p
            p *= 3
        p2 *= 2
    return best


def miller_sorted(L: float, ecut: float, strict_quarter: bool = False) -> np.ndarray:
    """Integer triples n with (2pi/L)^2 |n|^2 <= ecut (or < ecut/4 when strict_quarter),
    sorted by |n|^2, then n_x, n_y, n_z ascending. Shape [n, 3] int64."""
    lim = ecut / 4.0 if strict_quarter else ecut
    r2 = lim * L * L / (4.0 * math.pi ** 2)
    nm = int(math.floor(math.sqrt(r2))) + 1
    ax = np.arange(-nm, nm + 1)
    n = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    n2 = np.einsum("ij,ij->i", n, n)
    keep = (n2 < r2) if strict_quarter else (n2 <= r2)
    n, n2 = n[keep], n2[keep]
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0], n2))
    return n[order]


def _is_half_space_rep(n: np.ndarray) -> np.ndarray:
    return (n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0)) | ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0))


def random_dv(spec: CellSpec, n_pert: int | None = None, N: int | None = None):
    """Band-limited real perturbations.

    For |G|^2 < ecut/4: re, im ~ N(0,1) on the half-space representatives in the
    canonical order, dV(-G) = conj dV(G); G = 0 gets a real N(0,1) value. Each
    field is scaled to sum_G |dV(G)|^2 = 1 and synthesised on the N^3 grid as
    dV(r_j) = sum_G dV(G) exp(i G.r_j), r_j = L j / N.

    Returns (miller [m,3], coeff [n_pert, m] complex, dv_r [n_pert, N, N, N] float64
    indexed [ix, iy, iz]).
    """
    n_pert = spec.n_pert if n_pert is None else n_pert
    N = fft_size(spec.L, spec.ecut) if N is None else N
    mil = miller_sorted(spec.L, spec.ecut, strict_quarter=True)
    rep = _is_half_space_rep(mil)
    zero = np.all(mil == 0, axis=1)
    # partner index of -G for every G
    key = {tuple(v): k for k, v in enumerate(mil.tolist())}
    partner = np.array([key[(-a, -b, -c)] for a, b, c in mil.tolist()])
    rng = stream_rng(spec.config_id, spec.system_id, STREAM_DV)
    coeff = np.zeros((n_pert, len(mil)), dtype=np.complex128)
    for i in range(n_pert):
        for k in range(len(mil)):
            if zero[k]:
                coeff[i, k] = rng.standard_normal()
            elif rep[k]:
                re = rng.standard_normal()
                im = rng.standard_normal()
                coeff[i, k] = re + 1j * im
        for k in range(len(mil)):
            if not rep[k] and not zero[k]:
                coeff[i, k] = np.conj(coeff[i, partner[k]])
        coeff[i] /= np.sqrt(np.sum(np.abs(coeff[i]) ** 2))
    dv_r = np.empty((n_pert, N, N, N))
    for i in range(n_pert):
        box = np.zeros((N, N, N), dtype=np.complex128)
        box[mil[:, 0] % N, mil[:, 1] % N, mil[:, 2] % N] = coeff[i]
        f = np.fft.ifftn(box) * (N ** 3)
        dv_r[i] = f.real
    return mil, coeff, dv_r
