"""Cached ground states of the workload cells (input preparation only).

The occupied states of the larger cells take minutes to generate on the host,
so they are written once to <repo>/inputs_cache/ and re-read afterwards. A
missing or stale cache entry is regenerated from the seeds."""
from __future__ import annotations

import os

import numpy as np

from .cells import CellSpec, random_dv
from .ground import ground_state

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "inputs_cache")
VERSION = 1


def _key(spec: CellSpec) -> str:
    return (f"{spec.name}_s{spec.system_id}_L{spec.L:.6f}_E{spec.ecut:g}_a{spec.n_atoms}_o{spec.n_occ}"
            f"_A{spec.vloc_amp:g}_S{spec.vloc_sigma:g}_D{spec.kb_D:g}_W{spec.kb_width:g}_v{VERSION}")


def load_ground_state(spec: CellSpec, verbose: bool = False) -> dict:
    path = os.path.join(CACHE, _key(spec) + ".npz")
    if os.path.exists(path):
        z = np.load(path)
        return dict(spec=spec.with_system(int(z["system_id"])), pos=z["pos"], miller=z["miller"], psi=z["psi"],
                    eps=z["eps"], eps_lumo=float(z["eps_lumo"]), gap=float(z["gap"]), resid=z["resid"], N=int(z["N"]))
    gs = ground_state(spec, verbose=verbose)
    os.makedirs(CACHE, exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, system_id=gs["spec"].system_id, pos=gs["pos"], miller=gs["miller"], psi=gs["psi"], eps=gs["eps"],
             eps_lumo=gs["eps_lumo"], gap=gs["gap"], resid=gs["resid"], N=gs["N"])
    os.replace(tmp, path)
    return gs


def load_workload(spec: CellSpec, n_pert: int | None = None, verbose: bool = False) -> dict:
    """Ground state plus the seeded perturbation fields of one cell."""
    gs = load_ground_state(spec, verbose=verbose)
    _, coeff, dv = random_dv(gs["spec"], n_pert=n_pert, N=gs["N"])
    gs = dict(gs)
    gs["dv"] = dv
    gs["dv_coeff"] = coeff
    return gs
