import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def tiny_system():
    """Tiny cell (L=10 bohr, 8 atoms, 10 Ry): ground state, fields and the oracle cell."""
    import numpy as np
    from synth.cells import TINY, random_dv
    from synth.ground import ground_state
    from oracle import OracleCell
    gs = ground_state(TINY)
    sp = gs["spec"]
    cell = OracleCell(sp.L, sp.ecut, gs["pos"])
    _, coeff, dv = random_dv(sp)
    psi = cell.take(gs["psi"], gs["miller"])
    return dict(gs=gs, spec=sp, cell=cell, dv=dv, dv_coeff=coeff, psi=psi, eps=gs["eps"])


@pytest.fixture(scope="session")
def large_cell():
    """The large cell at full size (L=32 bohr, 512 atoms, 30 Ry: 91,047 PWs, 128^3, 1,024 occupied
    bands), ground state from the GPU eigensolver of the input generator, the first 8 seeded
    fields (0-3 the solved ones, 4-7 for training), and the library system that made it."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from synth.cells import LARGE
    from synth.ground_gpu import large_workload
    wl = large_workload(LARGE, n_pert=8)
    print(f"large cell ground state: {wl['passes']} passes, {wl['wall_s']:.1f} s, gap {wl['gap']:.2e} Ha, "
          f"max eigen-residual {wl['resid'].max():.2e}", flush=True)
    s = wl["system"]
    s.set_occupied(wl["psi"], torch.from_numpy(wl["eps"]).to(wl["psi"].device))
    yield wl
    s.close()
