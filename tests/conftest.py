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
