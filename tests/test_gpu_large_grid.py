"""Grids whose FP64 plane no longer fits in LDS, so the right-hand side, psi_v(r) and dn run
in the compact active-line layout: the large cell's grid (L=32 bohr, 30 Ry, 512 atoms: 91,047
PWs on 128^3, radices 16 x 8) with 32 bands and 4 fields, and a 108^3 cell (L=24, 38 Ry, 64
atoms: 54,795 PWs, radices 12 x 9) with 16 bands and 4 fields. Checked against the oracle one
pair at a time, with sampled solutions under the oracle's operator, and by properties that
hold at any size."""
import numpy as np
import pytest

from oracle import OracleCell, apply_chi0, project
from oracle.sternheimer import chi0_matrix, rel_l2, rhs

pytestmark = pytest.mark.gpu

CELLS = {"128": ("LARGE_GRID", 128, 91047, [(0, 0), (31, 0), (16, 2), (31, 3)], [(0, 1), (31, 3)]),
         "108": ("GRID108", 108, 54795, [(0, 0), (15, 0), (8, 2), (15, 3)], [(0, 1), (15, 3)])}


@pytest.fixture(scope="module", params=["128", "108"])
def large(request):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System, STERN_MIXED, STERN_FP64
    import synth.cells as cells
    from synth.inputs import load_workload
    name, n_grid, n_pw, pairs, singles = CELLS[request.param]
    wl = load_workload(getattr(cells, name))
    sp = wl["spec"]
    s = System(sp.L, sp.ecut, wl["pos"], sp.vloc_amp, sp.vloc_sigma, sp.kb_D, sp.kb_width)
    dev = torch.device("cuda:0")
    s.set_occupied(torch.from_numpy(np.ascontiguousarray(wl["psi"])).to(dev), torch.from_numpy(wl["eps"]).to(dev))
    dv = torch.from_numpy(wl["dv"]).to(dev)
    dn, info = s.apply_chi0(dv, tol=1e-8, samples=pairs, precision=STERN_MIXED)
    dn64, info64 = s.apply_chi0(dv, tol=1e-8, precision=STERN_FP64)
    cell = OracleCell(sp.L, sp.ecut, wl["pos"])
    psi = cell.take(wl["psi"], wl["miller"])
    yield dict(s=s, wl=wl, dv_t=dv, dn=dn.cpu().numpy(), info=info, dn64=dn64.cpu().numpy(), info64=info64,
               cell=cell, psi=psi, n_grid=n_grid, n_pw=n_pw, pairs=pairs, singles=singles,
               n_solves=wl["psi"].shape[0] * wl["dv"].shape[0])
    s.close()


def test_grid_and_convergence(large):
    s, info, info64 = large["s"], large["info"], large["info64"]
    assert s.fft_n == large["n_grid"] and s.n_pw == large["n_pw"]
    for i in (info, info64):
        assert i["n_solves"] == i["n_converged"] == large["n_solves"] and i["max_true_resid"] <= 1e-8


def test_sampled_solutions_satisfy_oracle_equation(large):
    cell, psi, wl = large["cell"], large["psi"], large["wl"]
    x = cell.take(large["info"]["samples"], wl["miller"])
    bands = [v for v, _ in large["pairs"]]
    perts = [i for _, i in large["pairs"]]
    b = rhs(cell, psi, wl["dv"], bands, perts)
    px = project(psi, x)
    ax = project(psi, cell.h_apply(px) - wl["eps"][bands][:, None] * px)
    res = np.linalg.norm(b - ax, axis=1) / np.linalg.norm(b, axis=1)
    assert res.max() <= 1.05e-8, res


@pytest.mark.parametrize("which", [0, 1])
def test_single_pair_dn_matches_oracle(large, which):
    """The FP64 path on one (band, field) pair at 1e-12 gives the oracle's dn of that pair:
    right-hand side, solve and dn accumulation of the compact kernels end to end."""
    from paper_2607_14025_amd import STERN_FP64
    cell, psi, wl = large["cell"], large["psi"], large["wl"]
    v, i = large["singles"][which]
    dn, info = large["s"].apply_chi0(large["dv_t"][i:i + 1].contiguous(), tol=1e-12, precision=STERN_FP64,
                                     band_range=(v, v + 1))
    assert info["n_converged"] == 1
    ref = apply_chi0(cell, psi, wl["eps"], wl["dv"], tol=1e-12, bands=[v], perts=[i])
    err = rel_l2(dn.cpu().numpy() if hasattr(dn, "cpu") else dn, ref["dn"][i:i + 1])
    assert err.max() < 1e-9, err


def test_mixed_matches_fp64_and_chi0_properties(large):
    dn, dn64, cell, wl = large["dn"], large["dn64"], large["cell"], large["wl"]
    assert rel_l2(dn, dn64).max() < 1e-6
    M = chi0_matrix(cell, wl["dv"], dn64)
    nrm = np.linalg.norm(M)
    assert np.linalg.norm(M - M.T) / nrm < 1e-6
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).max() <= 1e-6 * nrm
    tot = np.abs(dn64.sum(axis=(1, 2, 3))) / np.abs(dn64).sum(axis=(1, 2, 3))
    assert tot.max() < 1e-12
