"""The large-cell eigensolver of the input generator (Chebyshev-filtered subspace iteration,
synth/ground_gpu.py), run on the host with the generator's own H: its Ritz values equal the
dense eigenvalues and its residuals meet the tolerance (CPU only)."""
import numpy as np

from synth.cells import TINY, place_atoms
from synth.ground import ModelH
from synth.ground_gpu import chebyshev_eigs


def test_chebyshev_eigs_matches_dense_eigh():
    import torch
    H = ModelH(TINY, place_atoms(TINY))
    e = np.linalg.eigvalsh(H.dense())

    def app(Y, sh):
        out = H.apply(Y.numpy())
        if sh is not None:
            out -= np.asarray(sh)[:, None] * Y.numpy()
        return torch.from_numpy(out)

    gen = torch.Generator().manual_seed(7)
    X = torch.randn(24, H.npw, dtype=torch.complex128, generator=gen) / (1 + torch.from_numpy(0.5 * H.g2))[None, :]
    th, X, res, passes = chebyshev_eigs(app, X, 17, 1e-10, degree=12, gen=gen)
    assert res.max() <= 1e-10
    assert np.abs(th[:17] - e[:17]).max() < 1e-12
    G = (X.conj() @ X.T).numpy()
    assert np.abs(G - np.eye(len(G))).max() < 1e-13
