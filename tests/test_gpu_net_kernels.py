"""The learned net's kernels against the NumPy reference (oracle/net.py), through the C ABI:
one stern_model_fit_step gives the forward output, the per-solve loss, the weight and bias
gradients of all three layers (which pass through the data-gradient convolution with
flipped weights and the ReLU masks) and the Adam update."""
import numpy as np
import pytest

from oracle import net

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("Nc", [12, 10])
def test_fit_step_matches_numpy_reference(Nc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import Model
    rng = np.random.default_rng(100 + Nc)
    n = 3
    m = Model(seed=3)
    w0 = np.zeros(Model.num_params(), dtype=np.float32)
    for l, fan in enumerate((27 * 5, 27 * 16, 27 * 16)):
        blk = slice(l * net.LAYER, (l + 1) * net.LAYER)
        w0[blk] = (rng.standard_normal(net.LAYER) * np.sqrt(2.0 / fan)).astype(np.float32)
    m.set_weights(w0)
    inp = rng.standard_normal((n, Nc, Nc, Nc, 5)).astype(np.float32)
    tgt = rng.standard_normal((n, Nc, Nc, Nc, 2)).astype(np.float32)
    lr = 1e-3
    out, loss, grad = m.fit_step(inp, tgt, lr)
    w1 = m.get_weights()
    m.close()
    ro, rl, rg = net.fit_step(w0, inp.astype(np.float64), tgt.astype(np.float64))
    print(f"Nc={Nc}: out {_rel(out, ro):.2e}, loss {_rel(loss, rl):.2e}, "
          + ", ".join(f"grad layer {l} {_rel(grad[l * net.LAYER:(l + 1) * net.LAYER], rg[l * net.LAYER:(l + 1) * net.LAYER]):.2e}"
                      for l in range(3)))
    # The BF16 activations between layers are rounded from FP32 sums taken in another order than
    # the reference's float64 ones: a value within ~1e-7 of a rounding midpoint (a few per 1e5)
    # lands on the other side and differs by one BF16 unit (2^-8 relative), which moves the
    # outputs of its 27 neighbours by ~1e-3 and the relative L2 of the whole by ~1e-4. A wrong
    # tap, flip, transpose or channel gives O(1) errors.
    assert _rel(out, ro) < 2e-3
    assert _rel(loss, rl) < 2e-4
    for l in range(3):
        blk = slice(l * net.LAYER, (l + 1) * net.LAYER)
        assert _rel(grad[blk], rg[blk]) < 2e-3, l
        bias = slice((l + 1) * net.LAYER - 16, (l + 1) * net.LAYER)
        assert _rel(grad[bias], rg[bias]) < 2e-3, l
    # Adam from zero moments at step 1 with the gradient averaged over the n solves
    want = net.adam_update(w0[:3 * net.LAYER].astype(np.float64), grad.astype(np.float64), lr, 1, 1.0 / n)
    assert np.allclose(w1[:3 * net.LAYER], want, rtol=0, atol=1e-6 * lr + 1e-7 * np.abs(want).max())
    assert np.array_equal(w1[3 * net.LAYER:], w0[3 * net.LAYER:])  # the head is not part of this step


def test_fit_step_rejects_bad_arguments():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import Model
    from paper_2607_14025_amd.stern import SternError
    m = Model(seed=3)
    with pytest.raises(ValueError):
        m.fit_step(np.zeros((1, 4, 4, 4, 3)), np.zeros((1, 4, 4, 4, 2)), 1e-3)
    with pytest.raises(SternError):
        m.fit_step(np.zeros((1, 4, 4, 4, 5)), np.zeros((1, 4, 4, 4, 2)), -1.0)
    m.close()
