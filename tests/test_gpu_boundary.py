"""The C ABI's system-level entry points that carry no arithmetic of the method: the Miller
order a system exports, and the caller-supplied device allocator of stern_runtime."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_get_miller_is_the_canonical_order(tiny_system):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System
    from paper_2607_14025_amd.stern import basis_info
    from oracle import sphere_miller
    sp = tiny_system["spec"]
    s = System(sp.L, sp.ecut, tiny_system["gs"]["pos"])
    mil = s.miller()
    s.close()
    _, _, bi = basis_info(sp.L, sp.ecut)
    assert np.array_equal(mil, bi)
    assert np.array_equal(mil, sphere_miller(sp.L, sp.ecut))        # the oracle's own enumeration
    assert np.array_equal(mil, tiny_system["gs"]["miller"])          # the generator's order of psi


def test_torch_allocator_gives_the_same_results(tiny_system):
    """A system whose buffers come from torch's caching allocator (stern_runtime.dev_alloc) computes
    bitwise what a hipMalloc system computes, and returns every buffer on stern_free."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2607_14025_amd import System, STERN_MIXED
    t = tiny_system
    sp, gs = t["spec"], t["gs"]
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    a = System(sp.L, sp.ecut, gs["pos"], torch_allocator=True)
    a.set_occupied(gs["psi"], gs["eps"])
    held = torch.cuda.memory_allocated() - before
    assert held > 1 << 20  # the system's buffers are torch's
    b = System(sp.L, sp.ecut, gs["pos"])
    b.set_occupied(gs["psi"], gs["eps"])
    for prec in (0, STERN_MIXED):
        da, ia = a.apply_chi0(t["dv"], tol=1e-10, precision=prec)
        db, ib = b.apply_chi0(t["dv"], tol=1e-10, precision=prec)
        assert ia["n_converged"] == ia["n_solves"] == 128
        assert np.array_equal(da, db)
        assert np.array_equal(ia["iters"], ib["iters"])
    a.close()
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
