"""Device memory from PyTorch's caching allocator through fds_set_allocator:
a factor built with the hook holds its buffers in PyTorch (the library's own
cache stays empty), gives bitwise the same solution as one built on the
library's cache, and hands its buffers back to PyTorch when destroyed.  The
hook is refused while blocks of the other allocator are live."""
import gc

import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case():
    cfg = sy.config_small()
    return cfg, dict(leaf=cfg["leaf"])


def test_torch_allocator_hook():
    import paper_2411_18026_amd as fds
    fds.load()
    cfg, kw = _case()
    args = (cfg["curves"], cfg["omega"], cfg["lam"], cfg["mu"], cfg["rho"], cfg["tol"])
    F = fds.Factor(*args, **kw)
    rhs = F.rhs_plane([0, 1], [0.0, 0.7])
    x_ref = F.solve(rhs)
    # refused while the library's blocks are live
    with pytest.raises(fds.FdsError) as e:
        fds.use_torch_allocator()
    assert e.value.code == 1
    del F
    gc.collect()
    torch.cuda.synchronize()
    fds.use_torch_allocator()
    try:
        assert fds.cached_bytes() == 0
        before = torch.cuda.memory_allocated()
        F = fds.Factor(*args, **kw)
        held = torch.cuda.memory_allocated() - before
        assert held >= F.stats()["factor_bytes"]
        x = F.solve(rhs)
        assert torch.equal(x, x_ref)
        assert fds.cached_bytes() == 0
        del F
        gc.collect()
        torch.cuda.synchronize()
        # everything but the solution tensor went back to PyTorch
        assert torch.cuda.memory_allocated() - before <= x.numel() * x.element_size() + 512
    finally:
        gc.collect()
        fds.use_library_allocator()
    # and the library's cache works again afterwards
    F = fds.Factor(*args, **kw)
    assert torch.equal(F.solve(rhs), x_ref)
