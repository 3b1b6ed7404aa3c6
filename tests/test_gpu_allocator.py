"""A context whose device memory comes from PyTorch's caching allocator
(miugks_set_allocator through use_torch_allocator) computes exactly what a
hipMalloc-backed one does, and hands its memory back when closed."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def test_torch_caching_allocator_backs_a_context():
    import torch
    from paper_1704_03151_amd import Solver, use_torch_allocator
    case = wl.config1()
    print("[alloc] cavity16: torch caching allocator", flush=True)
    ref = Solver(case, precision="fp64")
    ref.init_macro(case.init)
    ref.iterate(3, tol=0.0)
    want = ref.macro()
    ref.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    assert use_torch_allocator(True) == 0
    try:
        s = Solver(case, precision="fp64")
    finally:
        use_torch_allocator(False)
    held = torch.cuda.memory_allocated() - before
    assert held > 2 * 8 * case.n_vel * case.n_cells, held   # at least f in torch's pool
    s.init_macro(case.init)
    s.iterate(3, tol=0.0)
    got = s.macro()
    for k in want:
        assert np.array_equal(got[k], want[k]), k
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
