"""miugks_get_f_noalloc (the allocation-free copy of the distribution)
against miugks_get_f, through the C ABI: two calls in a row, the second on a
smaller context; a conversion larger than the library's fixed device array
(several pieces), a conversion smaller than it, and the same-dtype copy.
With a caller-supplied counting allocator the entry point calls it never,
while miugks_get_f to a host buffer does (so the count is not vacuous)."""
import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _counting_allocator():
    """Allocator callbacks that forward to torch's caching allocator and count calls."""
    import torch
    from paper_1704_03151_amd import _C
    count = {"alloc": 0}

    def alloc(nbytes, user):
        count["alloc"] += 1
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:
            return None

    def free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    return count, (_C.ALLOC_FN(alloc), _C.FREE_FN(free))


def test_get_f_noalloc_matches_get_f_on_two_contexts():
    import torch
    from paper_1704_03151_amd import Solver, _C
    count, pair = _counting_allocator()
    assert _C.lib.miugks_set_allocator(pair[0], pair[1], None) == 0
    try:
        # 64x64 x 784 in FP32-f: 25.7 MB as FP64 is more than the 16 MiB array
        big = Solver(wl.config2(), precision="fp32f")
        # 16x16 x 256 in FP64: the second, smaller call
        small = Solver(wl.config1(), precision="fp64")
    finally:
        _C.lib.miugks_set_allocator(_C.ALLOC_FN(), _C.FREE_FN(), None)
    print("[noalloc] contexts created", flush=True)
    big.iterate(3, tol=0.0)
    small.iterate(3, tol=0.0)
    torch.cuda.synchronize()
    for s, dts in ((big, (np.float64, np.float32)), (small, (np.float32, np.float64))):
        for dt in dts:
            before = count["alloc"]
            got = s.get_f_noalloc(dt)
            assert count["alloc"] == before, "the allocation-free entry point called the allocator"
            want = s.get_f(dt)
            assert count["alloc"] > before or dt == s.dtype, "get_f to a host buffer stages through an allocation"
            assert got.dtype == want.dtype and np.array_equal(got, want), (s.case.name, dt)
            print(f"[noalloc] {s.case.name} as {np.dtype(dt).name}: {got.nbytes / 2**20:.1f} MiB equal", flush=True)
    # the conversion is exact from float to double, and rounds double to float
    f32 = big.get_f_noalloc(np.float32)
    assert np.array_equal(big.get_f_noalloc(np.float64), f32.astype(np.float64))
    assert np.array_equal(small.get_f_noalloc(np.float32), small.get_f_noalloc(np.float64).astype(np.float32))
    # bad arguments are refused
    assert _C.lib.miugks_get_f_noalloc(small.h, None, _C.FP64) == _C.EINVAL
    buf = np.zeros(4)
    assert _C.lib.miugks_get_f_noalloc(small.h, buf.ctypes.data_as(ctypes.c_void_p), 7) == _C.EINVAL
    big.close()
    small.close()
