"""Several contexts in one process.  A kernel's limit on dynamic LDS is a
property of the kernel, not of a context: a context created after another,
with smaller tiles that still need more than 64 KB, must not lower the limit
below what the first one launches with.  Two FP64 cavities of 128 and 112
cells across sweep their finest level in bands whose tiles need about 81 and
71 KB of LDS (walls on all four sides); one outer cycle of the larger one,
run after the smaller one was created, equals the same cycle run before it
bit for bit."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _cavity(n):
    return wl.cavity(n=n, Kn=0.1, n_levels=2, quad=wl.QUAD_TRAPEZOID, nvel=4, vlo=-4.0, vhi=4.0,
                     precision="fp64")


def test_lds_limits_survive_a_later_context():
    from paper_1704_03151_amd import Solver
    big, small = _cavity(128), _cavity(112)
    print("[contexts] cavity128 alone", flush=True)
    a = Solver(big, precision="fp64")
    a.init_macro(big.init)
    rc, n, _ = a.iterate(1, tol=0.0)
    assert n == 1
    ref = a.get_f(np.float64)
    a.close()
    print("[contexts] cavity128 after cavity112 was created", flush=True)
    a = Solver(big, precision="fp64")
    b = Solver(small, precision="fp64")
    a.init_macro(big.init)
    rc, n, _ = a.iterate(1, tol=0.0)
    assert n == 1
    out = a.get_f(np.float64)
    b.init_macro(small.init)
    rc, n, _ = b.iterate(1, tol=0.0)
    assert n == 1
    a.close()
    b.close()
    assert np.array_equal(out, ref)
