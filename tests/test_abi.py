"""The C-ABI library loads and exports every symbol its header declares, and
its host-side setup (quadrature rules, argument checks) agrees with the
oracle.  No GPU calls."""
import os
import re

import numpy as np
import pytest

from oracle import quadrature as oq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    with open(os.path.join(ROOT, "include", "miugks.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(miugks_[A-Za-z_]+)\s*\(", text)))


def test_header_constants_match_the_binding_and_the_inputs():
    """Every MIUGKS_ constant of the header has the value the Python binding
    and the case descriptions use."""
    import workloads as wl
    from paper_1704_03151_amd import _C
    with open(os.path.join(ROOT, "include", "miugks.h")) as fh:
        text = fh.read()
    consts = {k: int(v) for k, v in re.findall(r"#define MIUGKS_([A-Z0-9_]+) \(?(-?\d+)\)?", text)}
    for name in ("OK", "EINVAL", "ENOMEM", "EDEVICE", "EDIVERGED", "ENOTCONVERGED", "ESTATE", "FP64", "FP32F",
                 "QUAD_TRAPEZOID", "QUAD_SIMPSON38", "QUAD_GAUSS_HERMITE", "CYCLE_F", "LOAD_PRESSURE", "LOAD_SHEAR", "LOAD_HEAT",
                 "FACE_INTERIOR", "FACE_WALL", "FACE_FARFIELD", "FACE_OUTFLOW", "FACE_SYMMETRY"):
        assert consts[name] == getattr(_C, name), name
    for name in ("FACE_INTERIOR", "FACE_WALL", "FACE_FARFIELD", "FACE_OUTFLOW", "FACE_SYMMETRY", "CYCLE_F"):
        assert consts[name] == getattr(wl, name), name


def test_library_exports_every_declared_symbol():
    from paper_1704_03151_amd import _C
    names = _header_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(_C.lib, n), n
    assert set(names) == set(_C.EXPORTS)


@pytest.mark.parametrize("kind,name,n,lo,hi", [(0, "trapezoid", 16, -4, 4), (1, "simpson38", 40, -5, 5),
                                               (1, "simpson38", 100, -15, 15), (2, "gauss_hermite", 28, 0, 0),
                                               (2, "gauss_hermite", 7, 0, 0)])
def test_library_quadrature_matches_oracle(kind, name, n, lo, hi):
    from paper_1704_03151_amd import _C
    x, w = _C.quadrature(kind, n, lo, hi)
    xo, wo = oq.rule_1d(name, n, lo, hi)
    assert np.allclose(x, xo, rtol=0, atol=1e-13)
    assert np.allclose(w, wo, rtol=1e-12, atol=0)


def test_quadrature_rejects_bad_arguments():
    from paper_1704_03151_amd import _C
    with pytest.raises(_C.MiugksError):
        _C.quadrature(1, 11, -1, 1)          # (n-1) % 3 != 0
    with pytest.raises(_C.MiugksError):
        _C.quadrature(7, 10, -1, 1)          # unknown rule
    with pytest.raises(_C.MiugksError):
        _C.quadrature(0, 10, 1, -1)          # empty range


def test_allocator_pair_must_be_complete():
    """miugks_set_allocator refuses an allocator without its free (and the
    reverse) and accepts restoring hipMalloc / hipFree.  No GPU calls."""
    from paper_1704_03151_amd import _C
    alloc = _C.ALLOC_FN(lambda n, u: None)
    assert _C.lib.miugks_set_allocator(alloc, _C.FREE_FN(), None) == _C.EINVAL
    assert _C.lib.miugks_set_allocator(_C.ALLOC_FN(), _C.FREE_FN(lambda p, u: None), None) == _C.EINVAL
    assert _C.lib.miugks_set_allocator(_C.ALLOC_FN(), _C.FREE_FN(), None) == _C.OK
