"""MI355X (gfx950) implementation of the multigrid implicit unified gas-kinetic
scheme (MIUGKS) of Zhu, Zhong & Xu (arXiv:1704.03151).

The solver lives in the HIP library libmiugks.so (C ABI in include/miugks.h);
`Solver` wraps one problem context; `autograd.steady_wall_load` makes a
steady wall load a differentiable function of wall temperatures (backward by
the adjoint).  Importing the package loads the library and fails loudly when
it has not been built.
"""
from . import _C  # noqa: F401  (loads libmiugks.so)
from .solver import Solver, use_torch_allocator  # noqa: F401

__all__ = ["Solver", "use_torch_allocator"]
