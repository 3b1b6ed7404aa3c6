"""A steady wall load as a differentiable function of wall temperatures.

`steady_wall_load(solver, Tw, ...)` sets the temperatures of the given mesh
faces, converges the steady state on the GPU and returns the objective
J = sum S load over the given wall sides as a torch scalar; its backward pass
calls the library's adjoint (dJ/dTw at fixed mass in a closed domain), so
J.backward() or torch.autograd.grad give the gradient over all faces for the
cost of one adjoint solve.  Forward keeps its temperatures and converged
distribution (on the GPU); when the solver has been used since (another
forward, a line search), backward puts that state back before the adjoint,
so every J is differentiated at its own steady state.  Argument marshalling
only: the solves run in libmiugks.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _C


class _SteadyWallLoad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Tw, solver, kind, walls, faces, max_cycles, tol, adj_tol, adj_iter):
        T = Tw.detach().to("cpu", torch.float64).numpy()
        solver.set_wall_T(faces, T)
        rc, n, res = solver.iterate(max_cycles, tol)
        if rc != _C.OK:
            raise _C.MiugksError(rc, f"steady state not reached in {max_cycles} cycles (residual {res.max():.3e})")
        ctx.args = (solver, kind, walls, faces, adj_tol, adj_iter)
        ctx.device = Tw.device
        # the state this J belongs to
        ctx.Tw = T.copy()
        ctx.f = solver.get_f(out=torch.empty(solver.fshape, dtype=torch.float64, device="cuda"))
        ctx.version = solver.state_version
        return torch.tensor(solver.objective(kind, walls), dtype=torch.float64, device=Tw.device)

    @staticmethod
    def backward(ctx, gJ):
        solver, kind, walls, faces, adj_tol, adj_iter = ctx.args
        if solver.state_version != ctx.version:
            solver.set_wall_T(faces, ctx.Tw)
            solver.set_f(ctx.f)
        st, g, iters, rel = solver.adjoint(kind, walls, faces, tol=adj_tol, max_iter=adj_iter)
        ctx.version = solver.state_version
        if st != _C.OK:
            raise _C.MiugksError(st, f"adjoint not converged after {iters} corrections (residual {rel:.3e})")
        grad = torch.as_tensor(np.asarray(g), dtype=torch.float64, device=ctx.device) * gJ
        return grad, None, None, None, None, None, None, None, None


def steady_wall_load(solver, Tw, kind, walls, faces, max_cycles=1000, tol=1e-12, adj_tol=1e-8, adj_iter=5000):
    """J(Tw) of the converged steady state (see the module docstring); the
    solver must be an FP64 context."""
    return _SteadyWallLoad.apply(Tw, solver, int(kind), list(map(int, walls)), list(map(int, faces)),
                                 int(max_cycles), float(tol), float(adj_tol), int(adj_iter))
