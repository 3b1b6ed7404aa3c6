"""Preconditioners of the adjoint iteration, measured on the oracle (no GPU).

The adjoint solves (dr/df)^T lam = b by GMRES, right-preconditioned.  The
library's preconditioner is -A_d^-T, A_d the velocity-diagonal part of the
correction operator of Step 5 (Sec. II A 2: 1/tau, the upwind transport,
outflow ghosts; the diffuse-wall coupling across velocities left out), one
downwind-ordered sweep per velocity.  The alternative is the transposed CS
V-cycle, -B^T with B the oracle's CS V-cycle (Sec. II D) taken as a linear
map (applied to every unit vector), which approximates the full correction
operator's inverse, walls included.  On the dense tiny cavity at a converged
steady state, GMRES(30) to 1e-10 on the consistent system (dr/df)^T lam =
(dr/df)^T x counts:

    Kn 0.1:  sweep 43, transposed CS V-cycle 41, exact -A^-T 41, none 97
    Kn 2  :  sweep 23, transposed CS V-cycle 21, exact -A^-T 21, none 135

The V-cycle saves two steps out of 20-40 (5-9 %), while each application costs
a whole cycle (pre- and post-sweeps on every level, transfers, wall
densities) instead of one sweep, next to the adjoint product that dominates a
step.  The test holds these counts (the sweep within 15 % of the exact
transposed operator, the V-cycle no better than the exact operator), so the
choice of the single sweep rests on a measurement."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import workloads as wl
from oracle import adjoint as ad
from oracle import gas as gm
from oracle import sparse as osp
from oracle.cs import cs_cycle
from oracle.solver import Oracle


def _gmres_steps(M, b):
    steps = [0]

    def count(_):
        steps[0] += 1

    y, info = sla.gmres(M, b, rtol=1e-10, restart=30, maxiter=3000, callback=count, callback_type="pr_norm")
    assert info == 0
    assert np.linalg.norm(b - M @ y) <= 2e-10 * np.linalg.norm(b)
    return steps[0]


@pytest.mark.parametrize("Kn", [0.1, 2.0])
def test_transposed_cs_v_cycle_against_the_single_sweep(Kn):
    case = wl.cavity(n=4, Kn=Kn, n_levels=2, quad="gauss_hermite", nvel=6, vlo=0.0, vhi=0.0, mach=0.3,
                     precision="fp64")
    case.wall_y[0, :, 0] = 1.0 + np.random.default_rng(1704).uniform(-0.05, 0.05, 4)
    o = Oracle(case)
    ok, norms = o.iterate(400, tol=1e-8)
    assert ok, norms
    S = ad.Sensitivity(o)
    J = S.jacobian()
    n = J.shape[0]
    rho, U, V, lam = gm.primitive(o.W, o.gas.K)
    tau_inv = 1.0 / o.gas.tau(rho, lam)
    # the correction operator (no pseudo-time term), and its velocity-diagonal part
    A = osp.assemble(o.lev0, o.vel, o.gas.K_int, tau_inv).tocoo()
    per_plane = o.vel.n * o.lev0.nc
    same = (A.row // o.lev0.nc == A.col // o.lev0.nc)   # same plane and velocity
    A_d = sp.csr_matrix((A.data[same], (A.row[same], A.col[same])), shape=A.shape).toarray()
    A_full = A.toarray()
    assert A_full.shape == (n, n) and per_plane * 2 == n   # every cell is fluid: f's unknowns are A's
    # the CS V-cycle as a matrix: column j = CS(e_j)
    B = np.empty((n, n))
    tl = o.level_tau_inv(tau_inv)
    dz = [np.zeros(lev.nc) for lev in o.levels]
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        rG, rH = S.unpack(e)
        dG, dH = cs_cycle(o.cs_levels, o.levels, o.prolongs, 0, rG, rH, tl, dz, o.cs_params)
        B[:, j] = S.pack(dG, dH)
    b = J.T @ np.random.default_rng(7).standard_normal(n)
    steps = {
        "none": _gmres_steps(J.T, b),
        "sweep": _gmres_steps(J.T @ (-np.linalg.inv(A_d).T), b),
        "exact": _gmres_steps(J.T @ (-np.linalg.inv(A_full).T), b),
        "vcycle": _gmres_steps(J.T @ (-B.T), b),
    }
    print(f"[precond] Kn {Kn}: GMRES(30) steps to 1e-10 {steps}", flush=True)
    assert steps["sweep"] < 0.5 * steps["none"]
    assert steps["sweep"] <= 1.15 * steps["exact"]
    assert steps["vcycle"] >= steps["exact"]
