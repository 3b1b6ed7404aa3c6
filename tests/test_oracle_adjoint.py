"""Pins of the oracle's wall loads, objective and steady-state sensitivities
(no GPU): closed forms of a gas at rest, the momentum and energy balances of
a steady cavity, central differences of the residual, and central
differences of the objective over converged FP64 steady states."""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as ad
from oracle.solver import Oracle
from _parity import tiny_open_plate

N = 4


def _tiny_cavity(**kw):
    """4 x 4 cavity, 8 x 8 Gauss-Hermite velocities, Kn 2, lid Mach 0.3, two
    levels, seeded bottom-wall temperatures 1 + U(-0.05, 0.05); FP64 runs of
    it reach 2e-13."""
    case = wl.cavity(n=N, Kn=kw.pop("Kn", 2.0), n_levels=2, quad="gauss_hermite", nvel=8, vlo=0.0, vhi=0.0,
                     mach=0.3, precision="fp64", **kw)
    rng = np.random.default_rng(1704)
    case.wall_y[0, :, 0] = 1.0 + rng.uniform(-0.05, 0.05, N)
    return case


@pytest.fixture(scope="module")
def steady():
    case = _tiny_cavity()
    o = Oracle(case)
    ok, norms = o.iterate(200, tol=2e-13)
    assert ok, norms
    return case, o


def _lid(o):
    lev = o.lev0
    return [i for i, j in enumerate(ad.wall_list(lev)) if lev.bside[j] == 3]


def test_wall_loads_of_a_gas_at_rest():
    """A gas at rest at the wall temperature presses on every wall with
    p = rho T / 2 (nondimensional, 2 R T0 = 1) and carries no shear or heat
    flux (quadrature on a wide grid)."""
    case = wl.cavity(n=4, Kn=1.0, n_levels=1, quad="trapezoid", nvel=64, vlo=-9.0, vhi=9.0, mach=0.0,
                     precision="fp64")
    o = Oracle(case)
    ld = ad.wall_loads(o.G, o.H, o.lev0, o.vel, o.gas, case.farfield)
    assert ld.shape[1] == 16
    assert np.allclose(ld[0], 0.5, rtol=0, atol=1e-12)
    assert np.allclose(ld[1:3], 0.0, atol=1e-12)
    assert np.allclose(ld[3], 0.25)


def test_steady_wall_loads_balance_momentum_and_energy(steady):
    """In a steady closed cavity the walls take all the x-momentum and energy
    the gas exchanges: sum over walls of S (shear on the horizontal walls,
    +-pressure on the vertical ones) vanishes, and so does sum S (q + U_w tau)
    (the heat flux in each wall's frame plus the lid's work)."""
    case, o = steady
    lev = o.lev0
    ld = ad.wall_loads(o.G, o.H, lev, o.vel, o.gas, case.farfield)
    js = ad.wall_list(lev)
    side = lev.bside[js]
    cell = lev.bcell[js]
    sign = np.where(side % 2 == 0, -1.0, 1.0)
    mx = np.where(side < 2, sign * ld[0], ld[1])
    assert abs(np.sum(ld[3] * mx)) < 1e-11
    Uw = lev.wall[side, cell, 1]
    assert np.max(np.abs(Uw[side == 3] - case.wall_y[N, 0, 1])) == 0.0 and np.all(Uw[side != 3] == 0.0)
    assert abs(np.sum(ld[3] * (ld[2] + Uw * ld[1]))) < 1e-11
    # and the lid drags the gas along: the gas pulls the lid backwards
    assert np.all(ld[1][side == 3] < 0)


def test_complex_step_jacobian_matches_central_differences(steady):
    case, o = steady
    S = ad.Sensitivity(o)
    J = S.jacobian()
    x0 = S.pack(o.G, o.H)
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.standard_normal(x0.size) * np.abs(x0)
        e = 1e-6
        fd = (S.residual(x0 + e * d) - S.residual(x0 - e * d)) / (2 * e)
        assert np.max(np.abs(J @ d - fd)) < 1e-7 * np.max(np.abs(fd))
    # mass: the residual of a closed cavity has the mass row as a left null
    # vector, so the steady states form a one-parameter (mass) family
    assert np.max(np.abs(S.mass_row() @ J)) < 1e-11 * np.max(np.abs(J))


def test_objective_gradient_matches_steady_state_differences(steady):
    """dJ/dTw of the lid shear with respect to two bottom-face temperatures
    matches central differences (h = 2e-5) of J over FP64 steady states
    converged to 2e-13 at the same mass.  The limiter is only piecewise smooth:
    from this state a van Leer branch switches between +1e-4 and +3e-4 on the
    first face (its forward and backward differences part there), so the step
    stays below it; the convergence error over 2h is then about 1e-9."""
    case, o = steady
    S = ad.Sensitivity(o)
    lid = _lid(o)
    nfx = (N + 1) * N
    faces = [nfx + 0, nfx + 2]
    g = S.gradient(ad.LOAD_SHEAR, lid, faces)
    h = 2e-5
    fd = []
    for f in faces:
        vals = []
        for sgn in (1.0, -1.0):
            c2 = case.with_(wall_y=case.wall_y.copy())
            c2.wall_y[0, f - nfx, 0] += sgn * h
            o2 = Oracle(c2)
            o2.set_f(o.G, o.H)
            ok, norms = o2.iterate(200, tol=2e-13)
            assert ok, norms
            vals.append(ad.objective(o2.G, o2.H, o2.lev0, o2.vel, o2.gas, c2.farfield, ad.LOAD_SHEAR, lid))
        fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    assert np.all(np.abs(g - fd) <= 1e-4 * np.maximum(np.abs(fd), 1e-3 * np.max(np.abs(fd)))), (g, fd)
    # a face of the lid itself also moves J directly (the partial at fixed f)
    direct = S.dJ_dT(ad.LOAD_SHEAR, lid, [nfx + N * N + 1])
    assert abs(direct[0]) > 0


def test_open_domain_gradient_matches_steady_state_differences():
    """Open domain (plate in a farfield, no mass constraint, so the tangent is
    a plain solve): dJ/dTw of the plate's pressure, shear and heat loads,
    summed over both of its sides, with respect to the plate face's one
    temperature, against central differences (h = 2e-5) of J over FP64
    steady states converged to 2e-13."""
    case, face = tiny_open_plate()
    o = Oracle(case)
    ok, norms = o.iterate(200, tol=2e-13)
    assert ok and not o.closed, norms
    S = ad.Sensitivity(o)
    walls = list(range(len(ad.wall_list(o.lev0))))
    assert len(walls) == 2
    T = S.tangent(S.jacobian(), S.dr_dT([face]))
    kinds = (ad.LOAD_PRESSURE, ad.LOAD_SHEAR, ad.LOAD_HEAT)
    g = np.array([(S.dJ_df(k, walls) @ T + S.dJ_dT(k, walls, [face]))[0] for k in kinds])
    h = 2e-5
    vals = []
    for sgn in (1.0, -1.0):
        c2 = case.with_(wall_y=case.wall_y.copy())
        j, i = divmod(face - (case.nx + 1) * case.ny, case.nx)
        c2.wall_y[j, i, 0] += sgn * h
        o2 = Oracle(c2)
        o2.set_f(o.G, o.H)
        ok, norms = o2.iterate(300, tol=2e-13)
        assert ok, norms
        vals.append([ad.objective(o2.G, o2.H, o2.lev0, o2.vel, o2.gas, c2.farfield, k, walls) for k in kinds])
    fd = (np.array(vals[0]) - np.array(vals[1])) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-5 * np.max(np.abs(fd)), (g, fd)
