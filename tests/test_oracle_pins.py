"""Pins of the CPU oracle against facts fixed outside the oracle itself:
library routines, closed forms, exact integrals, printed values of the paper,
invariants and special cases.  No GPU."""
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import gas as gm
from oracle import flux as fx
from oracle import fas as fa
from oracle.cs import MicroLevel, cs_cycle
from oracle.mesh import Level, Prolongation, build_levels, restrict
from oracle.quadrature import VelocityGrid, gauss_hermite, simpson38, trapezoid
from oracle.solver import Oracle
from oracle.sparse import assemble
from _parity import free_molecular_closed_form

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- quadrature
def test_gauss_hermite_matches_numpy():
    for n in (4, 16, 28):
        u, w = gauss_hermite(n)
        x, wx = np.polynomial.hermite.hermgauss(n)
        assert np.allclose(u, x, atol=1e-13)
        assert np.allclose(w * np.exp(-u * u), wx, rtol=1e-11, atol=1e-300)


def test_gauss_hermite_exact_degree():
    n = 12
    u, w = gauss_hermite(n)
    wgh = w * np.exp(-u * u)
    for m in range(n):              # degree 2m <= 2n - 1
        exact = math.gamma(m + 0.5)
        assert abs(np.sum(wgh * u ** (2 * m)) - exact) <= 1e-12 * exact


def test_simpson38_cubic_exact_and_trapezoid_linear_exact():
    u, w = simpson38(10, -1.0, 2.0)
    for p in range(4):
        assert abs(np.sum(w * u ** p) - (2.0 ** (p + 1) - (-1.0) ** (p + 1)) / (p + 1)) < 1e-13
    u, w = trapezoid(7, -1.0, 2.0)
    assert abs(np.sum(w * (3 * u + 1)) - (1.5 * 4 + 2 - 1.5 - (-1))) < 1e-13


@pytest.mark.parametrize("kind,n,lo,hi", [("trapezoid", 48, -8, 8), ("gauss_hermite", 28, 0, 0),
                                          ("simpson38", 100, -8, 8)])
def test_maxwellian_moments(kind, n, lo, hi):
    vel = VelocityGrid(kind, n, n, lo, hi)
    rho, U, V, T = 1.3, 0.2, -0.1, 1.1
    G, H = gm.maxwellian(rho, U, V, 1.0 / T, vel.u, vel.v, 1)
    W = gm.moments(G, H, vel)
    exact = gm.conservative(rho, U, V, 1.0 / T, 3)
    assert np.allclose(W, exact, rtol=1e-10, atol=1e-12)
    # analytic energy: rho |U|^2 / 2 + 3 rho T / 4 for K = 3 in units R T0 = 1/2
    assert abs(exact[3] - (0.5 * rho * (U * U + V * V) + 0.75 * rho * T)) < 1e-15


# --------------------------------------------------------------------------- gas model
def test_mu_ref_hard_sphere_limit():
    # hard-sphere mean free path: mu = 5 sqrt(pi) rho lambda sqrt(2RT) / 16
    assert abs(gm.mu_ref_vhs(1.0, 0.5) - 5.0 * math.sqrt(math.pi) / 16.0) < 1e-15


def _shakhov_by_integration(rho, U, V, lam, q, Pr, K, cx, cy):
    """G and H of the Shakhov-type distribution over 2 + K degrees of
    freedom, by Gauss-Hermite integration over the K extra components xi:
    f = g (1 + (1 - Pr) (c.q) / ((N + 2) p R T) (s / (R T) - (N + 2))),
    s = |c|^2 + |xi|^2, N = 2 + K, R T = 1 / (2 lam), p = rho R T."""
    x, wx = np.polynomial.hermite.hermgauss(24)
    z = x / math.sqrt(lam)                        # weight exp(-lam z^2) per component
    wz = wx / math.sqrt(lam)
    grids = np.meshgrid(*([z] * K), indexing="ij")
    wts = np.ones_like(grids[0])
    for wk in np.meshgrid(*([wz] * K), indexing="ij"):
        wts = wts * wk
    xi2 = sum(gk * gk for gk in grids)
    N = 2 + K
    RT = 0.5 / lam
    p = rho * RT
    g = rho * (lam / math.pi) ** (N / 2) * np.exp(-lam * (cx * cx + cy * cy))
    fac = 1 + (1 - Pr) * (cx * q[0] + cy * q[1]) / ((N + 2) * p * RT) * ((cx * cx + cy * cy + xi2) / RT - (N + 2))
    return float(np.sum(wts * g * fac)), float(np.sum(wts * g * fac * xi2))


@pytest.mark.parametrize("K", [1, 3])
def test_shakhov_reduction_and_heat_flux(K):
    """Reduced Shakhov pair = integral of the Shakhov factor over 2 + K_int
    degrees of freedom; its discrete moments are the conservative variables
    and its heat flux is (1 - Pr) q (the correction conserves momentum for
    every K_int, not only for the monatomic K_int = 1)."""
    rho, U, V, T, Pr = 1.2, 0.3, -0.2, 0.9, 0.72
    lam = 1.0 / T
    q = np.array([0.05, -0.03])
    u, v = np.array([0.7, -0.4, 1.3]), np.array([0.2, 0.9, -1.1])
    Gs, Hs = gm.shakhov(rho, U, V, lam, q[0], q[1], u, v, K, Pr)
    for j in range(3):
        G, H = _shakhov_by_integration(rho, U, V, lam, q, Pr, K, u[j] - U, v[j] - V)
        assert abs(G - Gs[j]) < 1e-13 and abs(H - Hs[j]) < 1e-13, (K, j, G - Gs[j], H - Hs[j])
    vel = VelocityGrid("trapezoid", 64, 64, -9, 9)
    G, H = gm.shakhov(rho, U, V, lam, q[0], q[1], vel.u, vel.v, K, Pr)
    W = gm.moments(G, H, vel)
    assert np.allclose(W, gm.conservative(rho, U, V, lam, 2 + K), atol=1e-12)
    qq = gm.heat_flux(G, H, vel, U, V)
    assert np.allclose(qq, (1 - Pr) * q, atol=1e-12)


# --------------------------------------------------------------------------- flux pieces
def test_van_leer_values():
    assert fx.van_leer(np.array(2.0), np.array(2.0)) == 2.0
    assert fx.van_leer(np.array(1.0), np.array(3.0)) == 1.5           # harmonic mean
    assert fx.van_leer(np.array(1.0), np.array(-3.0)) == 0.0          # extremum
    assert fx.van_leer(np.array(0.0), np.array(0.0)) == 0.0


def test_micro_slope_round_trip():
    """<abar psi g0> over (u, v, xi) reproduces rho0 b (closed-form inverse)."""
    rho, U, V, lam, K_int = 1.1, 0.25, -0.15, 1.3, 1
    b = np.array([0.3, -0.2, 0.4, 0.1])
    a = fx.micro_slope(b, U, V, lam, K_int + 2)
    vel = VelocityGrid("trapezoid", 80, 80, -8, 8)
    G0, H0 = gm.maxwellian(rho, U, V, lam, vel.u, vel.v, K_int)
    Gs, Hs = fx.slope_times_g0(a, G0, H0, vel.u, vel.v, lam, K_int)
    assert np.allclose(gm.moments(Gs, Hs, vel), rho * b, atol=1e-12)


def test_time_coefficients_are_the_time_integrals():
    """q1..q5 against adaptive quadrature of the time factors, each factor
    evaluated in 40-digit decimal arithmetic so the reference does not cancel."""
    import decimal
    ctx = decimal.Context(prec=40)
    D = decimal.Decimal

    def factor(kind, t, tau):
        t, tau = D(repr(t)), D(repr(tau))
        e = ctx.exp(-t / tau)
        val = {1: 1 - e, 2: (t + tau) * e - tau, 3: t - tau + tau * e, 4: e, 5: -t * e}[kind]
        return float(val)

    for dt, tau in [(0.01, 0.3), (0.5, 0.05), (1e-3, 10.0), (0.2, 0.39), (0.2, 0.41), (1e-3, 1e6)]:
        q = fx.time_coefficients(dt, tau)
        for kind, a in zip(range(1, 6), q):
            r = si.quad(lambda t: factor(kind, t, tau), 0, dt, epsabs=0.0, epsrel=1e-12, limit=200)[0]
            assert abs(a - r) <= 1e-9 * abs(r), (dt, tau, kind, a, r)


def test_time_coefficients_limits():
    dt = 0.02
    q = fx.time_coefficients(dt, 1e9)                    # free molecular
    assert abs(q[0]) < 1e-12 and abs(q[1]) < 1e-12 and abs(q[2]) < 1e-12
    assert abs(q[3] - dt) < 1e-12 and abs(q[4] + 0.5 * dt * dt) < 1e-12
    q = fx.time_coefficients(dt, 1e-9)                   # continuum
    assert abs(q[0] - dt) < 1e-8 and abs(q[3]) < 1e-8


def _small_cavity(n=6, nvel=8, vlo=-6.0, vhi=6.0, lid=0.0, **kw):
    c = wl.cavity(n=n, Kn=kw.pop("Kn", 1.0), n_levels=kw.pop("n_levels", 1), quad="trapezoid",
                  nvel=nvel, vlo=vlo, vhi=vhi, **kw)
    c.wall_y[n, :, 1] = lid
    return c


def test_uniform_maxwellian_is_a_fixed_point():
    """At rest with matching walls (wide velocity grid) the residuals vanish
    and one full cycle leaves f unchanged."""
    case = _small_cavity(n=8, nvel=48, vlo=-8, vhi=8, n_levels=2)
    o = Oracle(case)
    n = o.step1()
    assert np.max(n) < 1e-13
    G0 = o.G.copy()
    o.advance()
    assert np.max(np.abs(o.G - G0)) < 1e-13 * np.max(G0)


def test_uniform_freestream_is_a_fixed_point():
    case = wl.flat_plate(scale=8, quad="trapezoid", nu=48, nv=48, vlo=-8, vhi=8, n_levels=1)
    case.face_type_y[:] = np.where(case.face_type_y == wl.FACE_WALL, 0, case.face_type_y)
    o = Oracle(case)
    assert np.max(o.step1()) < 1e-12


def test_closed_box_flux_conserves_mass():
    """sum_i V_i R_i^rho = 0 to round-off for any state in a closed box
    (interior fluxes cancel; diffuse walls carry zero mass flux)."""
    case = _small_cavity(n=8, nvel=12, vlo=-5, vhi=5, lid=0.2, Kn=0.5)
    o = Oracle(case)
    o.init_macro(wl.random_macro(case, seed=3))
    pert = wl.random_perturbation(case, seed=4)
    o.set_f(o.G * pert[0].reshape(o.G.shape), o.H * pert[1].reshape(o.H.shape))
    o.step1()
    lev = o.lev0
    total = np.sum(lev.V * o.R[0])
    assert abs(total) < 1e-14 * np.sum(lev.V * np.abs(o.R[0]))
    # and for energy when the walls do no work and are at the gas temperature? only mass is exact
    assert np.max(np.abs(o.R[0])) > 1e-6


# --------------------------------------------------------------------------- mesh and transfers
def test_prolongation_weights_printed_values():
    with open(os.path.join(GOLDEN, "prolongation_weights.json")) as fh:
        ref = json.load(fh)
    case = _small_cavity(n=8, n_levels=2)
    vel = VelocityGrid.from_case(case)
    lv = build_levels(case, vel)
    P = Prolongation(lv[0], lv[1])
    nx = lv[0].nx

    def weights(ix, iy):
        c = iy * nx + ix
        return dict(zip(["w_A", "w_B", "w_C", "w_D"], P.w[:, c]))

    for key, (ix, iy) in {"inner": (3, 3), "boundary": (0, 3), "corner": (0, 0)}.items():
        w = weights(ix, iy)
        for name in ("w_A", "w_B", "w_C", "w_D"):
            assert w[name] == pytest.approx(ref[key][name], abs=1e-15), (key, name)


def test_prolongation_linear_exact_on_stretched_mesh():
    case = wl.config2(n=32, first=0.01, n_levels=3, nvel=4)
    vel = VelocityGrid.from_case(case)
    lv = build_levels(case, vel)
    for l in range(2):
        P = Prolongation(lv[l], lv[l + 1])
        lin_c = 0.3 + 1.7 * lv[l + 1].cx - 0.6 * lv[l + 1].cy
        lin_f = 0.3 + 1.7 * lv[l].cx - 0.6 * lv[l].cy
        assert np.allclose(P.apply(lin_c), lin_f, atol=1e-13)
        assert np.allclose(P.w.sum(axis=0), 1.0, atol=1e-14)


def test_restriction_conserves_volume_integral():
    case = wl.square_cylinder(scale=4, nu=4, nv=4, n_levels=3)
    vel = VelocityGrid.from_case(case)
    lv = build_levels(case, vel)
    q = wl.random_field((3, lv[0].nc), seed=5) * lv[0].fluid
    qc = restrict(lv[0], q)
    assert np.allclose(np.sum(qc * lv[1].V * lv[1].fluid, axis=1), np.sum(q * lv[0].V, axis=1),
                       rtol=1e-13)


def test_coarse_levels_keep_bodies():
    case = wl.square_cylinder(scale=2, nu=4, nv=4, n_levels=4)
    lv = build_levels(case, VelocityGrid.from_case(case))
    for l, lev in enumerate(lv):
        assert lev.solid.sum() == (16 // 2 ** l) ** 2
    case = wl.flat_plate(scale=2, nu=4, nv=4, n_levels=3)
    lv = build_levels(case, VelocityGrid.from_case(case))
    for l, lev in enumerate(lv):
        assert (lev.fty == wl.FACE_WALL).sum() == 8 // 2 ** l


# --------------------------------------------------------------------------- macro prediction
def test_wall_jacobian_matches_finite_differences():
    K = 3
    W = gm.conservative(1.2, 0.3, -0.1, 1.0 / 1.15, K)
    wall = np.array([0.95, 0.14, 0.0])
    J = fa.wall_jacobian(W, wall, K)
    h = 1e-6
    for b in range(4):
        e = np.zeros(4)
        e[b] = h
        fd = (fa.wall_ghost(W + e, wall, K) - fa.wall_ghost(W - e, wall, K)) / (2 * h)
        assert np.allclose(J[:, b], fd, rtol=1e-7, atol=1e-8), b


def test_split_residual_vanishes_for_uniform_rest_state():
    case = _small_cavity(n=8, n_levels=1)
    o = Oracle(case)
    ml = o.fas_levels[0]
    W = np.repeat(gm.conservative(1.0, 0.0, 0.0, 1.0, 3)[:, None], o.lev0.nc, axis=1)
    ml.freeze_gamma(W)
    assert np.max(np.abs(ml.rsplit(W))) < 1e-13
    # a gas hotter than the walls loses energy through them
    W[3] *= 1.1
    ml.freeze_gamma(W)
    assert np.all(ml.rsplit(W)[3][o.lev0.nb.min(axis=0) < 0] < 0)


def test_fas_fixed_point_and_convergence():
    """FAS returns W unchanged when the UGKS residual is zero, and repeated
    smoothing with a frozen Gamma solves R_split(W) + P = 0."""
    case = _small_cavity(n=8, n_levels=3, lid=0.15, Kn=0.2)
    o = Oracle(case)
    o.init_macro(wl.random_macro(case, seed=7, amp=0.05))
    W0 = o.W.copy()
    Wt = fa.fas_cycle(o.fas_levels, o.levels, o.prolongs, 0, W0, np.zeros_like(W0), o.params,
                      [np.zeros(l.nc) for l in o.levels])
    assert np.array_equal(Wt, W0)
    # W- and F-cycles keep the fixed point as well
    for gamma in (2, wl.CYCLE_F):
        Wt = fa.fas_cycle(o.fas_levels, o.levels, o.prolongs, 0, W0, np.zeros_like(W0), o.params[:3] + (gamma,),
                          [np.zeros(l.nc) for l in o.levels])
        assert np.array_equal(Wt, W0)
    Rt = 0.01 * wl.random_field(W0.shape, seed=8)
    # a closed box conserves mass: the target must carry zero total mass
    Rt[0] -= np.sum(o.lev0.V * Rt[0]) / np.sum(o.lev0.V)
    ml = o.fas_levels[0]
    ml.freeze_gamma(W0)
    P = Rt - ml.rsplit(W0)
    W = W0.copy()
    for _ in range(400):
        W = ml.smooth(W, P, 0.0)
    assert np.max(np.abs(P + ml.rsplit(W))) < 1e-12


def test_fas_on_fewer_levels_is_the_shallower_hierarchy():
    """A prediction on the first k levels of an L-level case equals the
    prediction of the same case built with k levels (the coarse levels the
    FAS cycle does not visit change nothing)."""
    case = _small_cavity(n=8, n_levels=3, lid=0.15, Kn=0.2)
    prim = wl.random_macro(case, seed=11, amp=0.05)
    for k in (1, 2):
        deep = Oracle(case.with_(fas_levels=k))
        flat = Oracle(case.with_(n_levels=k))
        assert len(deep.fas_levels) == k
        for o in (deep, flat):
            o.init_macro(prim)
        R = 0.01 * wl.random_field(deep.W.shape, seed=12) * deep.lev0.fluid
        assert np.array_equal(deep.predict(R), flat.predict(R))


# --------------------------------------------------------------------------- micro correction
def _cs_setup(case, seed):
    vel = VelocityGrid.from_case(case)
    g = gm.Gas.from_case(case)
    lv = build_levels(case, vel)
    pro = [Prolongation(lv[l], lv[l + 1]) for l in range(len(lv) - 1)]
    mls = [MicroLevel(l, vel, g.K_int) for l in lv]
    rng = np.random.default_rng(seed)
    tau_inv = [rng.uniform(0.5, 2.0, lv[0].nc)]
    for l in range(len(lv) - 1):
        tau_inv.append(restrict(lv[l], tau_inv[-1]))
    rG = rng.uniform(-1, 1, (vel.n, lv[0].nc)) * lv[0].fluid
    rH = rng.uniform(-1, 1, (vel.n, lv[0].nc)) * lv[0].fluid
    return vel, g, lv, pro, mls, tau_inv, rG, rH


def test_sweep_is_exact_without_walls():
    """With no wall coupling one upwind-ordered sweep solves the upwind system."""
    case = wl.flat_plate(scale=16, quad="trapezoid", nu=6, nv=6, vlo=-3, vhi=3, n_levels=1)
    case.face_type_y[:] = np.where(case.face_type_y == wl.FACE_WALL, 0, case.face_type_y)
    case.face_type_x[:, -1] = wl.FACE_OUTFLOW
    vel, g, lv, pro, mls, tau_inv, rG, rH = _cs_setup(case, 11)
    A = assemble(lv[0], vel, g.K_int, tau_inv[0])
    x = spla.spsolve(A.tocsc(), np.concatenate([rG.ravel(), rH.ravel()]))
    D = mls[0].diagonal(tau_inv[0], 0.0)
    dG, dH = mls[0].smooth(np.zeros_like(rG), np.zeros_like(rH), rG, rH, D)
    assert np.allclose(np.concatenate([dG.ravel(), dH.ravel()]), x, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("n,levels,gamma", [(4, 2, 1), (8, 3, 2), (8, 3, wl.CYCLE_F)])
def test_cs_cycle_converges_to_sparse_direct_solve(n, levels, gamma):
    """CS cycles as an iteration on the correction equation converge to its
    direct sparse solution (V-cycle, and W- and F-cycles over three levels)."""
    case = _small_cavity(n=n, nvel=6, vlo=-3, vhi=3, n_levels=levels, lid=0.2)
    vel, g, lv, pro, mls, tau_inv, rG, rH = _cs_setup(case, 12)
    A = assemble(lv[0], vel, g.K_int, tau_inv[0])
    x = spla.spsolve(A.tocsc(), np.concatenate([rG.ravel(), rH.ravel()]))
    dG = np.zeros_like(rG)
    dH = np.zeros_like(rH)
    params = (2, 1, 10, gamma)
    dtn = [np.zeros(l.nc) for l in lv]
    D = mls[0].diagonal(tau_inv[0], 0.0)
    for _ in range(60):
        eG, eH = mls[0].defect(dG, dH, rG, rH, D)
        cG, cH = cs_cycle(mls, lv, pro, 0, eG, eH, tau_inv, dtn, params)
        dG, dH = dG + cG, dH + cH
    got = np.concatenate([dG.ravel(), dH.ravel()])
    assert np.allclose(got, x, rtol=1e-10, atol=1e-12 * np.max(np.abs(x)))
    # and the defect form agrees with the assembled matrix
    eG, eH = mls[0].defect(dG * 0 + 0.3 * rG, dH * 0 - 0.2 * rH, rG, rH, D)
    ref = np.concatenate([rG.ravel(), rH.ravel()]) - A @ np.concatenate([0.3 * rG.ravel(), -0.2 * rH.ravel()])
    assert np.allclose(np.concatenate([eG.ravel(), eH.ravel()]), ref, atol=1e-12)


def _visit_order(cycle, levels, params):
    """Levels in the order the recursive cycle smooths them, one smoothing per
    visit (nu1 = nu_coarse = 1, nu2 = 0): the order in which it visits them."""
    seen = []
    for k, lev in enumerate(levels):
        inner = lev.smooth
        lev.smooth = (lambda *a, _k=k, _f=inner: (seen.append(_k), _f(*a))[1])
    cycle(params)
    return seen


@pytest.mark.parametrize("kind", ["fas", "cs"])
def test_cycle_shapes_visit_levels_in_textbook_order(kind):
    """Over four levels a V-cycle visits each level once on the way down, a
    W-cycle visits level l 2^l times, and an F-cycle goes down to the coarsest
    level and climbs one level higher after each coarsest visit: levels
    0 1 2 3, 3, 2 3, 1 2 3 (level l visited l + 1 times)."""
    case = _small_cavity(n=16, nvel=6, vlo=-3, vhi=3, n_levels=4, lid=0.2)
    o = Oracle(case)
    assert len(o.levels) == 4
    dtn = [np.zeros(l.nc) for l in o.levels]
    W = o.W.copy()
    rG = 0.01 * wl.random_field(o.G.shape, seed=3) * o.lev0.fluid
    tau_inv = o.level_tau_inv(np.ones(o.lev0.nc))

    def run(params):
        if kind == "fas":
            fa.fas_cycle(o.fas_levels, o.levels, o.prolongs, 0, W, np.zeros_like(W), params, dtn)
        else:
            cs_cycle(o.cs_levels, o.levels, o.prolongs, 0, rG, rG, tau_inv, dtn, params)

    levels = o.fas_levels if kind == "fas" else o.cs_levels
    assert _visit_order(run, levels, (1, 0, 1, 1)) == [0, 1, 2, 3]
    w = _visit_order(run, levels, (1, 0, 1, 2))
    assert [w.count(k) for k in range(4)] == [1, 2, 4, 8]
    assert _visit_order(run, levels, (1, 0, 1, wl.CYCLE_F)) == [0, 1, 2, 3, 3, 2, 3, 1, 2, 3]


def test_f_cycle_on_two_levels_is_the_w_cycle():
    """Below the second-coarsest level an F- and a W-cycle both make two
    coarsest-level solves, so on two levels they coincide; on three they differ."""
    for levels, same in ((2, True), (3, False)):
        case = _small_cavity(n=8, nvel=6, vlo=-3, vhi=3, n_levels=levels, lid=0.2)
        vel, g, lv, pro, mls, tau_inv, rG, rH = _cs_setup(case, 21)
        dtn = [np.zeros(l.nc) for l in lv]
        w = cs_cycle(mls, lv, pro, 0, rG, rH, tau_inv, dtn, (1, 1, 2, 2))
        f = cs_cycle(mls, lv, pro, 0, rG, rH, tau_inv, dtn, (1, 1, 2, wl.CYCLE_F))
        assert (np.array_equal(w[0], f[0]) and np.array_equal(w[1], f[1])) == same


# --------------------------------------------------------------------------- whole scheme
def test_cavity_mass_is_conserved_and_residual_falls():
    case = _small_cavity(n=8, nvel=12, vlo=-5, vhi=5, n_levels=2, lid=0.15, Kn=1.0)
    o = Oracle(case)
    m0 = np.sum(o.lev0.V * o.W[0])
    for _ in range(6):
        o.step1()
        o.advance()
    assert abs(np.sum(o.lev0.V * o.W[0]) - m0) < 1e-14
    assert np.max(o.history[-1] if o.history else o.step1()) < np.max(o.step1()) * 10


@pytest.mark.parametrize("Kn", [1.0, 0.05])
def test_multigrid_steady_state_equals_single_grid(Kn):
    """The multigrid cycles only accelerate convergence: 1, 2 and 3 levels
    reach the same steady state (Sec. IV A, MG solution equals IUGKS)."""
    sols = []
    for L in (1, 2, 3):
        case = wl.cavity(n=8, Kn=Kn, n_levels=L, quad="gauss_hermite", nvel=12, vlo=0, vhi=0,
                         nu_coarse=4)
        case.wall_y[8, :, 1] = 0.15
        o = Oracle(case)
        ok, n = o.iterate(400, tol=1e-10)
        assert ok, (L, n)
        sols.append(np.array(o.primitive()))
    for s in sols[1:]:
        err = np.max(np.abs(s - sols[0]), axis=1) / np.max(np.abs(sols[0]), axis=1)
        assert np.all(err < 2e-8), err


def test_plate_residual_falls_to_round_off():
    """The flat plate in air (K_int = 3): MIUGKS cycles drive every residual
    component far below 1e-6 (a Shakhov correction that carried momentum
    would stall it near 1e-4 at the cells beside the plate)."""
    case = wl.flat_plate(scale=4, quad="trapezoid", nu=16, nv=16, vlo=-5.0, vhi=5.0, n_levels=2,
                         precision="fp64", Kn=0.2)
    o = Oracle(case)
    ok, res = o.iterate(60, tol=1e-7)
    assert ok, res


def test_fmg_keeps_a_fixed_point():
    """The full-multigrid start leaves a discrete steady state unchanged: the
    restriction and interpolation of the full distribution reproduce a
    uniform field and every stage's cycles keep it."""
    case = _small_cavity(n=8, nvel=48, vlo=-8, vhi=8, n_levels=3)
    o = Oracle(case)
    G0, H0 = o.G.copy(), o.H.copy()
    n = o.fmg(2, tol=0.0)
    assert n == 4
    assert np.max(np.abs(o.G - G0)) < 1e-12 and np.max(np.abs(o.H - H0)) < 1e-12


def test_fmg_reaches_the_plain_steady_state():
    """Started by FMG or from rest, the cycles converge to the same steady
    state (the start changes the path, not the discrete solution)."""
    case = _small_cavity(n=8, nvel=24, vlo=-6, vhi=6, n_levels=3, lid=0.2, Kn=0.5)
    a, b = Oracle(case), Oracle(case)
    assert a.iterate(200, tol=1e-10)[0]
    b.fmg(5, tol=1e-8)
    assert b.iterate(200, tol=1e-10)[0]
    pa, pb = a.primitive(), b.primitive()
    for x, y in zip(pa, pb):
        assert np.max(np.abs(x - y)) < 1e-8 * max(1.0, np.max(np.abs(x)))


def test_explicit_step_keeps_a_uniform_freestream():
    """A uniform freestream in a farfield box is a fixed point of the
    explicit time-accurate step."""
    case = wl.flat_plate(scale=8, quad="trapezoid", nu=48, nv=48, vlo=-8, vhi=8, n_levels=1)
    case.face_type_y[:] = np.where(case.face_type_y == wl.FACE_WALL, 0, case.face_type_y)
    o = Oracle(case)
    G0, H0 = o.G.copy(), o.H.copy()
    for _ in range(2):
        dt, norms = o.explicit_step()
    assert dt == float(np.min(o.lev0.dt)) and np.max(norms) < 1e-12
    assert np.max(np.abs(o.G - G0)) < 1e-13 and np.max(np.abs(o.H - H0)) < 1e-13


def test_explicit_steps_conserve_mass_in_a_closed_box():
    """Without the closed-domain renormalisation the explicit steps keep the
    total mass of a lid-driven box to round-off (wide velocity grid): the
    macroscopic update is a flux difference and the collision term conserves
    mass up to the quadrature of the Maxwellian."""
    case = _small_cavity(n=8, nvel=48, vlo=-8, vhi=8, n_levels=1, lid=0.3, Kn=0.3)
    o = Oracle(case)
    o.closed = False
    o.init_macro(wl.random_macro(case, seed=21, amp=0.05))
    m0 = float(np.sum(o.lev0.V * o.W[0]))
    for _ in range(4):
        o.explicit_step()
    m1 = float(np.sum(o.lev0.V * o.W[0]))
    assert abs(m1 - m0) < 1e-12 * m0


# --------------------------------------------------------------------------- symmetry faces
def test_symmetry_faces_carry_no_mass_shear_or_energy():
    """Specular reflection: for any distribution the flux through a symmetry
    face carries no mass, no tangential momentum and no energy (the incoming
    half is the mirror image of the outgoing half)."""
    case = wl.sheared_half_box(n=6, quad="trapezoid", nvel=10, vlo=-4, vhi=4)
    o = Oracle(case)
    rng = np.random.default_rng(31)
    G = o.G * rng.uniform(0.5, 1.5, o.G.shape)
    H = o.H * rng.uniform(0.5, 1.5, o.H.shape)
    un, Gf, Hf = fx.boundary_face_values(G, H, o.lev0, o.vel, o.gas, case.farfield)
    sym = o.lev0.btype == wl.FACE_SYMMETRY
    assert sym.sum() == 12
    for j in np.nonzero(sym)[0]:
        s = o.lev0.bside[j]
        ut = o.vel.v if s < 2 else o.vel.u
        w = o.vel.w
        mass = np.sum(w * un[:, j] * Gf[:, j])
        shear = np.sum(w * un[:, j] * ut * Gf[:, j])
        energy = 0.5 * np.sum(w * un[:, j] * ((o.vel.u ** 2 + o.vel.v ** 2) * Gf[:, j] + Hf[:, j]))
        scale = np.sum(w * np.abs(un[:, j]) * Gf[:, j])
        assert max(abs(mass), abs(shear)) < 1e-14 * scale and abs(energy) < 1e-13 * scale
    # the walls do transfer shear: the pin is not vacuous
    wall = np.nonzero(o.lev0.btype == wl.FACE_WALL)[0]
    assert np.any(np.abs(ad_shear(o, G, H)[wall]) > 1e-3)


def ad_shear(o, G, H):
    un, Gf, Hf = fx.boundary_face_values(G, H, o.lev0, o.vel, o.gas, o.case.farfield)
    ut = np.where(o.lev0.bside[None, :] < 2, o.vel.v[:, None], o.vel.u[:, None])
    return np.sum(o.vel.w[:, None] * un * ut * Gf, axis=0)


def test_uniform_flow_along_symmetry_planes_is_a_fixed_point():
    """A freestream parallel to two symmetry planes is steady: zero residuals,
    and a whole cycle (FAS prediction and CS correction with their symmetry
    ghosts) leaves f unchanged.  Reflecting the wrong velocity component
    would send the flow back upstream and break both."""
    case = wl.symmetric_channel(n=6, U=0.3, quad="trapezoid", nvel=24, vlo=-6, vhi=6, n_levels=2, Kn=0.5)
    o = Oracle(case)
    G0, H0 = o.G.copy(), o.H.copy()
    n = o.step1()
    assert np.max(n) < 1e-13
    assert np.max(np.abs(o.divG)) < 1e-12 * np.max(np.abs(o.G))
    o.advance()
    assert np.max(np.abs(o.G - G0)) < 1e-13 and np.max(np.abs(o.H - H0)) < 1e-13


def test_cs_cycle_with_symmetry_faces_converges_to_direct_solve():
    """The correction cycle with symmetry ghosts (lagged to the start of each
    sweep) converges to the direct sparse solution of the correction
    equation, whose symmetry rows couple each incoming velocity to its mirror."""
    case = wl.sheared_half_box(n=8, quad="trapezoid", nvel=6, vlo=-3, vhi=3, n_levels=2)
    vel, g, lv, pro, mls, tau_inv, rG, rH = _cs_setup(case, 32)
    A = assemble(lv[0], vel, g.K_int, tau_inv[0])
    x = spla.spsolve(A.tocsc(), np.concatenate([rG.ravel(), rH.ravel()]))
    dG = np.zeros_like(rG)
    dH = np.zeros_like(rH)
    dtn = [np.zeros(l.nc) for l in lv]
    D = mls[0].diagonal(tau_inv[0], 0.0)
    for _ in range(60):
        eG, eH = mls[0].defect(dG, dH, rG, rH, D)
        cG, cH = cs_cycle(mls, lv, pro, 0, eG, eH, tau_inv, dtn, (2, 1, 10))
        dG, dH = dG + cG, dH + cH
    got = np.concatenate([dG.ravel(), dH.ravel()])
    assert np.allclose(got, x, rtol=1e-10, atol=1e-12 * np.max(np.abs(x)))
    # the symmetry rows are really there: dropping them changes the solution
    assert mls[0].sym.sum() == 16


def test_free_molecular_gap_reaches_the_closed_form():
    """Survey pin 'free-molecular limit', as heat transfer between plates at
    rest: with collisions vanishing (Kn 1e12) the scheme's steady state is
    the uniform pair of half-range wall Maxwellians, and the heat flux is
    the closed form's."""
    case = wl.free_molecular_gap(quad="trapezoid", nvel=16, vlo=-5.0, vhi=5.0, n_levels=2)
    o = Oracle(case)
    ok, norms = o.iterate(200, tol=1e-13)
    assert ok, norms
    area = float(np.sum(o.lev0.V))
    G, H = free_molecular_closed_form(case, o.vel, o.gas.K_int, o.M0, area)
    assert np.max(np.abs(o.G - G[:, None])) < 1e-10 * np.max(G)
    assert np.max(np.abs(o.H - H[:, None])) < 1e-10 * np.max(H)
    # the bottom plate, hotter, heats the gap: upward heat flux everywhere
    qy = o.q[1]
    v, u, w = o.vel.v, o.vel.u, o.vel.w
    q_ref = 0.5 * np.sum(w * v * ((u * u + v * v) * G + H))
    assert q_ref > 0 and np.max(np.abs(qy - q_ref)) < 1e-10 * q_ref
