"""Explicit UGKS interface flux and the residuals of Step 1 (oracle; test infrastructure only).

The macroscopic residual R_i = -(1/V_i) sum_j S_ij F_ij (Sec. II A, residual
definitions) and the transport part of the microscopic residual
div_ik = (1/V_i) sum_j S_ij u_kn ftilde_ij,k are evaluated with the
time-averaged UGKS flux over the physical step dt_p (Sec. II A 1, the flux
equation F_ij = sum_k (1/dt_p) int_0^dt_p u_kn ftilde_ij,k(t) psi_k dt).
The paper defers the interface distribution to the UGKS literature; the
oracle uses the standard characteristic solution of the BGK-Shakhov model,
normal direction only:

  ftilde(t) = (1 - e^{-t/tau}) g0 (1 + Shakhov)
            + ((t + tau) e^{-t/tau} - tau) u_n abar g0
            + (t - tau + tau e^{-t/tau}) Abar g0
            + e^{-t/tau} (f_up - u_n t sigma_up)

with van Leer-limited slopes sigma, the upwind interface value f_up, g0 the
Maxwellian of the discrete moments of f_up, abar the micro-slope of the side
the particle comes from and Abar the time slope from the compatibility
condition.  Walls, farfield, outflow and symmetry faces carry first-order
kinetic boundary fluxes (diffuse reflection with the wall density fixed by
zero net mass flux; specular reflection at a symmetry face; Sec. III B).
"""
from __future__ import annotations

import numpy as np

from workloads import FACE_WALL, FACE_FARFIELD, FACE_OUTFLOW, FACE_SYMMETRY
from . import gas as gm


def _abs(a):
    """|a|, with the branch taken on the real part (the same values for real a;
    for complex a the analytic continuation of each branch, so that a complex
    step differentiates the limiter where it is smooth)."""
    return np.where(np.real(a) < 0, -a, a)


def van_leer(a, b):
    """(sgn a + sgn b) |a| |b| / (|a| + |b|), zero when both vanish."""
    den = _abs(a) + _abs(b)
    pos = np.real(den) > 0
    safe = np.where(pos, den, 1.0)
    return np.where(pos, (np.sign(np.real(a)) + np.sign(np.real(b))) * _abs(a) * _abs(b) / safe, 0.0)


def slopes(F, lev):
    """Limited slope of F (Nk, Nc) along x and y; zero difference across non-interior faces."""
    out = np.zeros((2,) + F.shape, dtype=F.dtype)
    for d in (0, 1):
        lo, hi = lev.nb[2 * d], lev.nb[2 * d + 1]
        sm = np.where(lo >= 0, (F - F[:, np.maximum(lo, 0)]) / np.where(lo >= 0, lev.dcent[2 * d], 1.0), 0.0)
        sp = np.where(hi >= 0, (F[:, np.maximum(hi, 0)] - F) / np.where(hi >= 0, lev.dcent[2 * d + 1], 1.0), 0.0)
        out[d] = van_leer(sm, sp)
    return out


def micro_slope(b, U, V, lam, K):
    """Coefficients (a1..a4) of abar = a1 + a2 u + a3 v + a4 (u^2 + v^2 + xi^2)/2 with
    <abar psi g0> = rho0 b, solved in closed form for a Maxwellian g0 (K total
    degrees of freedom)."""
    e = U * U + V * V + K / (2.0 * lam)
    R2 = b[1] - U * b[0]
    R3 = b[2] - V * b[0]
    R4 = 2.0 * b[3] - e * b[0]
    a4 = 4.0 * lam * lam / K * (R4 - 2.0 * U * R2 - 2.0 * V * R3)
    a3 = 2.0 * lam * R3 - V * a4
    a2 = 2.0 * lam * R2 - U * a4
    a1 = b[0] - U * a2 - V * a3 - 0.5 * a4 * e
    return np.array([a1, a2, a3, a4])


def slope_times_g0(a, G0, H0, u, v, lam, K_int):
    """G and H parts of abar * g0 after integrating over the extra components."""
    poly = a[0] + a[1] * u + a[2] * v + 0.5 * a[3] * (u * u + v * v)
    Gs = (poly + 0.5 * a[3] * K_int / (2.0 * lam)) * G0
    Hs = (poly + 0.5 * a[3] * (K_int + 2.0) / (2.0 * lam)) * H0
    return Gs, Hs


def time_coefficients(dt, tau):
    """Exact integrals over [0, dt] of the time factors of ftilde (x = dt/tau):

      q1 = int (1 - e^{-t/tau})              = dt - tau (1 - e^{-x})
      q2 = int ((t + tau) e^{-t/tau} - tau)  = 2 tau^2 (1 - e^{-x}) - tau dt (1 + e^{-x})
      q3 = int (t - tau + tau e^{-t/tau})    = dt^2/2 - tau dt + tau^2 (1 - e^{-x})
      q4 = int e^{-t/tau}                    = tau (1 - e^{-x})
      q5 = int -t e^{-t/tau}                 = tau dt e^{-x} - tau^2 (1 - e^{-x})

    For x < 1/2 the closed forms cancel badly, so their Taylor series are
    summed instead (q1 = dt sum_{m>=2} (-x)^m/(x m!), q2 = dt^2 sum_{m>=3}
    (-1)^m (m-2) x^(m-2)/m!, q3 = dt^2 sum_{m>=3} (-1)^(m+1) x^(m-2)/m!,
    q5 = dt^2 sum_{m>=2} (-1)^m (1-m) x^(m-2)/m!), 24 terms.
    """
    dt = np.asarray(dt, float)
    tau = np.asarray(tau)
    x = dt / tau
    em1 = -np.expm1(-x)           # 1 - e
    e = np.exp(-x)
    q1 = dt - tau * em1
    q2 = 2.0 * tau * tau * em1 - tau * dt - tau * dt * e
    q3 = 0.5 * dt * dt - tau * dt + tau * tau * em1
    q4 = tau * em1
    q5 = tau * dt * e - tau * tau * em1
    small = np.real(x) < 0.5
    if np.any(small):
        xs = np.where(small, x, 0.0)
        s1 = np.zeros_like(xs)
        s2 = np.zeros_like(xs)
        s3 = np.zeros_like(xs)
        s5 = np.zeros_like(xs)
        fact = 1.0
        for m in range(1, 26):
            fact *= m
            sg = -1.0 if m % 2 else 1.0
            if m >= 2:
                s1 += sg * xs ** (m - 1) / fact
                s5 += sg * (1 - m) * xs ** (m - 2) / fact
            if m >= 3:
                s2 += sg * (m - 2) * xs ** (m - 2) / fact
                s3 += -sg * xs ** (m - 2) / fact
        q1 = np.where(small, dt * s1, q1)
        q2 = np.where(small, dt * dt * s2, q2)
        q3 = np.where(small, dt * dt * s3, q3)
        q5 = np.where(small, dt * dt * s5, q5)
    return q1, q2, q3, q4, q5


class InterfaceState:
    """Per-face quantities of the UGKS interface distribution for the faces of
    one direction (velocity axis first where a quantity depends on k)."""


def interface_state(G, H, W, lev, vel, gas, d, sG=None, sH=None):
    """Interface states of the interior faces of direction d (0: x, 1: y),
    normal from L to R: the reconstructed values and limited slopes on both
    sides, the upwind pair, the interface equilibrium (moments W0, heat flux
    q0, collision time tau0, Maxwellian g0 and Shakhov g0+), the
    micro-slopes of both sides and the time slope, as the flux uses them."""
    if sG is None:
        sG, sH = slopes(G, lev), slopes(H, lev)
    K, Ki = gas.K, gas.K_int
    u = vel.u[:, None]
    v = vel.v[:, None]
    st = InterfaceState()
    m = lev.fdir == d
    st.mask = m
    L, R = lev.fL[m], lev.fR[m]
    dL, dR, dt = lev.fdL[m], lev.fdR[m], lev.fdt[m]
    st.L, st.R, st.dL, st.dR, st.dt = L, R, dL, dR, dt
    un = u if d == 0 else v
    st.un = un
    pos, neg = un > 0, un < 0

    def upwind(a, b):
        return np.where(pos, a, np.where(neg, b, 0.5 * (a + b)))

    st.GL = G[:, L] + sG[d][:, L] * dL
    st.GR = G[:, R] - sG[d][:, R] * dR
    st.HL = H[:, L] + sH[d][:, L] * dL
    st.HR = H[:, R] - sH[d][:, R] * dR
    st.sGL, st.sGR, st.sHL, st.sHR = sG[d][:, L], sG[d][:, R], sH[d][:, L], sH[d][:, R]
    st.Gup, st.Hup = upwind(st.GL, st.GR), upwind(st.HL, st.HR)
    st.sGup, st.sHup = upwind(st.sGL, st.sGR), upwind(st.sHL, st.sHR)

    # interface equilibrium from the discrete moments of the upwind distribution
    st.W0 = gm.moments(st.Gup, st.Hup, vel)
    rho0, U0, V0, lam0 = gm.primitive(st.W0, K)
    st.prim0 = (rho0, U0, V0, lam0)
    st.q0 = gm.heat_flux(st.Gup, st.Hup, vel, U0, V0)
    st.tau0 = gas.tau(rho0, lam0)
    st.G0, st.H0 = gm.maxwellian(rho0, U0, V0, lam0, u, v, Ki)
    st.Geq, st.Heq = gm.shakhov(rho0, U0, V0, lam0, st.q0[0], st.q0[1], u, v, Ki, gas.Pr)

    # spatial micro-slopes from the macroscopic slopes on each side
    st.aL = micro_slope((st.W0 - W[:, L]) / dL / rho0, U0, V0, lam0, K)
    st.aR = micro_slope((W[:, R] - st.W0) / dR / rho0, U0, V0, lam0, K)
    st.GaL, st.HaL = slope_times_g0(st.aL, st.G0, st.H0, u, v, lam0, Ki)
    st.GaR, st.HaR = slope_times_g0(st.aR, st.G0, st.H0, u, v, lam0, Ki)
    st.Gs, st.Hs = upwind(st.GaL, st.GaR), upwind(st.HaL, st.HaR)

    # time slope from the compatibility condition, in discrete form
    b = -gm.moments(un * st.Gs, un * st.Hs, vel) / rho0
    st.A = micro_slope(b, U0, V0, lam0, K)
    st.GA, st.HA = slope_times_g0(st.A, st.G0, st.H0, u, v, lam0, Ki)
    st.q = time_coefficients(dt, st.tau0)
    return st


def interior_fluxes(G, H, W, lev, vel, gas):
    """Time-averaged flux (Nk, nfaces) of G and H through every interior face,
    normal pointing from L to R."""
    sG, sH = slopes(G, lev), slopes(H, lev)
    nf = len(lev.fL)
    PhiG = np.zeros((vel.n, nf), dtype=G.dtype)
    PhiH = np.zeros((vel.n, nf), dtype=G.dtype)
    for d in (0, 1):
        if not (lev.fdir == d).any():
            continue
        st = interface_state(G, H, W, lev, vel, gas, d, sG, sH)
        m, un, dt = st.mask, st.un, st.dt
        q1, q2, q3, q4, q5 = st.q
        PhiG[:, m] = un * (q1 * st.Geq + q2 * un * st.Gs + q3 * st.GA + q4 * st.Gup + q5 * un * st.sGup) / dt
        PhiH[:, m] = un * (q1 * st.Heq + q2 * un * st.Hs + q3 * st.HA + q4 * st.Hup + q5 * un * st.sHup) / dt
    return PhiG, PhiH


def wall_maxwellian(Tw, Uw, Vw, u, v, K_int):
    """C_k of the diffuse wall (Sec. III B, wall distribution): unit-density Maxwellian."""
    lam = 1.0 / Tw
    CG = (lam / np.pi) * np.exp(-lam * ((u - Uw) ** 2 + (v - Vw) ** 2))
    return CG, (K_int / (2.0 * lam)) * CG


def boundary_face_values(G, H, lev, vel, gas, farfield):
    """Distribution on each boundary side of a fluid cell, (Nk, nsides), and u_n outward."""
    nb = len(lev.bcell)
    un = np.zeros((vel.n, nb))
    Gf = np.zeros((vel.n, nb), dtype=np.result_type(G, lev.wall))
    Hf = np.zeros((vel.n, nb), dtype=Gf.dtype)
    rho_inf, U_inf, V_inf, T_inf = farfield
    Ginf, Hinf = gm.maxwellian(rho_inf, U_inf, V_inf, 1.0 / T_inf, vel.u, vel.v, gas.K_int)
    for j in range(nb):
        c, s, t = lev.bcell[j], lev.bside[j], lev.btype[j]
        sign = -1.0 if s % 2 == 0 else 1.0
        u_n = sign * (vel.u if s < 2 else vel.v)
        un[:, j] = u_n
        out = u_n > 0
        if t == FACE_WALL:
            Tw, Uw, Vw = lev.wall[s, c]
            CG, CH = wall_maxwellian(Tw, Uw, Vw, vel.u, vel.v, gas.K_int)
            inn = u_n < 0
            rho_w = -np.sum((vel.w * u_n * G[:, c])[out]) / np.sum((vel.w * u_n * CG)[inn])
            Gf[:, j] = np.where(out, G[:, c], rho_w * CG)
            Hf[:, j] = np.where(out, H[:, c], rho_w * CH)
        elif t == FACE_FARFIELD:
            Gf[:, j] = np.where(out, G[:, c], Ginf)
            Hf[:, j] = np.where(out, H[:, c], Hinf)
        elif t == FACE_OUTFLOW:
            Gf[:, j] = G[:, c]
            Hf[:, j] = H[:, c]
        elif t == FACE_SYMMETRY:
            # specular reflection: the incoming velocity takes the cell's value
            # at the velocity with the normal component reversed
            mk = vel.mirror(s // 2)
            Gf[:, j] = np.where(out, G[:, c], G[mk, c])
            Hf[:, j] = np.where(out, H[:, c], H[mk, c])
        else:
            raise ValueError(f"unsupported face tag {t}")
    return un, Gf, Hf


def residuals(G, H, W, lev, vel, gas, farfield):
    """Step 1: div (Nk, Nc) for G and H and the macroscopic residual R (4, Nc)."""
    divG = np.zeros_like(G)
    divH = np.zeros_like(H)
    PhiG, PhiH = interior_fluxes(G, H, W, lev, vel, gas)
    cL = lev.fS / lev.V[lev.fL]
    cR = lev.fS / lev.V[lev.fR]
    np.add.at(divG.T, lev.fL, (PhiG * cL).T)
    np.add.at(divG.T, lev.fR, (-PhiG * cR).T)
    np.add.at(divH.T, lev.fL, (PhiH * cL).T)
    np.add.at(divH.T, lev.fR, (-PhiH * cR).T)
    if len(lev.bcell):
        un, Gf, Hf = boundary_face_values(G, H, lev, vel, gas, farfield)
        cb = lev.S[lev.bside, lev.bcell] / lev.V[lev.bcell]
        np.add.at(divG.T, lev.bcell, (un * Gf * cb).T)
        np.add.at(divH.T, lev.bcell, (un * Hf * cb).T)
    R = -gm.moments(divG, divH, vel)
    return divG, divH, R


def residual_norm(R, lev):
    """Root-mean-square residual of each conservative variable over fluid cells
    (Sec. IV A, residual definition)."""
    Rf = R[:, lev.fluid]
    return np.sqrt(np.sum(Rf * Rf, axis=1) / Rf.shape[1])
