"""The MIUGKS outer iteration, Steps 1-8 of Sec. II D (oracle; test infrastructure only).

  1  time-averaged UGKS fluxes -> div and R; RMS residual check (Sec. IV A)
  2  W~ = FAS(0, W^n, R^n)
  3  g~ = Shakhov(W~, q^n), tau~ = mu(T~)/p~
  4  r = (g~ - f^n)/tau~ - div
  5  dF = CS(0, r)
  6  f^{n+1} = f^n + dF
  7  W^{n+1}, q^{n+1} from the moments of f^{n+1}
  8  stop when every RMS residual component is below the tolerance

Readings added to the paper's steps: a cell whose predicted state has
non-positive density or temperature keeps W^n; in a closed domain (walls
only) f is rescaled after Step 6 so that the total mass keeps its initial
value, which selects one member of the one-parameter family of steady states
of a closed box; the optional pseudo step dt_n = a^n dt_p (Sec. III D and
Sec. IV C) adds 1/dt_n to the diagonals of both defect equations on every
level.
"""
from __future__ import annotations

import copy

import numpy as np

from . import gas as gm
from .cs import MicroLevel, cs_cycle
from .fas import MacroLevel, fas_cycle
from .flux import residuals, residual_norm
from .mesh import Prolongation, build_levels, restrict
from .quadrature import VelocityGrid


class Oracle:
    def __init__(self, case):
        self.case = case
        self.vel = VelocityGrid.from_case(case)
        self.gas = gm.Gas.from_case(case)
        self.levels = build_levels(case, self.vel)
        self.prolongs = [Prolongation(self.levels[l], self.levels[l + 1])
                         for l in range(len(self.levels) - 1)]
        # the FAS prediction may stop above the coarsest level of the CS cycle
        nfas = case.fas_levels if case.fas_levels > 0 else len(self.levels)
        self.fas_levels = [MacroLevel(lev, self.gas, case.farfield) for lev in self.levels[:nfas]]
        self.cs_levels = [MicroLevel(lev, self.vel, self.gas.K_int) for lev in self.levels]
        # coarse corrections per level visit: 1 V-cycle, 2 W-cycle, CYCLE_F
        # F-cycle (0: V-cycle)
        gamma = case.cycle_gamma if case.cycle_gamma != 0 else 1
        self.params = (case.nu1, case.nu2, case.nu_coarse, gamma)
        # the CS cycle may take its own number of coarsest-level smoothings
        # and of coarse corrections
        nuc_cs = case.nu_coarse_cs if case.nu_coarse_cs > 0 else case.nu_coarse
        gamma_cs = case.cycle_gamma_cs if case.cycle_gamma_cs != 0 else gamma
        self.cs_params = (case.nu1, case.nu2, nuc_cs, gamma_cs)
        self.closed = case.closed()
        self.cycle = 0
        self.history = []
        self.init_macro(case.init)

    # ---------------------------------------------------------------- state
    @property
    def lev0(self):
        return self.levels[0]

    def init_macro(self, prim):
        """f := reduced Maxwellian of (rho, U, V, T) per cell (solid cells hold zero)."""
        rho, U, V, T = (np.asarray(a, float).ravel() for a in prim)
        G, H = gm.maxwellian(rho, U, V, 1.0 / T, self.vel.u[:, None], self.vel.v[:, None],
                             self.gas.K_int)
        fl = self.lev0.fluid
        self.set_f(np.where(fl, G, 0.0), np.where(fl, H, 0.0))
        self.M0 = float(np.sum(self.lev0.V * self.W[0] * fl))

    def set_f(self, G, H):
        self.G = np.array(G, float)
        self.H = np.array(H, float)
        self._moments()

    def _moments(self):
        fl = self.lev0.fluid
        W = gm.moments(self.G, self.H, self.vel)
        with np.errstate(all="ignore"):
            U = W[1] / W[0]
            V = W[2] / W[0]
            q = gm.heat_flux(self.G, self.H, self.vel, U, V)
        self.W = np.where(fl, W, 0.0)
        self.q = np.where(fl, q, 0.0)

    def primitive(self):
        with np.errstate(all="ignore"):
            rho, U, V, lam = gm.primitive(self.W, self.gas.K)
        return rho, U, V, 1.0 / lam

    def dtn_inv(self):
        a = self.case.dtn_growth
        if a <= 0:
            return [np.zeros(lev.nc) for lev in self.levels]
        f = float(a) ** (-self.cycle)
        cap = getattr(self.case, "dtn_max", 0.0)
        if cap > 0:
            f = max(f, 1.0 / cap)
        return [f / lev.dt for lev in self.levels]

    # ---------------------------------------------------------------- steps
    def step1(self):
        """UGKS residuals of the current state and their RMS norms."""
        self.divG, self.divH, self.R = residuals(self.G, self.H, self.W, self.lev0, self.vel,
                                                 self.gas, self.case.farfield)
        return residual_norm(self.R, self.lev0)

    def predict(self, R):
        """Step 2: FAS V-cycle of the macroscopic defect equation, then the
        positivity guard."""
        dtn = self.dtn_inv()
        Wt = fas_cycle(self.fas_levels, self.levels, self.prolongs, 0, self.W, R,
                       self.params, dtn)
        with np.errstate(all="ignore"):
            rho, U, V, lam = gm.primitive(Wt, self.gas.K)
        bad = ~((rho > 0) & (lam > 0) & np.isfinite(lam))
        return np.where(bad & self.lev0.fluid, self.W, Wt)

    def micro_residual(self, Wt):
        """Steps 3-4: r = (g~ - f)/tau~ - div with the Shakhov g~ of W~ and q^n."""
        fl = self.lev0.fluid
        with np.errstate(all="ignore"):
            rho, U, V, lam = gm.primitive(Wt, self.gas.K)
            tau_inv = np.where(fl, 1.0 / self.gas.tau(rho, lam), 0.0)
            Gt, Ht = gm.shakhov(rho, U, V, lam, self.q[0], self.q[1], self.vel.u[:, None],
                                self.vel.v[:, None], self.gas.K_int, self.gas.Pr)
        rG = np.where(fl, (Gt - self.G) * tau_inv - self.divG, 0.0)
        rH = np.where(fl, (Ht - self.H) * tau_inv - self.divH, 0.0)
        return rG, rH, tau_inv

    def level_tau_inv(self, tau_inv):
        out = [tau_inv]
        for l in range(len(self.levels) - 1):
            out.append(restrict(self.levels[l], out[-1]))
        return out

    def correct(self, rG, rH, tau_inv):
        """Step 5: CS V-cycle of the correction equation."""
        return cs_cycle(self.cs_levels, self.levels, self.prolongs, 0, rG, rH,
                        self.level_tau_inv(tau_inv), self.dtn_inv(), self.cs_params)

    def update(self, dG, dH):
        """Steps 6-7 (+ mass renormalisation in closed domains)."""
        self.G = self.G + dG
        self.H = self.H + dH
        self._moments()
        if self.closed:
            M = float(np.sum(self.lev0.V * self.W[0] * self.lev0.fluid))
            s = self.M0 / M
            self.G *= s
            self.H *= s
            self.W *= s
            self.q *= s

    def advance(self):
        """Steps 2-7 after a Step 1 that did not meet the tolerance."""
        Wt = self.predict(self.R)
        rG, rH, tau_inv = self.micro_residual(Wt)
        dG, dH = self.correct(rG, rH, tau_inv)
        self.update(dG, dH)
        self.cycle += 1

    def _stage(self, top):
        """The same problem with level `top` as its finest level (a stage of
        the full-multigrid start): the levels below are dropped, the FAS depth
        counts from `top`, the pseudo-step counter restarts and the reference
        mass of a closed domain is kept."""
        st = copy.copy(self)
        st.levels = self.levels[top:]
        st.prolongs = self.prolongs[top:]
        nfas = self.case.fas_levels if self.case.fas_levels > 0 else len(st.levels)
        st.fas_levels = [MacroLevel(lev, self.gas, self.case.farfield) for lev in st.levels[:nfas]]
        st.cs_levels = self.cs_levels[top:]
        st.cycle = 0
        st.history = []
        return st

    def fmg_interpolate(self, l, qc):
        """FMG interpolation of a full distribution from level l + 1 to level
        l: the bilinear prolongation where its stencil interpolates (every
        weight non-negative), the parent cell's value where it would
        extrapolate, so that a positive distribution stays positive; zero on
        solid cells."""
        P = self.prolongs[l]
        w = np.array(P.w)
        inside = np.all(w >= 0.0, axis=0)
        out = np.where(inside, sum(w[a] * qc[..., P.idx[a]] for a in range(4)), qc[..., P.idx[0]])
        return out * self.levels[l].fluid

    def fmg(self, cycles, tol=1e-6):
        """Full-multigrid start (Sec. III C, FMG): the current distribution is
        restricted to the coarsest level (volume-weighted means); each level
        from the coarsest up to level 1 then runs up to `cycles` outer cycles
        as the finest level of its own sub-hierarchy, and the distribution it
        reaches (not a correction) is interpolated bilinearly to the next
        finer level.  Returns the number of cycles run on the coarse levels."""
        G, H = self.G, self.H
        for l in range(len(self.levels) - 1):
            G = restrict(self.levels[l], G)
            H = restrict(self.levels[l], H)
        done = 0
        for top in range(len(self.levels) - 1, 0, -1):
            st = self._stage(top)
            st.set_f(G, H)
            ok, _ = st.iterate(cycles, tol)
            done += len(st.history) - (1 if ok else 0)
            G = self.fmg_interpolate(top - 1, st.G)
            H = self.fmg_interpolate(top - 1, st.H)
        self.set_f(G, H)
        self.cycle = 0
        self.history = []
        return done

    def explicit_step(self):
        """One explicit, time-accurate UGKS step (the scheme behind the
        residuals of Sec. II A): the global step dt is the smallest CFL step of
        the finest level, used by every face; W* = W^n + dt R (cells with
        non-positive density or temperature keep W^n); Shakhov equilibria of
        W^n and W* with q^n; the trapezoidal collision update
        f = [f - dt div + dt/2 (g*/tau* + (g^n - f)/tau^n)] / (1 + dt/(2 tau*));
        the moments of the new f (and the closed-domain renormalisation).
        Returns dt and the RMS residuals of the step's fluxes."""
        lev = copy.copy(self.lev0)
        dt = float(np.min(lev.dt))
        lev.dt = np.full_like(lev.dt, dt)
        lev.fdt = np.full_like(lev.fdt, dt)
        divG, divH, R = residuals(self.G, self.H, self.W, lev, self.vel, self.gas, self.case.farfield)
        norms = residual_norm(R, lev)
        fl = lev.fluid
        Ws = np.where(fl, self.W + dt * R, self.W)
        with np.errstate(all="ignore"):
            rho, U, V, lam = gm.primitive(Ws, self.gas.K)
        bad = ~((rho > 0) & (lam > 0) & np.isfinite(lam))
        Ws = np.where(bad & fl, self.W, Ws)

        def equilibrium(W):
            with np.errstate(all="ignore"):
                rho, U, V, lam = gm.primitive(W, self.gas.K)
                ti = np.where(fl, 1.0 / self.gas.tau(rho, lam), 0.0)
                G, H = gm.shakhov(rho, U, V, lam, self.q[0], self.q[1], self.vel.u[:, None],
                                  self.vel.v[:, None], self.gas.K_int, self.gas.Pr)
            return G, H, ti

        G0, H0, t0 = equilibrium(self.W)
        G1, H1, t1 = equilibrium(Ws)
        den = 1.0 / (1.0 + 0.5 * dt * t1)
        G = np.where(fl, (self.G - dt * divG + 0.5 * dt * (G1 * t1 + (G0 - self.G) * t0)) * den, 0.0)
        H = np.where(fl, (self.H - dt * divH + 0.5 * dt * (H1 * t1 + (H0 - self.H) * t0)) * den, 0.0)
        self.G, self.H = G, H
        self._moments()
        if self.closed:
            M = float(np.sum(self.lev0.V * self.W[0] * fl))
            s = self.M0 / M
            self.G *= s
            self.H *= s
            self.W *= s
            self.q *= s
        return dt, norms

    def iterate(self, max_cycles, tol=1e-6):
        """Run outer cycles until max_c R_rms,c < tol; returns (converged, norms)."""
        norms = None
        for _ in range(max_cycles):
            norms = self.step1()
            self.history.append(norms)
            if np.max(norms) < tol:
                return True, norms
            self.advance()
        return False, norms
