"""FAS V-cycle of the macroscopic prediction step (oracle; test infrastructure only).

Step 2 of the outer iteration (Sec. II D) solves the defect equation of the
conservative variables with the split Euler flux on its left-hand side
(Sec. II A 1, flux-splitting equation):

  F_ij(W) = 1/2 [T(W_i).n + T(W_j).n + Gamma_ij (W_i - W_j)],
  Gamma_ij = |U.n| + a_s + 2 nu / (n.(x_j - x_i)),

  R_split(W)_i = -(1/V_i) sum_j S_ij F_ij(W),

by a full-approximation-storage V-cycle (Sec. II D, FAS steps (a)-(c)) with
the forcing function P = R - R_split(W^0) (Sec. II C 2) and renewed residuals
R^(m) = P + R_split(W^(m)).  One smoothing is the symmetric red-black
Gauss-Seidel sweep (colour 0, 1, 0) of the defect equation of Sec. II A 1:

  E_i = [R^(m)_i - (1/2V_i) sum_j S_ij (T(W_j + E_j).n - T(W_j).n - Gamma_ij E_j)] / D_i,
  D_i = (1/2V_i) sum_j S_ij Gamma_ij (+ 1/dt_n),

starting from E = 0, followed by W += E.

Readings where the paper is silent: Gamma uses the arithmetic mean of the
two cells' primitive variables (rho, U, V, T) and is frozen for a whole visit
of a level; ghost cells follow the boundary relations of Sec. III B (wall
ghost map and its linearisation), farfield ghosts are the freestream and
outflow ghosts copy the cell; the linearised ghost correction uses the
cell's correction from before the current half-sweep.
"""
from __future__ import annotations

import numpy as np

from workloads import CYCLE_F, FACE_WALL, FACE_FARFIELD, FACE_OUTFLOW, FACE_SYMMETRY
from . import gas as gm
from .mesh import restrict


def euler_flux(W, d, sign, K):
    """Euler flux T(W).n for the normal sign * e_d (W shaped (4, ...))."""
    rho = W[0]
    U = W[1] / rho
    V = W[2] / rho
    p = (2.0 / K) * (W[3] - 0.5 * rho * (U * U + V * V))
    un = sign * (U if d == 0 else V)
    nx = sign if d == 0 else 0.0
    ny = sign if d == 1 else 0.0
    return np.array([rho * un, W[1] * un + p * nx, W[2] * un + p * ny, (W[3] + p) * un])


def wall_ghost(W, wall, K):
    """Ghost state of an isothermal moving wall (Sec. III B, wall relation):
    rho_j = rho_i, (rho U)_j = 2 rho_i U_w - rho_i U_i, lambda_j = 2 lambda_w - lambda_i."""
    rho, U, V, lam = gm.primitive(W, K)
    Tw, Uw, Vw = wall[..., 0], wall[..., 1], wall[..., 2]
    Ug = 2.0 * Uw - U
    Vg = 2.0 * Vw - V
    lg = 2.0 / Tw - lam
    return gm.conservative(rho, Ug, Vg, lg, K)


def wall_jacobian(W, wall, K):
    """Linearised wall ghost map dW_j = J dW_i (Sec. III B, matrix equation), K the
    total number of degrees of freedom.  Returns J shaped (4, 4, ...)."""
    rho, U, V, lam = gm.primitive(W, K)
    Tw, Uw, Vw = wall[..., 0], wall[..., 1], wall[..., 2]
    lw = 1.0 / Tw
    Y = lam / (lam - 2.0 * lw)
    z = np.zeros_like(rho)
    o = np.ones_like(rho)
    J = np.array([
        [o, z, z, z],
        [2.0 * Uw, -o, z, z],
        [2.0 * Vw, z, -o, z],
        [2.0 * (Uw * Uw + Vw * Vw) - 0.5 * (U * U + V * V) * (1.0 + Y * Y) + K / (4.0 * lam) * (Y * Y - Y),
         U - 2.0 * Uw + U * Y * Y, V - 2.0 * Vw + V * Y * Y, -Y * Y],
    ])
    return J


class MacroLevel:
    """Per-level data of the FAS cycle: geometry from the mesh level, frozen Gamma."""

    def __init__(self, lev, gas, farfield):
        self.lev = lev
        self.gas = gas
        rho, U, V, T = farfield
        self.Winf = gm.conservative(rho, U, V, 1.0 / T, gas.K)

    def neighbour(self, W, s):
        """State across side s of every cell (neighbour or ghost), (4, Nc)."""
        lev, K = self.lev, self.gas.K
        nb, t = lev.nb[s], lev.ftype[s]
        Wn = W[:, np.maximum(nb, 0)]
        with np.errstate(all="ignore"):
            Wg = wall_ghost(W, lev.wall[s], K)
        Wj = np.where(nb >= 0, Wn, W)
        Wj = np.where(t == FACE_WALL, Wg, Wj)
        Wj = np.where(t == FACE_FARFIELD, self.Winf[:, None], Wj)
        Wj = np.where(t == FACE_SYMMETRY, mirror_state(W, s), Wj)
        return Wj

    def neighbour_correction(self, W, E, Eold, s):
        lev, K = self.lev, self.gas.K
        nb, t = lev.nb[s], lev.ftype[s]
        with np.errstate(all="ignore"):
            J = wall_jacobian(W, lev.wall[s], K)
        Eg = np.einsum("ab...,b...->a...", J, Eold)
        Ej = np.where(nb >= 0, E[:, np.maximum(nb, 0)], Eold)
        Ej = np.where(t == FACE_WALL, Eg, Ej)
        Ej = np.where(t == FACE_FARFIELD, 0.0, Ej)
        Ej = np.where(t == FACE_SYMMETRY, mirror_state(Eold, s), Ej)
        return Ej

    def freeze_gamma(self, W):
        """Gamma per cell side from the mean primitive state of the two cells."""
        lev, gas = self.lev, self.gas
        self.Gam = np.zeros((4, lev.nc))
        with np.errstate(all="ignore"):
            rho, U, V, lam = gm.primitive(W, gas.K)
            for s in range(4):
                rj, Uj, Vj, lj = gm.primitive(self.neighbour(W, s), gas.K)
                rm = 0.5 * (rho + rj)
                Um = 0.5 * (U + Uj)
                Vm = 0.5 * (V + Vj)
                Tm = 0.5 * (1.0 / lam + 1.0 / lj)
                un = np.abs(Um if s < 2 else Vm)
                a_s = np.sqrt(gas.gamma * Tm / 2.0)
                nu = gas.mu(Tm) / rm
                self.Gam[s] = np.where(lev.fluid, un + a_s + 2.0 * nu / lev.dcent[s], 0.0)

    def rsplit(self, W):
        lev, K = self.lev, self.gas.K
        out = np.zeros((4, lev.nc))
        with np.errstate(all="ignore"):
            for s in range(4):
                d, sign = s // 2, (-1.0 if s % 2 == 0 else 1.0)
                Wj = self.neighbour(W, s)
                F = 0.5 * (euler_flux(W, d, sign, K) + euler_flux(Wj, d, sign, K)
                           + self.Gam[s] * (W - Wj))
                out -= lev.S[s] * F
            out = out / lev.V
        return np.where(lev.fluid, out, 0.0)

    def smooth(self, W, P, dtn_inv):
        """One symmetric red-black sweep of the linearised defect equation; returns W + E."""
        lev, K = self.lev, self.gas.K
        Rm = P + self.rsplit(W)
        E = np.zeros_like(W)
        D = np.sum(lev.S * self.Gam, axis=0) / (2.0 * lev.V) + dtn_inv
        with np.errstate(all="ignore"):
            for col in (0, 1, 0):
                Eold = E.copy()
                acc = np.zeros_like(W)
                for s in range(4):
                    d, sign = s // 2, (-1.0 if s % 2 == 0 else 1.0)
                    Wj = self.neighbour(W, s)
                    Ej = self.neighbour_correction(W, E, Eold, s)
                    acc += lev.S[s] * (euler_flux(Wj + Ej, d, sign, K) - euler_flux(Wj, d, sign, K)
                                       - self.Gam[s] * Ej)
                Enew = (Rm - acc / (2.0 * lev.V)) / D
                m = (lev.colour == col) & lev.fluid
                E = np.where(m, Enew, E)
        return W + E


def mirror_state(W, s):
    """Mirror image of W (4, ...) across a face on side s: the momentum
    component normal to the face reversed (symmetry ghost, Sec. III B)."""
    out = np.array(W, copy=True)
    out[1 if s < 2 else 2] *= -1.0
    return out


def coarse_visits(params):
    """Parameters of the coarse-level cycles that one visit of a level makes,
    in order.  params = (nu1, nu2, nu_coarse[, gamma]): gamma > 0 gives gamma
    cycles of the same kind (1: V-cycle, 2: W-cycle); CYCLE_F gives the
    F-cycle, whose visit makes an F-cycle and then a V-cycle on the coarser
    level (each starting from the level's current iterate, as in a W-cycle)."""
    gamma = params[3] if len(params) > 3 else 1
    if gamma == CYCLE_F:
        return [params[:3] + (CYCLE_F,), params[:3] + (1,)]
    return [params] * gamma


def fas_cycle(mlevels, meshes, prolongs, l, W0, Rt, params, dtn_inv):
    """W_l^{n+1} = FAS(l, W_l^n, R_l^n) (Sec. II D, recursive FAS cycle).

    params = (nu1, nu2, nu_coarse[, gamma]): the coarse-grid corrections per
    visit of a level are those of coarse_visits (V-, W- or F-cycle)."""
    ml = mlevels[l]
    ml.freeze_gamma(W0)
    P = Rt - ml.rsplit(W0)
    W = W0.copy()
    nu1, nu2, nuc = params[:3]
    if l == len(mlevels) - 1:
        for _ in range(nuc):
            W = ml.smooth(W, P, dtn_inv[l])
        return W
    for _ in range(nu1):
        W = ml.smooth(W, P, dtn_inv[l])
    for sub in coarse_visits(params):
        Rm = P + ml.rsplit(W)
        Wc0 = restrict(meshes[l], W)
        Rc = restrict(meshes[l], Rm)
        Wc = fas_cycle(mlevels, meshes, prolongs, l + 1, Wc0, Rc, sub, dtn_inv)
        W = W + prolongs[l].apply(Wc - Wc0) * meshes[l].fluid
    for _ in range(nu2):
        W = ml.smooth(W, P, dtn_inv[l])
    return W
