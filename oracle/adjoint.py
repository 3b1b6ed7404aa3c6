"""Wall loads of a steady state and their sensitivity to the wall temperatures
(oracle; test infrastructure only).

The steady state solves the microscopic residual of Steps 3-4 with the
equilibrium of the state itself (Sec. II A, the residual r(f) that the cycle
drives to zero once the prediction returns W unchanged):

    r_ik(f; Tw) = (g_ik(W_i(f), q_i(f)) - f_ik) / tau_i(W_i(f)) - div_ik(f; Tw),

with the Shakhov g, the moments W and heat flux q of f, and the transport
div of Step 1, whose diffuse walls depend on their temperatures Tw through
the wall Maxwellians C_k and the wall densities (Sec. III B).  A closed
domain keeps its total mass (the renormalisation of the update).

Wall loads (the momentum and energy the gas hands to a wall per unit area,
Sec. IV B, the skin friction from the momentum transferred to the wall) are
taken from the distribution on the wall side of the face, in the frame of
the wall (c = u - U_w): pressure p = sum_k w c_n^2 f^G, shear
tau = sum_k w c_t c_n f^G with c_t the component along the face (x on a
y-face, y on an x-face), heat flux q = 1/2 sum_k w c_n (|c|^2 f^G + f^H);
c_n is the velocity along the normal pointing out of the gas.  An objective
is J = sum_j S_j load_j over chosen wall sides.

The sensitivity is formed here by its plain definition: the exact Jacobians
of r by complex steps (every operation of the residual continues
analytically; the limiter's branches follow the real part), the tangent
df/dTw from the linearised state equation, with the mass constraint of a
closed domain appended as one more row (least squares on the consistent
system), and dJ/dTw = dJ/df df/dTw + dJ/dTw|_f.  Sizes suit a few dozen cells.
"""
from __future__ import annotations

import copy

import numpy as np

from workloads import FACE_WALL
from . import gas as gm
from .flux import boundary_face_values, residuals

LOAD_PRESSURE, LOAD_SHEAR, LOAD_HEAT = 0, 1, 2


def steady_residual(G, H, lev, vel, gas, farfield):
    """r(f) for G and H (Nk, Nc), zero on solid cells."""
    fl = lev.fluid
    u = vel.u[:, None]
    v = vel.v[:, None]
    W = gm.moments(G, H, vel)
    with np.errstate(all="ignore"):
        rho, U, V, lam = gm.primitive(W, gas.K)
        q = gm.heat_flux(G, H, vel, U, V)
        tau_inv = np.where(fl, 1.0 / gas.tau(rho, lam), 0.0)
        Gt, Ht = gm.shakhov(rho, U, V, lam, q[0], q[1], u, v, gas.K_int, gas.Pr)
    W = np.where(fl, W, 0.0)
    divG, divH, _ = residuals(G, H, W, lev, vel, gas, farfield)
    rG = np.where(fl, (Gt - G) * tau_inv - divG, 0.0)
    rH = np.where(fl, (Ht - H) * tau_inv - divH, 0.0)
    return rG, rH


def wall_list(lev):
    """Indices into the boundary sides of lev that are walls, in the order of
    their cells and then of the sides (-x, +x, -y, +y)."""
    return np.nonzero(lev.btype == FACE_WALL)[0]


def wall_loads(G, H, lev, vel, gas, farfield):
    """(p, tau, q, S) per wall side, in the order of wall_list."""
    un, Gf, Hf = boundary_face_values(G, H, lev, vel, gas, farfield)
    js = wall_list(lev)
    out = np.zeros((4, len(js)), dtype=Gf.dtype)
    for n, j in enumerate(js):
        c, s = lev.bcell[j], lev.bside[j]
        Tw, Uw, Vw = lev.wall[s, c]
        cx = vel.u - Uw
        cy = vel.v - Vw
        sign = -1.0 if s % 2 == 0 else 1.0
        cn = sign * (cx if s < 2 else cy)
        ct = cy if s < 2 else cx
        w = vel.w
        out[0, n] = np.sum(w * cn * cn * Gf[:, j])
        out[1, n] = np.sum(w * ct * cn * Gf[:, j])
        out[2, n] = 0.5 * np.sum(w * cn * ((cx * cx + cy * cy) * Gf[:, j] + Hf[:, j]))
        out[3, n] = lev.S[s, c]
    return out


def objective(G, H, lev, vel, gas, farfield, kind, ids):
    """J = sum over the wall sides ids of S_j load_j (load: LOAD_PRESSURE,
    LOAD_SHEAR or LOAD_HEAT)."""
    ld = wall_loads(G, H, lev, vel, gas, farfield)
    ids = np.asarray(ids, np.int64)
    return np.sum(ld[3, ids] * ld[kind, ids])


def face_sides(lev, nx, ny, face):
    """(side, cell) pairs of lev's fluid cells that lie on a face of the mesh,
    numbered x-faces first (iy (nx + 1) + ix), then y-faces ((nx + 1) ny +
    iy nx + ix)."""
    nfx = (nx + 1) * ny
    out = []
    if face < nfx:
        iy, ix = divmod(face, nx + 1)
        for s, i in ((1, ix - 1), (0, ix)):
            if 0 <= i < nx:
                out.append((s, iy * nx + i))
    else:
        iy, ix = divmod(face - nfx, nx)
        for s, j in ((3, iy - 1), (2, iy)):
            if 0 <= j < ny:
                out.append((s, j * nx + ix))
    return [(s, c) for s, c in out if not lev.solid[c] and lev.ftype[s, c] == FACE_WALL]


class Sensitivity:
    """Dense linearisation of the steady state of an Oracle at its current f
    (the finest level only: coarse levels do not enter the steady state)."""

    def __init__(self, o):
        self.o = o
        self.lev = o.lev0
        self.cols = np.nonzero(self.lev.fluid)[0]
        self.nk = o.vel.n

    # f restricted to fluid cells, (G, H) stacked
    def pack(self, G, H):
        return np.concatenate([G[:, self.cols].ravel(), H[:, self.cols].ravel()])

    def unpack(self, x):
        n = self.nk * len(self.cols)
        dtype = x.dtype
        G = np.zeros((self.nk, self.lev.nc), dtype=dtype)
        H = np.zeros((self.nk, self.lev.nc), dtype=dtype)
        G[:, self.cols] = x[:n].reshape(self.nk, -1)
        H[:, self.cols] = x[n:].reshape(self.nk, -1)
        return G, H

    def _lev_with_walls(self, dT):
        """A copy of the finest level with wall temperatures Tw + dT (dT per
        (side, cell), complex allowed)."""
        lev = copy.copy(self.lev)
        lev.wall = np.array(self.lev.wall, dtype=np.result_type(self.lev.wall, dT))
        lev.wall[:, :, 0] += dT
        return lev

    def residual(self, x, lev=None):
        G, H = self.unpack(x)
        o = self.o
        rG, rH = steady_residual(G, H, lev or self.lev, o.vel, o.gas, o.case.farfield)
        return self.pack(rG, rH)

    def jacobian(self, h=1e-30):
        """dr/df (n x n), one complex step per column."""
        x0 = self.pack(self.o.G, self.o.H).astype(complex)
        n = x0.size
        J = np.empty((n, n))
        for j in range(n):
            x = x0.copy()
            x[j] += 1j * h
            J[:, j] = self.residual(x).imag / h
        return J

    def mass_row(self):
        """m with m . f = total mass (sum over cells of V_i sum_k w_k G_ik)."""
        lev, vel = self.lev, self.o.vel
        mG = (vel.w[:, None] * lev.V[None, self.cols]).ravel()
        return np.concatenate([mG, np.zeros_like(mG)])

    def wall_perturbation(self, faces, h):
        """dT per (side, cell) for a step h on the listed mesh faces."""
        case = self.o.case
        dT = np.zeros((4, self.lev.nc), dtype=complex)
        for f in faces:
            for s, c in face_sides(self.lev, case.nx, case.ny, f):
                dT[s, c] += h
        return dT

    def dr_dT(self, faces, h=1e-30):
        """dr/dTw per listed face (n x nfaces)."""
        x0 = self.pack(self.o.G, self.o.H).astype(complex)
        out = np.empty((x0.size, len(faces)))
        for m, f in enumerate(faces):
            lev = self._lev_with_walls(self.wall_perturbation([f], 1j * h))
            out[:, m] = self.residual(x0, lev).imag / h
        return out

    def objective(self, x, kind, ids, lev=None):
        G, H = self.unpack(x)
        o = self.o
        return objective(G, H, lev or self.lev, o.vel, o.gas, o.case.farfield, kind, ids)

    def dJ_df(self, kind, ids, h=1e-30):
        x0 = self.pack(self.o.G, self.o.H).astype(complex)
        g = np.empty(x0.size)
        for j in range(x0.size):
            x = x0.copy()
            x[j] += 1j * h
            g[j] = self.objective(x, kind, ids).imag / h
        return g

    def dJ_dT(self, kind, ids, faces, h=1e-30):
        x0 = self.pack(self.o.G, self.o.H).astype(complex)
        return np.array([self.objective(x0, kind, ids, self._lev_with_walls(self.wall_perturbation([f], 1j * h))).imag / h
                         for f in faces])

    def tangent(self, J, B):
        """df/dTw: J df = -B, plus m . df = 0 in a closed domain."""
        if self.o.closed:
            A = np.vstack([J, self.mass_row()[None, :]])
            rhs = np.vstack([-B, np.zeros((1, B.shape[1]))])
            return np.linalg.lstsq(A, rhs, rcond=None)[0]
        return np.linalg.solve(J, -B)

    def gradient(self, kind, ids, faces):
        """dJ/dTw for the listed mesh faces at the current (steady) state."""
        J = self.jacobian()
        B = self.dr_dT(faces)
        T = self.tangent(J, B)
        return self.dJ_df(kind, ids) @ T + self.dJ_dT(kind, ids, faces)
