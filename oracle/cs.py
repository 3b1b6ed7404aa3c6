"""CS V-cycle of the microscopic correction (oracle; test infrastructure only).

Step 5 of the outer iteration (Sec. II D) solves the linear correction
equation of the distribution (Sec. II A 2, upwind defect equation and its
coefficients):

  D_ik e_ik + sum_j D_jk e_jk = r_ik,
  D_ik = 1/tau_i + (1/2V_i) sum_j u_kn S_ij (1 + sgn u_kn)  (+ 1/dt_n),
  D_jk = (1/2V_i) u_kn S_ij (1 - sgn u_kn),

for the reduced pair (G, H) with the correction scheme of Sec. II D (CS steps
(a)-(c)): pre-smoothing, restriction of the renewed residual
r - A dF (algebraically the same as the accumulated form of Sec. II C 2),
recursion, bilinear prolongation of the coarse correction, post-smoothing.
The smoother is the Gauss-Seidel (LU-SGS) sweep of Sec. II A 2 taken, for
every discrete velocity, in that velocity's upwind cell order; for the upwind
operator this sweep is an exact solve of the transport part, as the
lexicographic LU-SGS sweep is for the velocities aligned with it.

Boundary ghosts (Sec. III B): a diffuse wall returns C_k drho_w with drho_w
from zero net mass flux of the correction through the wall, recomputed from
the current correction before every half-sweep and before the renewal; a
farfield ghost carries no correction; an outflow ghost copies the cell,
which moves its inflow term onto the diagonal.

Coarse levels use the coarse geometry, the volume-weighted mean collision
frequency of the fine cells and the pseudo step from the coarse CFL step.
"""
from __future__ import annotations

import numpy as np

from workloads import FACE_WALL, FACE_OUTFLOW, FACE_SYMMETRY
from .flux import wall_maxwellian
from .fas import coarse_visits
from .mesh import restrict


class MicroLevel:
    """Per-level operator of the correction equation for all velocities.

    For velocity k and cell i each axis has one upwind side (the side whose
    outward normal speed is negative).  Across it the correction is the
    neighbour's (interior face), C_k drho_w (wall), zero (farfield), the
    cell's own (outflow, folded into the diagonal) or the cell's own at the
    velocity with the normal component reversed (symmetry face).
    """

    def __init__(self, lev, vel, K_int):
        self.lev = lev
        self.vel = vel
        nk = vel.n
        self.un = np.zeros((4, nk, 1))
        for s in range(4):
            sign = -1.0 if s % 2 == 0 else 1.0
            self.un[s, :, 0] = sign * (vel.u if s < 2 else vel.v)
        self.coef = lev.S / lev.V                      # (4, Nc)
        self.outflow = lev.ftype == FACE_OUTFLOW       # (4, Nc)
        self.interior = lev.nb >= 0
        self.sym = lev.ftype == FACE_SYMMETRY
        self.mirror = [vel.mirror(0), vel.mirror(1)] if self.sym.any() else None
        # transport part of the diagonal: outgoing normal speeds; outflow faces
        # add their (negative) inflow speeds as well
        diag = np.zeros((nk, lev.nc))
        for s in range(4):
            a = np.where(self.outflow[s], self.un[s], np.maximum(self.un[s], 0.0))
            diag += self.coef[s] * a
        self.diag = diag
        # wall sides of fluid cells
        m = (lev.btype == FACE_WALL)
        self.wcell = lev.bcell[m]
        self.wside = lev.bside[m]
        nw = len(self.wcell)
        self.widx = np.full((4, lev.nc), -1, np.int64)
        self.widx[self.wside, self.wcell] = np.arange(nw)
        self.CG = np.zeros((nk, nw))
        self.CH = np.zeros((nk, nw))
        self.den = np.zeros(nw)
        for j in range(nw):
            Tw, Uw, Vw = lev.wall[self.wside[j], self.wcell[j]]
            CG, CH = wall_maxwellian(Tw, Uw, Vw, vel.u, vel.v, K_int)
            un = self.un[self.wside[j], :, 0]
            self.CG[:, j] = CG
            self.CH[:, j] = CH
            self.den[j] = np.sum((vel.w * un * CG)[un < 0])
        # upwind side per axis and velocity: side 0 (-x) when u >= 0, else side 1
        self.upx = np.where(vel.u >= 0, 0, 1)
        self.upy = np.where(vel.v >= 0, 2, 3)

    def wall_drho(self, dG):
        """drho_w = -sum_{u_n>0} w u_n dG_i / sum_{u_n<0} w u_n C_k (Sec. III B)."""
        out = np.zeros(len(self.wcell))
        for j in range(len(self.wcell)):
            un = self.un[self.wside[j], :, 0]
            out[j] = -np.sum((self.vel.w * un * dG[:, self.wcell[j]])[un > 0]) / self.den[j]
        return out

    def upwind_term(self, kq, c, s, dG, dH, drho, mG, mH):
        """D_jk times the correction across side s of cell c for velocities kq;
        a symmetry ghost reads the mirror velocity's correction in mG, mH."""
        un = self.un[s, kq, 0]
        w = self.coef[s, c] * np.where(un < 0, un, 0.0)
        if self.interior[s, c]:
            o = self.lev.nb[s, c]
            return w * dG[kq, o], w * dH[kq, o]
        if self.sym[s, c]:
            mk = self.mirror[s // 2][kq]
            return w * mG[mk, c], w * mH[mk, c]
        j = self.widx[s, c]
        if j >= 0:
            return w * self.CG[kq, j] * drho[j], w * self.CH[kq, j] * drho[j]
        return 0.0 * w, 0.0 * w

    def diagonal(self, tau_inv, dtn_inv):
        return tau_inv + dtn_inv + self.diag

    def quadrants(self):
        u, v = self.vel.u, self.vel.v
        for sx in (1, -1):
            for sy in (1, -1):
                kq = np.nonzero(((u >= 0) if sx > 0 else (u < 0)) & ((v >= 0) if sy > 0 else (v < 0)))[0]
                if len(kq):
                    yield sx, sy, kq

    def smooth(self, dG, dH, rG, rH, D):
        """One Gauss-Seidel sweep of every velocity in its own upwind order.

        The wall densities and the symmetry ghosts (a cell's own correction at
        the mirror velocity) are taken from the correction before the sweep;
        each cell then uses its already-updated upwind neighbours, so the
        sweep solves the transport part of the equation exactly.  The cells
        are visited row by row here; any order that visits upwind neighbours
        first (such as the anti-diagonal wavefronts of the GPU) gives the
        same arithmetic.
        """
        lev = self.lev
        drho = self.wall_drho(dG)
        nG = np.zeros_like(dG)
        nH = np.zeros_like(dH)
        for sx, sy, kq in self.quadrants():
            xs = range(lev.nx) if sx > 0 else range(lev.nx - 1, -1, -1)
            ys = range(lev.ny) if sy > 0 else range(lev.ny - 1, -1, -1)
            sxs = self.upx[kq[0]]
            sys_ = self.upy[kq[0]]
            for iy in ys:
                for ix in xs:
                    c = iy * lev.nx + ix
                    if lev.solid[c]:
                        continue
                    txG, txH = self.upwind_term(kq, c, sxs, nG, nH, drho, dG, dH)
                    tyG, tyH = self.upwind_term(kq, c, sys_, nG, nH, drho, dG, dH)
                    nG[kq, c] = (rG[kq, c] - txG - tyG) / D[kq, c]
                    nH[kq, c] = (rH[kq, c] - txH - tyH) / D[kq, c]
        return nG, nH

    def defect(self, dG, dH, rG, rH, D):
        """r - A dF with the wall densities of dF itself."""
        lev = self.lev
        drho = self.wall_drho(dG)
        eG = np.zeros_like(dG)
        eH = np.zeros_like(dH)
        for sx, sy, kq in self.quadrants():
            sxs = self.upx[kq[0]]
            sys_ = self.upy[kq[0]]
            for c in range(lev.nc):
                if lev.solid[c]:
                    continue
                txG, txH = self.upwind_term(kq, c, sxs, dG, dH, drho, dG, dH)
                tyG, tyH = self.upwind_term(kq, c, sys_, dG, dH, drho, dG, dH)
                eG[kq, c] = rG[kq, c] - D[kq, c] * dG[kq, c] - txG - tyG
                eH[kq, c] = rH[kq, c] - D[kq, c] * dH[kq, c] - txH - tyH
        return eG, eH


def cs_cycle(mlevels, meshes, prolongs, l, rG, rH, tau_inv, dtn_inv, params):
    """dF_l = CS(l, r_l) (Sec. II D, recursive CS cycle); tau_inv, dtn_inv per level."""
    ml = mlevels[l]
    D = ml.diagonal(tau_inv[l], dtn_inv[l])
    dG = np.zeros_like(rG)
    dH = np.zeros_like(rH)
    nu1, nu2, nuc = params[:3]
    if l == len(mlevels) - 1:
        for _ in range(nuc):
            dG, dH = ml.smooth(dG, dH, rG, rH, D)
        return dG, dH
    for _ in range(nu1):
        dG, dH = ml.smooth(dG, dH, rG, rH, D)
    fl = meshes[l].fluid
    # coarse corrections per visit: V-, W- or F-cycle (coarse_visits)
    for sub in coarse_visits(params):
        eG, eH = ml.defect(dG, dH, rG, rH, D)
        cG, cH = cs_cycle(mlevels, meshes, prolongs, l + 1, restrict(meshes[l], eG),
                          restrict(meshes[l], eH), tau_inv, dtn_inv, sub)
        dG = dG + prolongs[l].apply(cG) * fl
        dH = dH + prolongs[l].apply(cH) * fl
    for _ in range(nu2):
        dG, dH = ml.smooth(dG, dH, rG, rH, D)
    return dG, dH
