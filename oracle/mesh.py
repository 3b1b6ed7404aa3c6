"""Structured mesh levels and grid-transfer operators (oracle; test infrastructure only).

Coarse levels delete every second grid line in each direction (Sec. III A);
a level has nx x ny rectangular cells, cell index c = iy * nx + ix, and its
cells are coloured c(ix, iy) = (ix + iy) mod 2 for the red-black smoothers.

Cell sides are numbered s = 0 (-x), 1 (+x), 2 (-y), 3 (+y); the outward
normal of side s points along axis s // 2 with sign -1 for even s.

A coarse face carries the tag of its two fine sub-faces (they must agree);
a coarse wall takes the area-weighted mean wall state of its sub-faces.
A coarse cell is solid when its four children are solid (mixed is an error).
"""
from __future__ import annotations

import numpy as np

from workloads import FACE_INTERIOR, FACE_WALL, FACE_FARFIELD, FACE_OUTFLOW  # noqa: F401


class Level:
    def __init__(self, xn, yn, ftx, fty, wallx, wally, solid, vel, cfl):
        self.xn = np.asarray(xn, float)
        self.yn = np.asarray(yn, float)
        self.nx = len(self.xn) - 1
        self.ny = len(self.yn) - 1
        nx, ny = self.nx, self.ny
        self.nc = nx * ny
        self.ftx, self.fty = ftx, fty
        self.wallx, self.wally = wallx, wally
        self.solid2d = solid.astype(bool)
        self.solid = self.solid2d.ravel()
        self.fluid = ~self.solid
        self.xc = 0.5 * (self.xn[1:] + self.xn[:-1])
        self.yc = 0.5 * (self.yn[1:] + self.yn[:-1])
        self.dx = np.diff(self.xn)
        self.dy = np.diff(self.yn)
        IX, IY = np.meshgrid(np.arange(nx), np.arange(ny))
        self.ix = IX.ravel()
        self.iy = IY.ravel()
        self.V = (self.dx[self.ix] * self.dy[self.iy])
        self.colour = (self.ix + self.iy) % 2
        self.cx = self.xc[self.ix]
        self.cy = self.yc[self.iy]

        # per cell side: neighbour, face tag, area, distances, wall state
        self.nb = np.full((4, self.nc), -1, np.int64)
        self.ftype = np.zeros((4, self.nc), np.int64)
        self.S = np.zeros((4, self.nc))
        self.dface = np.zeros((4, self.nc))
        self.dcent = np.zeros((4, self.nc))
        self.wall = np.zeros((4, self.nc, 3))
        for c in range(self.nc):
            i, j = self.ix[c], self.iy[c]
            sides = [
                (ftx[j, i], wallx[j, i], i - 1 >= 0 and (j, i - 1), self.dy[j], 0.5 * self.dx[i],
                 (self.xc[i] - self.xc[i - 1]) if i > 0 else 0.0),
                (ftx[j, i + 1], wallx[j, i + 1], i + 1 < nx and (j, i + 1), self.dy[j], 0.5 * self.dx[i],
                 (self.xc[i + 1] - self.xc[i]) if i + 1 < nx else 0.0),
                (fty[j, i], wally[j, i], j - 1 >= 0 and (j - 1, i), self.dx[i], 0.5 * self.dy[j],
                 (self.yc[j] - self.yc[j - 1]) if j > 0 else 0.0),
                (fty[j + 1, i], wally[j + 1, i], j + 1 < ny and (j + 1, i), self.dx[i], 0.5 * self.dy[j],
                 (self.yc[j + 1] - self.yc[j]) if j + 1 < ny else 0.0),
            ]
            for s, (t, wl, other, area, dfc, dct) in enumerate(sides):
                self.ftype[s, c] = t
                self.S[s, c] = area
                self.dface[s, c] = dfc
                self.wall[s, c] = wl
                if t == FACE_INTERIOR:
                    if not other:
                        raise ValueError("interior tag on a domain-boundary face")
                    o = other[0] * nx + other[1]
                    if not self.solid[c] and self.solid[o]:
                        raise ValueError("a face between fluid and solid cells must be a wall")
                    self.nb[s, c] = o
                    self.dcent[s, c] = dct
                else:
                    self.dcent[s, c] = 2.0 * dfc

        # interior faces, each once: L is the cell on the negative side
        fl, fr, fd = [], [], []
        for c in range(self.nc):
            if self.solid[c]:
                continue
            for s in (1, 3):
                o = self.nb[s, c]
                if o >= 0 and not self.solid[o]:
                    fl.append(c)
                    fr.append(o)
                    fd.append(s // 2)
        self.fL = np.array(fl, np.int64)
        self.fR = np.array(fr, np.int64)
        self.fdir = np.array(fd, np.int64)
        side_hi = 2 * self.fdir + 1
        self.fS = self.S[side_hi, self.fL]
        self.fdL = self.dface[side_hi, self.fL]
        self.fdR = self.dface[side_hi - 1, self.fR]

        # boundary sides of fluid cells
        bc, bs = [], []
        for c in range(self.nc):
            if self.solid[c]:
                continue
            for s in range(4):
                if self.ftype[s, c] != FACE_INTERIOR:
                    bc.append(c)
                    bs.append(s)
        self.bcell = np.array(bc, np.int64)
        self.bside = np.array(bs, np.int64)
        self.btype = self.ftype[self.bside, self.bcell] if bc else np.zeros(0, np.int64)

        # physical time step per cell (CFL condition, Sec. II A 1)
        self.dt = cfl / (vel.umax / self.dx[self.ix] + vel.vmax / self.dy[self.iy])
        self.fdt = np.minimum(self.dt[self.fL], self.dt[self.fR])

    def coarsen(self, vel, cfl):
        nx, ny = self.nx, self.ny
        if nx % 2 or ny % 2:
            raise ValueError("cannot coarsen an odd number of cells")
        NX, NY = nx // 2, ny // 2
        ftx = np.zeros((NY, NX + 1), np.int64)
        fty = np.zeros((NY + 1, NX), np.int64)
        wallx = np.zeros((NY, NX + 1, 3))
        wally = np.zeros((NY + 1, NX, 3))
        for J in range(NY):
            for I in range(NX + 1):
                a, b = self.ftx[2 * J, 2 * I], self.ftx[2 * J + 1, 2 * I]
                if a != b:
                    raise ValueError("coarse x-face with mixed tags")
                ftx[J, I] = a
                sa, sb = self.dy[2 * J], self.dy[2 * J + 1]
                wallx[J, I] = (sa * self.wallx[2 * J, 2 * I] + sb * self.wallx[2 * J + 1, 2 * I]) / (sa + sb)
        for J in range(NY + 1):
            for I in range(NX):
                a, b = self.fty[2 * J, 2 * I], self.fty[2 * J, 2 * I + 1]
                if a != b:
                    raise ValueError("coarse y-face with mixed tags")
                fty[J, I] = a
                sa, sb = self.dx[2 * I], self.dx[2 * I + 1]
                wally[J, I] = (sa * self.wally[2 * J, 2 * I] + sb * self.wally[2 * J, 2 * I + 1]) / (sa + sb)
        s4 = (self.solid2d[0::2, 0::2].astype(int) + self.solid2d[1::2, 0::2]
              + self.solid2d[0::2, 1::2] + self.solid2d[1::2, 1::2])
        if np.any((s4 > 0) & (s4 < 4)):
            raise ValueError("coarse cell with mixed solid and fluid children")
        return Level(self.xn[::2], self.yn[::2], ftx, fty, wallx, wally, s4 == 4, vel, cfl)

    def children(self):
        """(4, Nc_coarse) fine indices of the children of each coarse cell."""
        NX, NY = self.nx // 2, self.ny // 2
        I, J = np.meshgrid(np.arange(NX), np.arange(NY))
        I, J = I.ravel(), J.ravel()
        return np.array([(2 * J + a) * self.nx + 2 * I + b for a in (0, 1) for b in (0, 1)])


def build_levels(case, vel):
    lv = [Level(case.x, case.y, case.face_type_x, case.face_type_y, case.wall_x, case.wall_y,
                case.solid, vel, case.cfl)]
    for _ in range(case.n_levels - 1):
        lv.append(lv[-1].coarsen(vel, case.cfl))
    return lv


def restrict(fine: Level, q):
    """Volume-weighted mean over the four subcells (Sec. II C 1, restriction equations).

    q has the cell axis last; solid children carry zero volume weight.
    """
    ch = fine.children()
    vol = fine.V * fine.fluid
    num = sum(q[..., ch[a]] * vol[ch[a]] for a in range(4))
    den = sum(vol[ch[a]] for a in range(4))
    return num / np.where(den > 0, den, 1.0)


class Prolongation:
    """Bilinear prolongation with extrapolation (Sec. II C 3, Eqs. of I_H^h).

    For fine cell i the stencil is its parent A, the parent's neighbour B in x
    and D in y on the side of i's centre, and the diagonal C.  The weights are
    the paper's w_A = h_BC h_CD / S, w_B = h_CD h_AD / S, w_C = h_AD h_AB / S,
    w_D = h_AB h_BC / S with S = (h_AB + h_CD)(h_BC + h_AD), h being signed
    distances from i's centre to the lines joining stencil centres, negative
    on the far side of a line (extrapolation).

    Choice of partners (the paper is silent beyond boundary and corner cells):
    a partner across a non-interior coarse face (domain edge, wall) is replaced
    by the parent's neighbour on the opposite side, which turns interpolation
    into extrapolation; candidate pairs are tried in the order
    (near x, near y), (far x, near y), (near x, far y), (far x, far y) and the
    first whose diagonal cell is fluid is used; without such a pair, or without
    any valid partner in one direction, the weights are linear in the other
    direction only (constant in both as the last resort).
    """

    def __init__(self, fine: Level, coarse: Level):
        nc = fine.nc
        self.idx = np.zeros((4, nc), np.int64)
        self.w = np.zeros((4, nc))
        NX = coarse.nx
        for c in range(nc):
            if fine.solid[c]:
                self.idx[:, c] = 0
                self.w[:, c] = 0.0
                continue
            ix, iy = fine.ix[c], fine.iy[c]
            I, J = ix // 2, iy // 2
            A = J * NX + I
            x, y = fine.cx[c], fine.cy[c]
            sx = 1 if x > coarse.xc[I] else -1
            sy = 1 if y > coarse.yc[J] else -1
            side_x = {1: 1, -1: 0}
            side_y = {1: 3, -1: 2}
            cand_x = [I + d for d in (sx, -sx) if coarse.nb[side_x[d], A] >= 0]
            cand_y = [J + d for d in (sy, -sy) if coarse.nb[side_y[d], A] >= 0]
            pick = None
            for py in cand_y:
                for px in cand_x:
                    if not coarse.solid[py * NX + px]:
                        pick = (px, py)
                        break
                if pick:
                    break
            if pick is None:
                pick = (cand_x[0], None) if cand_x else ((None, cand_y[0]) if cand_y else (None, None))
            px, py = pick
            X_A, Y_A = coarse.xc[I], coarse.yc[J]
            if px is not None and py is not None:
                X_B, Y_D = coarse.xc[px], coarse.yc[py]
                ox = np.sign(X_B - X_A)
                oy = np.sign(Y_D - Y_A)
                h_AD = (x - X_A) * ox
                h_BC = (X_B - x) * ox
                h_AB = (y - Y_A) * oy
                h_CD = (Y_D - y) * oy
                S = (h_AB + h_CD) * (h_BC + h_AD)
                self.idx[:, c] = [A, J * NX + px, py * NX + px, py * NX + I]
                self.w[:, c] = [h_BC * h_CD / S, h_CD * h_AD / S, h_AD * h_AB / S, h_AB * h_BC / S]
            elif px is not None:
                X_B = coarse.xc[px]
                ox = np.sign(X_B - X_A)
                h_AD = (x - X_A) * ox
                h_BC = (X_B - x) * ox
                self.idx[:, c] = [A, J * NX + px, A, A]
                self.w[:, c] = [h_BC / (h_AD + h_BC), h_AD / (h_AD + h_BC), 0.0, 0.0]
            elif py is not None:
                Y_D = coarse.yc[py]
                oy = np.sign(Y_D - Y_A)
                h_AB = (y - Y_A) * oy
                h_CD = (Y_D - y) * oy
                self.idx[:, c] = [A, A, A, py * NX + I]
                self.w[:, c] = [h_CD / (h_AB + h_CD), 0.0, 0.0, h_AB / (h_AB + h_CD)]
            else:
                self.idx[:, c] = [A, A, A, A]
                self.w[:, c] = [1.0, 0.0, 0.0, 0.0]

    def apply(self, qc):
        """Interpolate a coarse field (cell axis last) to the fine cells."""
        return sum(self.w[a] * qc[..., self.idx[a]] for a in range(4))
