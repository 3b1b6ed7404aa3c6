"""Direct assembly of the correction equation as a sparse matrix (oracle; test infrastructure only).

Written straight from the coefficient definitions of Sec. II A 2 (upwind
defect equation, D_ik and D_jk), the diffuse-wall ghost of Sec. III B
(dF_j,k = C_k drho_j with drho_j fixed by zero normal mass flux through the
wall) and the symmetry ghost (dF_j,k = dF_i,k' at the velocity with the
normal component reversed), independently of the smoother code, so that a direct sparse solve
pins the multigrid correction cycle.

Unknown ordering: index (s, k, c) -> (s * Nk + k) * Nc + c, s = 0 for G and
1 for H.  Rows of solid cells are identity rows.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads import FACE_INTERIOR, FACE_WALL, FACE_OUTFLOW, FACE_SYMMETRY
from .flux import wall_maxwellian


def assemble(lev, vel, K_int, tau_inv, dtn_inv=None):
    nk, nc = vel.n, lev.nc
    if dtn_inv is None:
        dtn_inv = np.zeros(nc)

    def idx(s, k, c):
        return (s * nk + k) * nc + c

    rows, cols, vals = [], [], []

    def put(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    for c in range(nc):
        if lev.solid[c]:
            for s in range(2):
                for k in range(nk):
                    put(idx(s, k, c), idx(s, k, c), 1.0)
            continue
        V = lev.V[c]
        for k in range(nk):
            diag = tau_inv[c] + dtn_inv[c]
            offd = []            # (column, value) pairs shared by G and H rows
            wall = []            # (side, un, S) of incoming wall sides
            sym = []             # (mirror velocity, coefficient) of incoming symmetry sides
            for side in range(4):
                sign = -1.0 if side % 2 == 0 else 1.0
                un = sign * (vel.u[k] if side < 2 else vel.v[k])
                S = lev.S[side, c]
                t = lev.ftype[side, c]
                # (1/2V) u_n S (1 + sgn u_n) on the diagonal
                diag += 0.5 / V * un * S * (1.0 + np.sign(un))
                # (1/2V) u_n S (1 - sgn u_n) on the neighbour / ghost
                dj = 0.5 / V * un * S * (1.0 - np.sign(un))
                if dj == 0.0:
                    continue
                if t == FACE_INTERIOR:
                    offd.append((lev.nb[side, c], dj))
                elif t == FACE_OUTFLOW:
                    diag += dj          # ghost copies the cell
                elif t == FACE_WALL:
                    wall.append((side, dj))
                elif t == FACE_SYMMETRY:
                    # ghost correction = the cell's own at the mirror velocity
                    sym.append((vel.mirror(side // 2)[k], dj))
                # farfield: the ghost correction vanishes
            for s in range(2):
                put(idx(s, k, c), idx(s, k, c), diag)
                for o, dj in offd:
                    put(idx(s, k, c), idx(s, k, o), dj)
                for km, dj in sym:
                    put(idx(s, k, c), idx(s, km, c), dj)
            for side, dj in wall:
                Tw, Uw, Vw = lev.wall[side, c]
                CG, CH = wall_maxwellian(Tw, Uw, Vw, vel.u, vel.v, K_int)
                sign = -1.0 if side % 2 == 0 else 1.0
                unk = sign * (vel.u if side < 2 else vel.v)
                den = np.sum(vel.w[unk < 0] * unk[unk < 0] * CG[unk < 0])
                for kp in np.nonzero(unk > 0)[0]:
                    coeff = -vel.w[kp] * unk[kp] / den     # d(drho)/d(dG_kp)
                    put(idx(0, k, c), idx(0, kp, c), dj * CG[k] * coeff)
                    put(idx(1, k, c), idx(0, kp, c), dj * CH[k] * coeff)
    n = 2 * nk * nc
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
