"""Synthetic workload recipes and seeded input generators.

This module holds inputs only: mesh node lines, boundary tags, wall and
freestream states, gas constants as plain numbers, the velocity-grid recipe
(kind, size, range) and seeded random fields for parity tests.  It contains
none of the scheme's arithmetic (no equilibrium, flux, smoother or quadrature
formula), so both the CPU oracle and the GPU library can consume it without
sharing any part of the method.

Units are nondimensional: lengths by the reference length (cavity side, plate
length or square side), density by the reference density, temperature by T0
and speeds by sqrt(2 R T0).  In these units a Mach number M at temperature 1
corresponds to a speed M * sqrt(gamma / 2).

The five cases mirror the paper's three workloads (Sec. IV: lid-driven cavity,
finite flat plate, Mach-5 square cylinder) at synthetic sizes; none of the
paper's meshes or reference data are reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Boundary tags of a face (data format shared by the oracle and the library).
FACE_INTERIOR = 0
FACE_WALL = 1
FACE_FARFIELD = 2
FACE_OUTFLOW = 3
FACE_SYMMETRY = 4   # specular reflection: the mirror image of the cell (Sec. III B)

# Value of cycle_gamma / cycle_gamma_cs that selects F-cycles (data format
# shared by the oracle and the library).
CYCLE_F = -1

QUAD_TRAPEZOID = "trapezoid"
QUAD_SIMPSON38 = "simpson38"
QUAD_GAUSS_HERMITE = "gauss_hermite"


@dataclasses.dataclass
class Case:
    """One steady-flow problem in the input format of both solvers.

    Cell (ix, iy) spans [x[ix], x[ix+1]] x [y[iy], y[iy+1]].  The x-face
    (ix, iy) lies on the line x = x[ix] between cells (ix-1, iy) and (ix, iy);
    the y-face (ix, iy) lies on y = y[iy] between cells (ix, iy-1) and (ix, iy).
    """

    name: str
    x: np.ndarray                 # (nx+1,) node coordinates
    y: np.ndarray                 # (ny+1,)
    face_type_x: np.ndarray       # (ny, nx+1) uint8
    face_type_y: np.ndarray       # (ny+1, nx) uint8
    wall_x: np.ndarray            # (ny, nx+1, 3) wall (T, U, V) of WALL x-faces
    wall_y: np.ndarray            # (ny+1, nx, 3)
    solid: np.ndarray             # (ny, nx) uint8, 1 = solid cell
    n_levels: int
    quad: str                     # velocity quadrature kind
    nu: int
    nv: int
    vlo: float                    # velocity range (trapezoid / Simpson rules)
    vhi: float
    K_int: int                    # internal degrees of freedom
    Pr: float
    omega: float                  # viscosity temperature exponent
    Kn: float
    farfield: tuple               # (rho, U, V, T) of the freestream
    init: np.ndarray              # (4, ny, nx) initial (rho, U, V, T)
    precision: str = "fp64"       # "fp64" or "fp32f"
    dtn_growth: float = 0.0       # a in dt_n = a^n dt_p; 0 disables the pseudo step
    dtn_max: float = 0.0          # cap of a^n (0: none)
    nu1: int = 2
    nu2: int = 1
    nu_coarse: int = 10
    cfl: float = 0.8
    fas_levels: int = 0           # levels of the FAS prediction (0: all n_levels)
    nu_coarse_cs: int = 0         # CS smoothings on the coarsest level (0: nu_coarse)
    cycle_gamma: int = 1          # coarse corrections per level visit (1: V-cycle, 2: W-cycle,
                                  # CYCLE_F: F-cycle), FAS
    cycle_gamma_cs: int = 0       # the same for the CS cycle (0: cycle_gamma)

    @property
    def nx(self) -> int:
        return len(self.x) - 1

    @property
    def ny(self) -> int:
        return len(self.y) - 1

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny

    @property
    def n_fluid(self) -> int:
        return int((self.solid == 0).sum())

    @property
    def n_vel(self) -> int:
        return self.nu * self.nv

    def closed(self) -> bool:
        """True when no face lets mass in or out (walls only)."""
        return not (np.isin(self.face_type_x, (FACE_FARFIELD, FACE_OUTFLOW)).any()
                    or np.isin(self.face_type_y, (FACE_FARFIELD, FACE_OUTFLOW)).any())

    def with_(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# node-line recipes
# ----------------------------------------------------------------------------

def _bisect(fun, lo, hi, iters=200):
    flo = fun(lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = fun(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def tanh_two_sided(n: int, first: float) -> np.ndarray:
    """n cells on [0, 1] clustered at both ends, first cell of width `first`."""
    s = np.arange(n + 1) / n

    def width(beta):
        return 0.5 * (1.0 - math.tanh(beta * (1.0 - 2.0 / n)) / math.tanh(beta)) - first

    beta = _bisect(width, 1e-6, 20.0)
    x = 0.5 * (1.0 + np.tanh(beta * (2.0 * s - 1.0)) / math.tanh(beta))
    x[0], x[-1] = 0.0, 1.0
    return x


def tanh_one_sided(n: int, first: float) -> np.ndarray:
    """n cells on [0, 1] clustered at x = 1, last cell of width `first`."""
    s = np.arange(n + 1) / n
    if first * n >= 1.0:
        return s

    def width(beta):
        return 1.0 - math.tanh(beta * (1.0 - 1.0 / n)) / math.tanh(beta) - first

    beta = _bisect(width, 1e-6, 50.0)
    x = np.tanh(beta * s) / math.tanh(beta)
    x[0], x[-1] = 0.0, 1.0
    return x


def _blank(nx, ny):
    ftx = np.zeros((ny, nx + 1), np.uint8)
    fty = np.zeros((ny + 1, nx), np.uint8)
    wx = np.zeros((ny, nx + 1, 3))
    wy = np.zeros((ny + 1, nx, 3))
    return ftx, fty, wx, wy


def lid_speed(mach: float, gamma: float) -> float:
    """Wall speed of a given Mach number at unit temperature."""
    return mach * math.sqrt(gamma / 2.0)


# ----------------------------------------------------------------------------
# the cases
# ----------------------------------------------------------------------------

ARGON = dict(K_int=1, Pr=2.0 / 3.0, omega=0.81)
AIR = dict(K_int=3, Pr=0.72, omega=0.77)


def cavity(n=16, first=None, Kn=10.0, mach=0.16, n_levels=2, quad=QUAD_TRAPEZOID,
           nvel=16, vlo=-4.0, vhi=4.0, precision="fp64", name=None, wall_T_bottom=None,
           ny=None, nvel_y=None, **kw) -> Case:
    """Lid-driven cavity on [0,1]^2: diffuse walls at T = 1, top lid moving in +x.

    n (and optionally ny) cells, nvel (and optionally nvel_y) velocities per
    axis; `wall_T_bottom` optionally gives one wall temperature per bottom face.
    """
    nx = n
    ny = n if ny is None else ny
    xn = np.linspace(0.0, 1.0, nx + 1) if first is None else tanh_two_sided(nx, first)
    yn = np.linspace(0.0, 1.0, ny + 1) if first is None else tanh_two_sided(ny, first)
    ftx, fty, wx, wy = _blank(nx, ny)
    ftx[:, 0] = ftx[:, nx] = FACE_WALL
    fty[0, :] = fty[ny, :] = FACE_WALL
    gamma = (ARGON["K_int"] + 4.0) / (ARGON["K_int"] + 2.0)
    wx[:, 0, 0] = wx[:, nx, 0] = 1.0
    wy[0, :, 0] = 1.0 if wall_T_bottom is None else np.asarray(wall_T_bottom, float)
    wy[ny, :, 0] = 1.0
    wy[ny, :, 1] = lid_speed(mach, gamma)
    init = np.zeros((4, ny, nx))
    init[0] = 1.0
    init[3] = 1.0
    return Case(name=name or f"cavity{nx}x{ny}", x=xn.copy(), y=yn.copy(), face_type_x=ftx,
                face_type_y=fty, wall_x=wx, wall_y=wy, solid=np.zeros((ny, nx), np.uint8),
                n_levels=n_levels, quad=quad, nu=nvel, nv=nvel if nvel_y is None else nvel_y,
                vlo=vlo, vhi=vhi, Kn=Kn, farfield=(1.0, 0.0, 0.0, 1.0), init=init,
                precision=precision, **ARGON, **kw)


def sheared_half_box(n=8, ny=None, Kn=1.0, mach=0.3, **kw) -> Case:
    """A box with two symmetry planes: specular reflection on the left side
    and the top, diffuse walls at T = 1 on the right side and the bottom,
    which moves in +x (the cavity builder's cells and velocity grids)."""
    case = cavity(n=n, ny=ny, Kn=Kn, mach=mach, name=kw.pop("name", None) or "sheared_half_box", **kw)
    gamma = (ARGON["K_int"] + 4.0) / (ARGON["K_int"] + 2.0)
    case.face_type_x[:, 0] = FACE_SYMMETRY
    case.face_type_y[case.ny, :] = FACE_SYMMETRY
    case.wall_x[:, 0] = 0.0
    case.wall_y[case.ny] = 0.0
    case.wall_y[0, :, 1] = lid_speed(mach, gamma)
    return case


def symmetric_channel(n=6, ny=None, U=0.3, **kw) -> Case:
    """A straight channel in a uniform freestream (rho 1, U, 0, T 1): farfield
    ends, symmetry planes on both sides; the freestream is its steady state."""
    case = cavity(n=n, ny=ny, name=kw.pop("name", None) or "symmetric_channel", **kw)
    case.face_type_x[:, 0] = case.face_type_x[:, case.nx] = FACE_FARFIELD
    case.face_type_y[0, :] = case.face_type_y[case.ny, :] = FACE_SYMMETRY
    case.wall_x[:] = 0.0
    case.wall_y[:] = 0.0
    case.farfield = (1.0, U, 0.0, 1.0)
    case.init[1] = U
    return case


def free_molecular_gap(n=6, ny=4, T_bottom=1.1, T_top=0.9, Kn=1e12, **kw) -> Case:
    """Gas at rest between two diffuse plates at different temperatures
    (bottom and top), specular sides, Kn so large that collisions vanish."""
    case = cavity(n=n, ny=ny, Kn=Kn, mach=0.0, name=kw.pop("name", None) or "free_molecular_gap", **kw)
    case.face_type_x[:, 0] = case.face_type_x[:, case.nx] = FACE_SYMMETRY
    case.wall_x[:] = 0.0
    case.wall_y[0, :, 0] = T_bottom
    case.wall_y[case.ny, :, 0] = T_top
    case.wall_y[:, :, 1:] = 0.0
    return case


def config1(**kw) -> Case:
    """Cavity 16x16 uniform, 16x16 trapezoid on [-4,4]^2, Kn 10, lid Mach 0.16, 2 levels."""
    args = dict(n=16, Kn=10.0, n_levels=2, quad=QUAD_TRAPEZOID, nvel=16, vlo=-4.0, vhi=4.0,
                precision="fp64", name="cavity16_kn10")
    args.update(kw)
    return cavity(**args)


def config2(**kw) -> Case:
    """Cavity 64x64 tanh-clustered (first cell 0.005), 28x28 Gauss-Hermite, Kn 0.075, 4 levels."""
    args = dict(n=64, first=0.005, Kn=0.075, n_levels=4, quad=QUAD_GAUSS_HERMITE, nvel=28,
                vlo=0.0, vhi=0.0, precision="fp32f", name="cavity64_kn0.075", nu_coarse_cs=2)
    args.update(kw)
    return cavity(**args)


def config5(seed=1704, **kw) -> Case:
    """Config 2 at Kn 0.1 with 64 seeded bottom-wall temperatures 1 + U(-0.05, 0.05)."""
    rng = np.random.default_rng(seed)
    tw = 1.0 + rng.uniform(-0.05, 0.05, 64)
    args = dict(Kn=0.1, wall_T_bottom=tw, name="cavity64_kn0.1_adjoint")
    args.update(kw)
    return config2(**args)


def flat_plate(scale=1, **kw) -> Case:
    """Zero-thickness plate y = 15, x in [19.5, 20.5] inside [0,40] x [0,30].

    scale=1 gives 128 x 96 cells; the plate edges sit on node indices that are
    multiples of 8 so that every level of a 4-level hierarchy keeps them.
    Farfield on all four sides, diffuse plate at the freestream temperature.
    The 40 x 40 Newton-Cotes velocity grid on [-5, 5]^2 is the composite
    closed two-point Newton-Cotes (trapezoid) rule on equally spaced nodes.
    """
    n_side, n_mid, n_y = 56 // scale, 16 // scale, 48 // scale
    h = 1.0 / n_mid
    left = 19.5 * tanh_one_sided(n_side, h / 19.5)
    mid = 19.5 + np.arange(1, n_mid + 1) * h
    right = 40.0 - left[::-1]
    x = np.concatenate([left, mid, right[1:]])
    lower = 15.0 * tanh_one_sided(n_y, 0.01 * scale / 15.0)
    y = np.concatenate([lower, 30.0 - lower[::-1][1:]])
    nx, ny = len(x) - 1, len(y) - 1
    ftx, fty, wx, wy = _blank(nx, ny)
    ftx[:, 0] = ftx[:, nx] = FACE_FARFIELD
    fty[0, :] = fty[ny, :] = FACE_FARFIELD
    fty[n_y, n_side:n_side + n_mid] = FACE_WALL
    wy[n_y, n_side:n_side + n_mid, 0] = 1.0
    gamma = (AIR["K_int"] + 4.0) / (AIR["K_int"] + 2.0)
    uinf = lid_speed(0.1, gamma)
    init = np.zeros((4, ny, nx))
    init[0], init[1], init[3] = 1.0, uinf, 1.0
    args = dict(name=f"plate{nx}x{ny}", x=x, y=y, face_type_x=ftx, face_type_y=fty,
                wall_x=wx, wall_y=wy, solid=np.zeros((ny, nx), np.uint8), n_levels=4,
                quad=QUAD_TRAPEZOID, nu=40, nv=40, vlo=-5.0, vhi=5.0, Kn=0.1,
                farfield=(1.0, uinf, 0.0, 1.0), init=init, precision="fp32f", nu_coarse_cs=2, **AIR)
    args.update(kw)
    return Case(**args)


def config3(**kw) -> Case:
    return flat_plate(**kw)


def square_cylinder(scale=1, **kw) -> Case:
    """Mach-5 argon past the square [0,1] x [-0.5,0.5] in [-5,10] x [-7.5,7.5].

    scale=1 gives 160 x 160 cells with 32 x 32 solid cells whose edges are on
    node indices that are multiples of 16 (5 levels).  Farfield on the left,
    top and bottom, zero-gradient outflow on the right, diffuse square at the
    freestream temperature.  The strip behind the square starts at 0.1 of the
    freestream density and at rest.  The 100 x 100 Newton-Cotes velocity grid
    on [-15, 15]^2 is the composite trapezoid rule, as for the plate.  The
    pseudo step grows as 3^n (the paper's choice) up to 300 physical steps.
    """
    nw, nsq, ne, nyo = 48 // scale, 32 // scale, 80 // scale, 64 // scale
    first = 0.01 * scale
    xw = -5.0 + 5.0 * tanh_one_sided(nw, first / 5.0)
    xs = np.arange(1, nsq + 1) / nsq
    xe = 1.0 + 9.0 * (1.0 - tanh_one_sided(ne, first / 9.0)[::-1])
    x = np.concatenate([xw, xs, xe[1:]])
    yl = -7.5 + 7.0 * tanh_one_sided(nyo, first / 7.0)
    ys = -0.5 + np.arange(1, nsq + 1) / nsq
    yu = 0.5 + 7.0 * (1.0 - tanh_one_sided(nyo, first / 7.0)[::-1])
    y = np.concatenate([yl, ys, yu[1:]])
    nx, ny = len(x) - 1, len(y) - 1
    ftx, fty, wx, wy = _blank(nx, ny)
    ftx[:, 0] = FACE_FARFIELD
    ftx[:, nx] = FACE_OUTFLOW
    fty[0, :] = fty[ny, :] = FACE_FARFIELD
    solid = np.zeros((ny, nx), np.uint8)
    solid[nyo:nyo + nsq, nw:nw + nsq] = 1
    # faces between fluid and solid cells are diffuse walls at T = 1
    ftx[nyo:nyo + nsq, nw] = FACE_WALL
    ftx[nyo:nyo + nsq, nw + nsq] = FACE_WALL
    fty[nyo, nw:nw + nsq] = FACE_WALL
    fty[nyo + nsq, nw:nw + nsq] = FACE_WALL
    wx[ftx == FACE_WALL, 0] = 1.0
    wy[fty == FACE_WALL, 0] = 1.0
    gamma = (ARGON["K_int"] + 4.0) / (ARGON["K_int"] + 2.0)
    uinf = lid_speed(5.0, gamma)
    init = np.zeros((4, ny, nx))
    init[0], init[1], init[3] = 1.0, uinf, 1.0
    xc = 0.5 * (x[1:] + x[:-1])
    yc = 0.5 * (y[1:] + y[:-1])
    wake = (xc[None, :] >= 1.0) & (np.abs(yc[:, None]) <= 0.5)
    init[0][wake] = 0.1
    init[1][wake] = 0.0
    args = dict(name=f"square{nx}x{ny}", x=x, y=y, face_type_x=ftx, face_type_y=fty,
                wall_x=wx, wall_y=wy, solid=solid, n_levels=5, quad=QUAD_TRAPEZOID,
                nu=100, nv=100, vlo=-15.0, vhi=15.0, Kn=0.1,
                farfield=(1.0, uinf, 0.0, 1.0), init=init, precision="fp32f",
                dtn_growth=3.0, dtn_max=300.0, fas_levels=2, nu_coarse_cs=2, **ARGON)
    args.update(kw)
    return Case(**args)


def config4(**kw) -> Case:
    return square_cylinder(**kw)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


# ----------------------------------------------------------------------------
# seeded random inputs for parity tests
# ----------------------------------------------------------------------------

def random_macro(case: Case, seed: int, amp: float = 0.1) -> np.ndarray:
    """Smooth positive (rho, U, V, T) fields: the case's initial state plus seeded waves."""
    rng = np.random.default_rng(seed)
    ny, nx = case.ny, case.nx
    xc = 0.5 * (case.x[1:] + case.x[:-1])
    yc = 0.5 * (case.y[1:] + case.y[:-1])
    sx = (xc - case.x[0]) / (case.x[-1] - case.x[0])
    sy = (yc - case.y[0]) / (case.y[-1] - case.y[0])
    out = case.init.copy()
    for c in range(4):
        a, b, p, q = rng.uniform(0.5, 3.0, 4)
        wave = np.sin(2 * np.pi * a * sx + p)[None, :] * np.cos(2 * np.pi * b * sy + q)[:, None]
        noise = rng.uniform(-1.0, 1.0, (ny, nx))
        pert = amp * (0.8 * wave + 0.2 * noise)
        if c in (0, 3):
            out[c] = out[c] * (1.0 + pert)
        else:
            out[c] = out[c] + 0.5 * pert
    return out


def random_perturbation(case: Case, seed: int, amp: float = 0.05) -> np.ndarray:
    """Seeded multiplicative factors (2, Nk, ny, nx) in [1-amp, 1+amp]."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.uniform(-1.0, 1.0, (2, case.n_vel, case.ny, case.nx))


def random_field(shape, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, shape)
