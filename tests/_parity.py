"""Shared helpers of the GPU parity tests: small cases covering every boundary
tag, ragged sizes, and the comparison metrics."""
import numpy as np

import workloads as wl
from oracle import flux as fx


def small_cases():
    """Cases the oracle finishes in seconds, spanning several 64-cell tiles and
    32-velocity chunks, with ragged tails (down to a one-velocity chunk), and
    every boundary tag."""
    c = {}
    c["cavity16_kn10"] = wl.config1()
    c["box12x10_ragged"] = wl.cavity(n=12, ny=10, Kn=0.3, n_levels=2, quad="gauss_hermite", nvel=9, nvel_y=10,
                                     vlo=0.0, vhi=0.0, mach=0.3, name="box12x10_ragged")
    c["plate32x24"] = wl.flat_plate(scale=4, quad="trapezoid", nu=14, nv=12, vlo=-5.0, vhi=5.0, n_levels=2,
                                    precision="fp64", Kn=0.2)
    c["square20x20"] = wl.square_cylinder(scale=8, quad="trapezoid", nu=16, nv=16, vlo=-12.0, vhi=12.0,
                                          n_levels=2, precision="fp64", nu_coarse=4)
    # 65 velocities: the last 32-velocity chunk holds one, and three of the
    # four waves of its blocks hold none
    c["box8_vel65"] = wl.cavity(n=8, Kn=0.3, n_levels=2, quad="gauss_hermite", nvel=13, nvel_y=5, vlo=0.0,
                                vhi=0.0, mach=0.3, name="box8_vel65")
    return c


def tiny_open_plate():
    """7 x 6 cells around a one-face plate (both of its sides are walls at the
    face's one temperature), farfield sides and an outflow side, 6 x 6
    Gauss-Hermite velocities, Kn 0.3, one level; FP64 runs of it reach 2e-13
    in about sixty cycles.  An open domain: no mass constraint."""
    case = wl.flat_plate(scale=16, quad="gauss_hermite", nu=6, nv=6, vlo=0.0, vhi=0.0, n_levels=1,
                         precision="fp64", Kn=0.3)
    case.face_type_x[:, -1] = wl.FACE_OUTFLOW
    j, i = np.argwhere(case.face_type_y == wl.FACE_WALL)[0]
    plate_face = (case.nx + 1) * case.ny + j * case.nx + i
    return case, int(plate_face)


def rel_max(a, ref):
    """max |a - ref| / max |ref| (a max-norm scale: fields cross zero)."""
    return float(np.max(np.abs(np.asarray(a) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def field_errors(macro, prim_ref, fluid=None):
    """Per-field max-norm relative error of rho, U, V, T over fluid cells
    (solid cells carry no gas); NaN anywhere counts as an infinite error."""
    out = {}
    for name, ref in zip(("rho", "U", "V", "T"), prim_ref):
        ref = np.asarray(ref).reshape(macro[name].shape)
        got = macro[name]
        if fluid is not None:
            m = np.asarray(fluid).reshape(ref.shape)
            ref, got = ref[m], got[m]
        if not (np.all(np.isfinite(ref)) and np.all(np.isfinite(got))):
            out[name] = float("inf")
            continue
        scale = max(np.max(np.abs(ref)), 1e-300)
        out[name] = float(np.max(np.abs(got - ref)) / scale)
    return out


def perturbed_state(case, seed):
    """Seeded macro fields and multiplicative perturbation of f (inputs only)."""
    prim = wl.random_macro(case, seed=seed, amp=0.08)
    pert = wl.random_perturbation(case, seed=seed + 1, amp=0.05)
    return prim, pert


def to_oracle(f):
    """(2, Nk, ny, nx) -> (G, H) each (Nk, Nc)."""
    nk = f.shape[1]
    return f[0].reshape(nk, -1).astype(float), f[1].reshape(nk, -1).astype(float)


def from_oracle(G, H, case):
    return np.stack([G.reshape(-1, case.ny, case.nx), H.reshape(-1, case.ny, case.nx)])


def free_molecular_closed_form(case, vel, K_int, M0, area):
    """Heat transfer through a free-molecular gap: every point holds the bottom
    plate's half-range Maxwellian rho_b C_b for upward velocities and the top
    plate's rho_t C_t for downward ones; zero net mass flux and the total mass
    fix rho_b and rho_t (discrete sums over the velocity grid)."""
    Cb, Hb = fx.wall_maxwellian(case.wall_y[0, 0, 0], 0.0, 0.0, vel.u, vel.v, K_int)
    Ct, Ht = fx.wall_maxwellian(case.wall_y[case.ny, 0, 0], 0.0, 0.0, vel.u, vel.v, K_int)
    up, dn = vel.v > 0, vel.v < 0
    # rho_b Fb = rho_t Ft (flux balance), area (rho_b Mb + rho_t Mt) = M0 (mass)
    Fb = np.sum((vel.w * vel.v * Cb)[up])
    Ft = -np.sum((vel.w * vel.v * Ct)[dn])
    Mb = np.sum((vel.w * Cb)[up])
    Mt = np.sum((vel.w * Ct)[dn])
    rb, rt = np.linalg.solve([[Fb, -Ft], [area * Mb, area * Mt]], [0.0, M0])
    G = np.where(up, rb * Cb, rt * Ct)
    H = np.where(up, rb * Hb, rt * Ht)
    return G, H
