"""Gas model and velocity moments (oracle; test infrastructure only).

Nondimensional units with R T0 = 1/2, so lambda = 1/(2 R T) = 1/T and the
pressure is p = rho / (2 lambda).  The distribution is carried as the reduced
pair (G, H): G integrates f over the K_int extra velocity components and H
integrates their squared magnitude (the paper calls f "reduced" in Sec. III B,
equation of the wall distribution).  K = K_int + 2 is the total number of
degrees of freedom entering the energy, gamma = (K + 2) / K.

Conservative variables W = (rho, rho U, rho V, rho eps) (Sec. II A) with
rho eps = rho |U|^2 / 2 + K rho / (4 lambda).
"""
from __future__ import annotations

import math

import numpy as np


class Gas:
    def __init__(self, K_int: int, Pr: float, omega: float, Kn: float):
        self.K_int = int(K_int)
        self.K = self.K_int + 2
        self.gamma = (self.K + 2.0) / self.K
        self.Pr = float(Pr)
        self.omega = float(omega)
        self.Kn = float(Kn)
        self.mu_ref = mu_ref_vhs(Kn, omega)

    @classmethod
    def from_case(cls, case):
        return cls(case.K_int, case.Pr, case.omega, case.Kn)

    # viscosity law mu = mu_ref (T / T0)^omega (Sec. IV A) and tau = mu / p
    def mu(self, T):
        return self.mu_ref * np.power(T, self.omega)

    def tau(self, rho, lam):
        T = 1.0 / lam
        p = rho / (2.0 * lam)
        return self.mu(T) / p


def mu_ref_vhs(Kn: float, omega: float, alpha: float = 1.0) -> float:
    """Reference viscosity from the VHS mean free path, lambda_mfp = Kn.

    mu = 5 (alpha+1)(alpha+2) sqrt(pi) Kn / (4 alpha (5 - 2 omega)(7 - 2 omega))
    at rho = 1 and 2 R T = 1 (Bird's VHS relation between viscosity and mean
    free path; the paper defines Kn by the mean free path, Sec. IV).
    """
    return (5.0 * (alpha + 1.0) * (alpha + 2.0) * math.sqrt(math.pi) * Kn
            / (4.0 * alpha * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega)))


def primitive(W, K):
    """(rho, U, V, lambda) from W = (rho, rho U, rho V, rho eps)."""
    rho = W[0]
    U = W[1] / rho
    V = W[2] / rho
    e_int = W[3] - 0.5 * rho * (U * U + V * V)
    lam = K * rho / (4.0 * e_int)
    return rho, U, V, lam


def conservative(rho, U, V, lam, K):
    return np.array([rho, rho * U, rho * V,
                     0.5 * rho * (U * U + V * V) + K * rho / (4.0 * lam)])


def maxwellian(rho, U, V, lam, u, v, K_int):
    """Reduced Maxwellian: G = rho (lam/pi) exp(-lam |c|^2), H = K_int/(2 lam) G.

    Cell quantities broadcast against velocity arrays; the result has the
    velocity axis first when u, v are shaped (Nk, 1).
    """
    cx = u - U
    cy = v - V
    G = rho * (lam / np.pi) * np.exp(-lam * (cx * cx + cy * cy))
    H = (K_int / (2.0 * lam)) * G
    return G, H


def shakhov(rho, U, V, lam, qx, qy, u, v, K_int, Pr):
    """Shakhov equilibrium for the reduced pair (Sec. II A, Shakhov-type model
    with the Prandtl-number correction).

    The gas has N = 2 + K_int degrees of freedom, the K_int beyond the plane
    velocity entering like extra velocity components xi.  The Shakhov factor
    over all of them is 1 + (1 - Pr) (c.q) / ((N + 2) p R T) (s / (R T) - (N + 2))
    with s = |c|^2 + |xi|^2; integrating it over xi (and xi^2 for H) gives

    g+ = 4/(K_int + 4) (1 - Pr) lam^2 (c.q) / rho * (2 lam |c|^2 - 4) G_eq   (G part)
    g+ = 4/(K_int + 4) (1 - Pr) lam^2 (c.q) / rho * (2 lam |c|^2 - 2) H_eq   (H part)

    The correction carries no mass, momentum or energy and the heat flux of
    the pair is (1 - Pr) q, for any K_int (for K_int = 1 it is the 3-D
    factor (c^2/(RT) - 5) / (5 p R T) of a monatomic gas).
    """
    G, H = maxwellian(rho, U, V, lam, u, v, K_int)
    cx = u - U
    cy = v - V
    c2 = cx * cx + cy * cy
    fac = 4.0 / (K_int + 4.0) * (1.0 - Pr) * lam * lam * (cx * qx + cy * qy) / rho
    Gp = fac * (2.0 * lam * c2 - 4.0) * G
    Hp = fac * (2.0 * lam * c2 - 2.0) * H
    return G + Gp, H + Hp


def moments(G, H, vel):
    """W = sum_k w_k psi_k f_k with psi = (1, u, v, (u^2+v^2)/2 [+ H/2]).

    G, H have the velocity axis first.
    """
    w = vel.w.reshape((-1,) + (1,) * (G.ndim - 1))
    u = vel.u.reshape(w.shape)
    v = vel.v.reshape(w.shape)
    rho = np.sum(w * G, axis=0)
    mx = np.sum(w * u * G, axis=0)
    my = np.sum(w * v * G, axis=0)
    en = 0.5 * np.sum(w * ((u * u + v * v) * G + H), axis=0)
    return np.array([rho, mx, my, en])


def heat_flux(G, H, vel, U, V):
    """q = 1/2 sum_k w_k c_k (|c_k|^2 G_k + H_k), c = u - U (peculiar velocity)."""
    w = vel.w.reshape((-1,) + (1,) * (G.ndim - 1))
    cx = vel.u.reshape(w.shape) - U
    cy = vel.v.reshape(w.shape) - V
    e = (cx * cx + cy * cy) * G + H
    return np.array([0.5 * np.sum(w * cx * e, axis=0), 0.5 * np.sum(w * cy * e, axis=0)])
