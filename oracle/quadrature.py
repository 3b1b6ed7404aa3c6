"""Discrete velocity grids (oracle; test infrastructure only).

The paper integrates the discrete distribution with the trapezoidal rule for
the cavity (Sec. IV A) and with Newton-Cotes rules for the square cylinder
(Sec. IV C).  The synthetic workloads also use a Gauss-Hermite grid.  The
2-D grid is the tensor product of two 1-D rules, velocity index
k = ku * nv + kv.
"""
from __future__ import annotations

import numpy as np


def trapezoid(n: int, lo: float, hi: float):
    """Composite trapezoidal rule on n equally spaced nodes of [lo, hi]."""
    u = np.linspace(lo, hi, n)
    h = (hi - lo) / (n - 1)
    w = np.full(n, h)
    w[0] = w[-1] = 0.5 * h
    return u, w


def simpson38(n: int, lo: float, hi: float):
    """Composite Simpson 3/8 rule (closed Newton-Cotes, 4 points per panel).

    Needs (n - 1) divisible by 3; weights 3h/8 * (1, 3, 3, 2, 3, 3, 2, ..., 3, 3, 1).
    """
    if (n - 1) % 3 != 0:
        raise ValueError("Simpson 3/8 needs n - 1 divisible by 3")
    u = np.linspace(lo, hi, n)
    h = (hi - lo) / (n - 1)
    w = np.zeros(n)
    for p in range((n - 1) // 3):
        w[3 * p: 3 * p + 4] += np.array([1.0, 3.0, 3.0, 1.0]) * (3.0 * h / 8.0)
    return u, w


def gauss_hermite(n: int):
    """Gauss-Hermite nodes for the weight exp(-u^2).

    Nodes: eigenvalues of the symmetric Jacobi matrix of the physicists'
    Hermite recurrence (zero diagonal, off-diagonal sqrt(j/2); Golub-Welsch),
    polished by Newton steps on the orthonormal polynomial p_n.  Weights: the
    Christoffel numbers 1 / sum_{j<n} p_j(u_k)^2 of the orthonormal
    polynomials p_0 = pi^(-1/4), p_{j+1} = sqrt(2/(j+1)) u p_j - sqrt(j/(j+1)) p_{j-1},
    which keep full relative accuracy for the tiny outer weights.  Returned
    weights integrate plain functions: w_k = w_k^GH * exp(u_k^2).
    """
    off = np.sqrt(np.arange(1, n) / 2.0)
    jac = np.diag(off, 1) + np.diag(off, -1)
    u = np.linalg.eigvalsh(jac)

    def orthonormal(x):
        p = [np.full_like(x, np.pi ** -0.25)]
        p.append(np.sqrt(2.0) * x * p[0])
        for j in range(1, n):
            p.append(np.sqrt(2.0 / (j + 1)) * x * p[j] - np.sqrt(j / (j + 1.0)) * p[j - 1])
        return p

    for _ in range(3):
        p = orthonormal(u)
        u = u - p[n] / (np.sqrt(2.0 * n) * p[n - 1])
    u = 0.5 * (u - u[::-1])                  # exact symmetry of the rule
    p = orthonormal(u)
    wgh = 1.0 / np.sum(np.array(p[:n]) ** 2, axis=0)
    wgh = 0.5 * (wgh + wgh[::-1])
    return u, wgh * np.exp(u * u)


def rule_1d(kind: str, n: int, lo: float, hi: float):
    if kind == "trapezoid":
        return trapezoid(n, lo, hi)
    if kind == "simpson38":
        return simpson38(n, lo, hi)
    if kind == "gauss_hermite":
        return gauss_hermite(n)
    raise ValueError(kind)


class VelocityGrid:
    """Tensor-product grid: u[k], v[k], w[k] with k = ku * nv + kv."""

    def __init__(self, kind: str, nu: int, nv: int, lo: float, hi: float):
        uu, wu = rule_1d(kind, nu, lo, hi)
        vv, wv = rule_1d(kind, nv, lo, hi)
        self.nu, self.nv = nu, nv
        self.u = np.repeat(uu, nv)
        self.v = np.tile(vv, nu)
        self.w = np.repeat(wu, nv) * np.tile(wv, nu)
        self.u1, self.v1, self.wu, self.wv = uu, vv, wu, wv
        self.umax = float(np.max(np.abs(uu)))
        self.vmax = float(np.max(np.abs(vv)))

    @property
    def n(self) -> int:
        return self.nu * self.nv

    def mirror(self, d):
        """Index of the velocity with component d reversed (d = 0: u, 1: v),
        for every k; the grid must be symmetric in that component."""
        a = np.arange(self.n) // self.nv
        b = np.arange(self.n) % self.nv
        if d == 0:
            if not np.allclose(self.u1[::-1], -self.u1, rtol=0, atol=1e-12):
                raise ValueError("velocity grid not symmetric in u")
            return (self.nu - 1 - a) * self.nv + b
        if not np.allclose(self.v1[::-1], -self.v1, rtol=0, atol=1e-12):
            raise ValueError("velocity grid not symmetric in v")
        return a * self.nv + (self.nv - 1 - b)

    @classmethod
    def from_case(cls, case):
        return cls(case.quad, case.nu, case.nv, case.vlo, case.vhi)
