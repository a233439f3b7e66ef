"""Discrete velocity sets (Sec. 2.3 "Discrete velocity formulation").

The paper uses Newton-Cotes quadrature on a uniform Cartesian velocity grid
without naming the rule.  Reading used here: composite closed Boole rule when
(n - 1) is a multiple of 4, composite closed Simpson rule when (n - 1) is
even, and the composite midpoint rule (cell-centred nodes) when n is even.
Gauss-Hermite is offered for the cavity workload: nodes sqrt(2 R T0) x_k and
weights that integrate f itself, sqrt(2 R T0) omega_k exp(x_k^2).
"""
from __future__ import annotations

import numpy as np


def newton_cotes_1d(n: int, a: float):
    """Nodes and weights on [-a, a]; see the module docstring for the rule."""
    if n < 2:
        raise ValueError("need at least two nodes")
    if n % 2 == 0:
        h = 2.0 * a / n
        x = -a + h * (np.arange(n) + 0.5)
        return x, np.full(n, h)
    x = a * (2.0 * np.arange(n) - (n - 1)) / (n - 1)
    h = 2.0 * a / (n - 1)
    w = np.zeros(n)
    if (n - 1) % 4 == 0:
        # Boole: h*2/45 * [7, 32, 12, 32, 7] per panel of four intervals
        pattern = np.array([7.0, 32.0, 12.0, 32.0, 7.0]) * (2.0 * h / 45.0)
        for p in range(0, n - 1, 4):
            w[p:p + 5] += pattern
    else:
        pattern = np.array([1.0, 4.0, 1.0]) * (h / 3.0)
        for p in range(0, n - 1, 2):
            w[p:p + 3] += pattern
    return x, w


def gauss_hermite_1d(n: int, R: float, T0: float):
    """Gauss-Hermite nodes scaled by sqrt(2 R T0), weights integrating f itself."""
    xk, wk = np.polynomial.hermite.hermgauss(n)
    c = np.sqrt(2.0 * R * T0)
    return c * xk, c * wk * np.exp(xk * xk)


def tensor_grid(x1, w1, y1=None, wy=None):
    """2-D tensor grid, point index b = ix + nx*iy (x fastest)."""
    if y1 is None:
        y1, wy = x1, w1
    XX, YY = np.meshgrid(x1, y1)
    WW = np.outer(wy, w1)
    xi = np.stack([XX.ravel(), YY.ravel()], axis=1)
    return xi, WW.ravel().copy()


def base_grid(problem):
    """Base velocity set V_base for a workload: (xi (N, D), w (N,), nx, ny)."""
    if problem.vel_kind == "gh":
        x1, w1 = gauss_hermite_1d(problem.nv, problem.R, problem.gh_scale_T)
    else:
        x1, w1 = newton_cotes_1d(problem.nv, problem.vmax)
    if problem.dim == 1:
        return x1[:, None].copy(), w1.copy(), problem.nv, 1
    xi, w = tensor_grid(x1, w1)
    return xi, w, problem.nv, problem.nv
