"""Pins of the oracle's quadrature, equilibria and compatibility correction.

Each check compares against something fixed outside the oracle's own
formulas: polynomial exactness of the rules, closed-form Gaussian moments,
the three-dimensional Shakhov target integrated numerically over the passive
velocity, and the paper's worked compatibility example (Sec. 4.1.1).
"""
import math
import os

import numpy as np
import pytest

from oracle import kinetic as kin
from oracle import levels as lv
from oracle.quadrature import gauss_hermite_1d, newton_cotes_1d, tensor_grid

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n,deg", [(101, 5), (89, 5), (33, 5), (31, 3), (7, 3), (28, 1)])
def test_newton_cotes_polynomial_exactness(n, deg):
    x, w = newton_cotes_1d(n, 3.0)
    for k in range(deg + 1):
        exact = 0.0 if k % 2 else 2.0 * 3.0 ** (k + 1) / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) <= 1e-12 * max(1.0, abs(exact))


def test_newton_cotes_symmetric_zero_node():
    x, _ = newton_cotes_1d(101, 10.0)
    assert x[50] == 0.0 and np.all(x == -x[::-1])


def test_gauss_hermite_integrates_gaussian_moments_exactly():
    R, T0 = 0.5, 1.0
    x, w = gauss_hermite_1d(28, R, T0)
    g = np.exp(-x * x / (2 * R * T0)) / math.sqrt(2 * math.pi * R * T0)
    for k, exact in [(0, 1.0), (2, R * T0), (4, 3 * (R * T0) ** 2), (6, 15 * (R * T0) ** 3)]:
        assert abs(np.sum(w * g * x ** k) - exact) < 1e-13


def _wide_grid():
    x, w = newton_cotes_1d(161, 8.0)
    return tensor_grid(x, w)


def test_shakhov_moments_closed_form():
    xi, w = _wide_grid()
    R, Pr, K = 0.5, 2.0 / 3.0, 0
    rho, u, T, q = 1.3, np.array([0.4, -0.25]), 1.1, np.array([0.03, -0.02])
    g, h = kin.shakhov(xi, rho, u, T, q, R, Pr, K)
    r, m, E = kin.conserved(xi, w, g, h)
    assert abs(r - rho) < 1e-12
    assert np.allclose(m, rho * u, atol=1e-12)
    assert abs(E - (0.5 * rho * u @ u + 1.5 * rho * R * T)) < 1e-12
    qs = kin.heat_flux(xi, w, g, h, u)
    assert np.allclose(qs, (1 - Pr) * q, atol=1e-12)


def test_reduced_forms_match_3d_shakhov_integrated_over_eta():
    """Integrate f_S(xi, eta) of Eq. shakhov_eq over eta numerically (D=2, K=0)."""
    R, Pr = 0.5, 2.0 / 3.0
    rho, u, T, q = 0.9, np.array([0.3, 0.1]), 1.2, np.array([-0.04, 0.05])
    xi = np.array([[0.1, -0.3], [1.2, 0.7], [-0.8, 1.5], [2.0, -1.0]])
    eta, weta = newton_cotes_1d(401, 10.0)
    p = rho * R * T
    c = xi - u
    c2 = np.sum(c * c, 1)
    cq = c @ q
    f = (rho / (2 * math.pi * R * T) ** 1.5 * np.exp(-(c2[:, None] + eta[None, :] ** 2) / (2 * R * T))
         * (1 + (1 - Pr) * cq[:, None] / (5 * p * R * T) * ((c2[:, None] + eta[None, :] ** 2) / (R * T) - 5)))
    g_num = f @ weta
    h_num = (f * eta[None, :] ** 2) @ weta
    g, h = kin.shakhov(xi, rho, u, T, q, R, Pr, 0)
    assert np.allclose(g, g_num, rtol=1e-12, atol=1e-15)
    assert np.allclose(h, h_num, rtol=1e-12, atol=1e-15)


def test_pr_one_is_bgk():
    xi, w = tensor_grid(*newton_cotes_1d(17, 4.0))
    g, h = kin.shakhov(xi, 1.0, np.array([0.1, 0.2]), 1.0, np.array([0.3, -0.1]), 0.5, 1.0, 0)
    ge, he = kin.maxwell(xi, 1.0, np.array([0.1, 0.2]), 1.0, 0.5, 0)
    assert np.array_equal(g, ge) and np.array_equal(h, he)


def test_one_d_equilibrium_energy():
    x, w = newton_cotes_1d(201, 12.0)
    g, h = kin.maxwell(x[:, None], 0.7, np.array([0.2]), 0.9, 1.0, 0)
    r, m, E = kin.conserved(x[:, None], w, g, h)
    assert abs(E - (0.5 * 0.7 * 0.04 + 1.5 * 0.7 * 0.9)) < 1e-12


def _quadtree_level(nv=32, a=4.0):
    """A nonuniform quadtree grid: 8x8 merges in one corner, 4x4 and 2x2 elsewhere."""
    x, w = newton_cotes_1d(nv, a)
    xi, ww = tensor_grid(x, w)
    base = lv.BaseGrid(xi, ww, nv, nv)
    k = np.zeros(base.Nb, np.uint8)
    kk = k.reshape(base.nby, base.nbx)
    kk[0:4, 0:4] = 3
    kk[0:4, 8:12] = 3
    kk[4:6, 0:2] = 2
    kk[12:16, 12:16] = 2
    kk[6:8, 2:6] = 1
    kk[14, 0] = 1
    return lv.Level(base, k)


def test_compat_correction_restores_moments_on_nonuniform_grid():
    with open(os.path.join(GOLD, "h1_compat.txt")) as f:
        rows = [l.split() for l in f if not l.startswith("#")]
    rho, u, v, T, R = map(float, rows[0])
    paper_eps = float(rows[1][0])
    L = _quadtree_level()
    xi, w = L.xi, L.w
    uu = np.array([u, v])
    g0, h0 = kin.maxwell(xi, rho, uu, T, R, 0)
    tgt = np.array([rho, rho * u, rho * v, 0.5 * rho * (u * u + v * v) + 1.5 * rho * R * T])

    def eps(g, h):
        return np.max(np.abs(lv.moments4(xi, w, g, h) - tgt) / np.abs(tgt))

    assert eps(g0, h0) > 1e-6                     # discrete defect exists before correction
    g1, h1, _ = kin.compat_correct4(xi, w, g0, h0, rho, uu, T, R, 0)
    assert eps(g1, h1) < 50 * max(paper_eps, np.finfo(float).eps)


def test_compat8_satisfies_all_eight_constraints():
    L = _quadtree_level(nv=48, a=5.0)
    xi, w = L.xi, L.w
    R, Pr = 0.5, 2.0 / 3.0
    rho, u, T, q = 1.1, np.array([0.5, -0.2]), 0.9, np.array([0.02, 0.03])
    gS, hS = kin.shakhov(xi, rho, u, T, q, R, Pr, 0)
    g, h, _ = kin.compat_correct8(xi, w, gS, hS, rho, u, T, (1 - Pr) * q, R, 0)
    c = xi - u
    c2 = np.sum(c * c, 1)
    m = [np.sum(w * g), np.sum(w * xi[:, 0] * g), np.sum(w * xi[:, 1] * g),
         0.5 * np.sum(w * (h + np.sum(xi * xi, 1) * g)),
         0.5 * np.sum(w * (h + c2 * g) * c[:, 0]), 0.5 * np.sum(w * (h + c2 * g) * c[:, 1]),
         np.sum(w * (c[:, 0] ** 2 - c[:, 1] ** 2) * g), np.sum(w * c[:, 0] * c[:, 1] * g)]
    tgt = [rho, rho * u[0], rho * u[1], 0.5 * rho * u @ u + 1.5 * rho * R * T,
           (1 - Pr) * q[0], (1 - Pr) * q[1], 0.0, 0.0]
    assert np.allclose(m, tgt, rtol=0, atol=1e-13)


def test_compat_one_d_three_by_three():
    x, w = newton_cotes_1d(21, 4.0)
    g, h = kin.maxwell(x[:, None], 1.0, np.array([0.6]), 1.0, 1.0, 0)
    gc, hc, a = kin.compat_correct4(x[:, None], w, g, h, 1.0, np.array([0.6]), 1.0, 1.0, 0)
    assert a.shape == (3,)
    r, m, E = kin.conserved(x[:, None], w, gc, hc)
    assert abs(r - 1) < 1e-14 and abs(m[0] - 0.6) < 1e-14 and abs(E - (0.18 + 1.5)) < 1e-14


def test_vhs_reference_viscosity_constant():
    # 15 sqrt(pi) / (2 (5 - 2w)(7 - 2w)) at w = 0.81
    assert abs(kin.mu_ref_from_kn(1.0, 1.0, 1.0, 0.5, 1.0, 0.81) - 0.73097) < 1e-4
