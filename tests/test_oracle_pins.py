"""Pins of oracle parts that the other oracle tests leave open.

* The criterion's arithmetic (Sec. 3.2, Eqs. M2, block-contribution-indicator,
  merge-transport-error, combined-merge-condition, block-hysteresis-rule) on a
  4 x 4 grid whose indicators, normalisations S_r and transport errors eps_B
  were worked out by hand (the fractions below); the merge decisions follow
  from them.
* The far-field boundary (reading R8): one cell with far-field faces on all
  four sides, free-molecular (tau -> infinity, so phi_bar+ = phi~ and
  phi_f = phi_bar_f), zero slopes.  The mass and x-momentum it gains in one
  step are the closed-form half-range fluxes of two Maxwellians: the cell's
  own leaving through every face and the free stream's entering.
* The selector's features (reading R25) for rotated bi-Maxwellian states on a
  linear density field: the stress comes from the distribution (closed form
  rho R (T_a - T_b) sin(t) cos(t) and friends), the gradient from the mesh.
* The weighting chi = (g_S, h_S) of the compatibility correction (Eq.
  gh_model_correction): g*/g_S - 1 lies in the span of the correction basis
  and h*/h_S - 1 equals it point by point.  chi = 1 would fail both.
* The positivity band of the exponential fallback (reading R22) on both of
  its sides.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import workloads as W
from oracle import kinetic as kin
from oracle import levels as lv
from oracle import mlp
from oracle.quadrature import newton_cotes_1d, tensor_grid
from oracle.solver import Solver


# ---------------------------------------------------------------------------
# criterion, worked by hand
# ---------------------------------------------------------------------------
# Axis nodes {-3, -1, 1, 3} with unit weights; point b = ix + 4 iy.
# g = 1 everywhere except g = 5 at (xi_x, xi_y) = (3, 3); h = 2 everywhere.
#   rho_tot = 15 + 5 = 20.  |xi|^2 is 2 on the 4 inner points, 10 on the 8
#   edge points, 18 on the corners: sum |xi|^2 g = 8 + 80 + 3*18 + 5*18 = 232,
#   sum h = 32, so E_tot = (232 + 32)/2 = 132.
#   2x2 block (0,0) (xi in {-3,-1}^2): sum M1 = 4/20, sum M2 = (40 + 8)/2/132
#   = 2/11, I = 1/5; blocks (1,0), (0,1) the same; block (1,1): sum M1 = 8/20,
#   sum M2 = (2 + 10 + 10 + 90 + 8)/2/132 = 5/11, I = 5/11; the 4x4 block: 1.
#   S_0 = sum |xi_x| g = 32 + 12 = 44; S_1 = S_2 = sum xi_x^2 g = 80 + 36 = 116
#   (the cross sum |xi_x xi_y| g is 64 + 36 = 100 < 116); S_3 = sum |xi_x|
#   (h + |xi|^2 g)/2 = (64 + 384 + 216)/2 = 332.
#   eps_B of block (1,1): merged point xi_B = (2, 2), g_B = 2, H_B = 30; along
#   +x the fine flux of xi_x g is 1 + 9 + 1 + 45 = 56 against 4*2*4 = 32:
#   24/116 = 6/29, the largest of its 16 ratios.  Blocks (0,0), (1,0), (0,1):
#   g is constant, the mass flux matches, the xi_d^2 g flux differs by
#   20 - 16 = 4: 4/116 = 1/29.  The 4x4 block has xi_B = 0, so every merged
#   flux vanishes and the largest fine one is the energy flux along +x:
#   (72 + 40 + 40 + 288)/2 = 220 -> 220/332 = 55/83.
def _hand_case():
    x1 = np.array([-3.0, -1.0, 1.0, 3.0])
    xi, w = tensor_grid(x1, np.ones(4))
    base = lv.BaseGrid(xi, w, 4, 4)
    g = np.ones(16)
    g[3 + 4 * 3] = 5.0
    h = np.full(16, 2.0)
    return base, g, h


def test_criterion_indicators_by_hand():
    base, g, h = _hand_case()
    M1, M2 = lv.indicators(base, g, h)
    assert np.sum(M1) == pytest.approx(1.0, abs=1e-15) and np.sum(M2) == pytest.approx(1.0, abs=1e-15)
    want = {(0, 0): 1 / 5, (1, 0): 1 / 5, (0, 1): 1 / 5, (1, 1): 5 / 11}
    for (bx, by), v in want.items():
        assert lv.block_indicator(base, M1, M2, 1, bx, by) == pytest.approx(v, rel=1e-14)
    assert lv.block_indicator(base, M1, M2, 2, 0, 0) == pytest.approx(1.0, rel=1e-14)


def test_criterion_flux_scale_and_transport_error_by_hand():
    base, g, h = _hand_case()
    S = lv.flux_scale(base, g, h)
    assert np.allclose(S, [44.0, 116.0, 116.0, 332.0], rtol=1e-15)
    want = {(1, 0, 0): 1 / 29, (1, 1, 0): 1 / 29, (1, 0, 1): 1 / 29, (1, 1, 1): 6 / 29, (2, 0, 0): 55 / 83}
    for (s, bx, by), v in want.items():
        assert lv.block_flux_error(base, g, h, S, s, bx, by) == pytest.approx(v, rel=1e-14)


def test_criterion_decisions_by_hand():
    base, g, h = _hand_case()
    L0 = lv.Level(base, np.zeros(4, np.uint8))
    # C_merge 0.25 < I = 0.2?  no: I = 0.2 < 0.25 merges blocks (0,0), (1,0),
    # (0,1) unless eps_B = 1/29 = 0.0345 exceeds eps_merge; block (1,1) has
    # I = 5/11 > C_split and stays fine; the 4x4 block (I = 1) never merges.
    assert list(lv.criterion(L0, g, h, 0.3, 0.25, 0.05, True)) == [1, 1, 1, 0]
    assert list(lv.criterion(L0, g, h, 0.3, 0.25, 0.03, True)) == [0, 0, 0, 0]
    assert list(lv.criterion(L0, g, h, 0.3, 0.25, 0.0, False)) == [1, 1, 1, 0]
    # hysteresis band C_merge 0.15 <= I = 0.2 <= C_split 0.25: a block merges
    # only if the cell's current level already merges it.  On a level that
    # merges block (0,0) the stored state is that level's (the projection of
    # the base state), whose block sums of g and h + |xi|^2 g are unchanged.
    L1 = lv.Level(base, np.array([1, 0, 0, 0], np.uint8))
    g1, h1 = lv.project(L0, L1, g, h)
    assert list(lv.criterion(L1, g1, h1, 0.25, 0.15, 0.0, False)) == [1, 0, 0, 0]
    assert list(lv.criterion(L0, g, h, 0.25, 0.15, 0.0, False)) == [0, 0, 0, 0]
    # 5/11 = 0.4545 decides block (1,1) at C_merge just above / below it
    assert list(lv.criterion(L0, g, h, 0.9, 0.46, 0.0, False)) == [1, 1, 1, 1]
    assert list(lv.criterion(L0, g, h, 0.9, 0.45, 0.0, False)) == [1, 1, 1, 0]


# ---------------------------------------------------------------------------
# far-field boundary against closed-form half-range fluxes
# ---------------------------------------------------------------------------
def _half_flux_mass(rho, un, RT):
    """int_{c_n > 0} c_n f dc of a Maxwellian with normal velocity un."""
    s = un / math.sqrt(2.0 * RT)
    return rho * (math.sqrt(RT / (2.0 * math.pi)) * math.exp(-s * s) + 0.5 * un * (1.0 + erf(s)))


def _half_flux_normal_momentum(rho, un, RT):
    """int_{c_n > 0} c_n^2 f dc."""
    s = un / math.sqrt(2.0 * RT)
    return rho * (0.5 * (un * un + RT) * (1.0 + erf(s)) + un * math.sqrt(RT / (2.0 * math.pi)) * math.exp(-s * s))


def _one_cell_farfield(cell, ff, nv, vmax):
    R = 0.5
    X, Y = np.meshgrid(np.array([0.0, 1.0]), np.array([0.0, 1.0]))
    one = np.ones((1, 1))
    bcs = [W.BC(W.FARFIELD, rho=ff[0], u=ff[1], v=ff[2], T=ff[3])]
    z = np.zeros(1, np.int32)
    return W.Problem("ff1", 2, X.copy(), Y.copy(), False, False, bcs, z, z.copy(), z.copy(), z.copy(),
                     cell[0] * one, cell[1] * one, cell[2] * one, cell[3] * one, R=R, Pr=1.0, K=0,
                     omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0, Kn=1e9, cfl=0.5, vel_kind="nc",
                     nv=nv, vmax=vmax)


@pytest.mark.parametrize("nv", [160, 320])
def test_farfield_fluxes_match_half_range_closed_form(nv):
    cell = (1.0, 0.15, -0.25, 1.0)
    ff = (0.4, 0.6, 0.3, 1.6)
    p = _one_cell_farfield(cell, ff, nv, 8.0)
    s = Solver(p, compat=0)
    R, dt = p.R, s.dt
    m0 = s.totals()
    s.step()
    m1 = s.totals()
    # outward normals -x, +x, -y, +y of the unit cell: the cell's own state
    # leaves through each face, the free stream's enters
    out_mass = in_mass = out_mx = in_mx = 0.0
    for axis, sgn in ((0, -1.0), (0, 1.0), (1, -1.0), (1, 1.0)):
        unc = sgn * cell[1 + axis]
        unf = sgn * ff[1 + axis]
        out_mass += _half_flux_mass(cell[0], unc, R * cell[3])
        in_mass += _half_flux_mass(ff[0], -unf, R * ff[3])        # int_{c_n < 0} |c_n| f
        if axis == 0:
            # x-momentum through the x-faces: c_n xi_x = sgn c_n^2
            out_mx += sgn * _half_flux_normal_momentum(cell[0], unc, R * cell[3])
            in_mx -= sgn * _half_flux_normal_momentum(ff[0], -unf, R * ff[3])
        else:
            # through the y-faces: the tangential mean velocity times the mass flux
            out_mx += cell[1] * _half_flux_mass(cell[0], unc, R * cell[3])
            in_mx += ff[1] * _half_flux_mass(ff[0], -unf, R * ff[3])
    dm = m1[0] - m0[0]
    dmx = m1[1] - m0[1]
    assert dm == pytest.approx(dt * (in_mass - out_mass), rel=4e-3 * (160 / nv) ** 2)
    assert dmx == pytest.approx(dt * (in_mx - out_mx), rel=4e-3 * (160 / nv) ** 2)
    # a boundary that reflected the cell's own state would gain nothing
    assert abs(dm) > 0.1 * dt


def test_uniform_freestream_in_farfield_box_is_fixed():
    # the free stream itself, on a grid that integrates the Maxwellian to round-off
    state = (1.0, 0.3, -0.2, 1.0)
    p = _one_cell_farfield(state, state, 80, 8.0)
    p = W.Problem("ffbox", 2, *np.meshgrid(np.linspace(0, 1, 4), np.linspace(0, 0.75, 4)), False, False,
                  p.bcs, np.zeros(3, np.int32), np.zeros(3, np.int32), np.zeros(3, np.int32),
                  np.zeros(3, np.int32), np.ones((3, 3)), np.full((3, 3), 0.3), np.full((3, 3), -0.2),
                  np.ones((3, 3)), R=0.5, Pr=2.0 / 3.0, K=0, omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0,
                  Kn=0.05, cfl=0.5, vel_kind="nc", nv=80, vmax=8.0)
    s = Solver(p, compat=4)
    g0 = [x.copy() for x in s.g]
    for _ in range(3):
        s.step()
    assert max(np.max(np.abs(a - b)) for a, b in zip(s.g, g0)) < 1e-14 * max(np.max(x) for x in g0)


# ---------------------------------------------------------------------------
# selector features in closed form
# ---------------------------------------------------------------------------
def _bimaxwell(xi, rho, u, v, Ta, Tb, Tz, th, R):
    """g of a bi-Maxwellian with temperatures (Ta, Tb) along axes rotated by th,
    h = R Tz g (the passive third direction)."""
    c = xi - np.array([u, v])[None, :]
    ca = c[:, 0] * math.cos(th) + c[:, 1] * math.sin(th)
    cb = -c[:, 0] * math.sin(th) + c[:, 1] * math.cos(th)
    g = rho / (2.0 * math.pi * R * math.sqrt(Ta * Tb)) * np.exp(-ca * ca / (2 * R * Ta) - cb * cb / (2 * R * Tb))
    return g, R * Tz * g


def test_features_closed_form():
    R, a, u, v, Ta, Tb, Tz, th = 0.5, 0.6, 0.2, -0.1, 1.5, 0.9, 1.2, 0.3
    X, Y = np.meshgrid(np.linspace(0, 1, 4), np.linspace(0, 1, 4))
    z = np.zeros(3, np.int32)
    p = W.Problem("feat", 2, X, Y, False, False, [W.BC(W.OUTFLOW)], z, z.copy(), z.copy(), z.copy(),
                  np.ones((3, 3)), np.zeros((3, 3)), np.zeros((3, 3)), np.ones((3, 3)), R=R, Pr=2.0 / 3.0,
                  K=0, omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0, Kn=0.05, cfl=0.5, vel_kind="nc",
                  nv=64, vmax=8.0)
    s = Solver(p, compat=0)
    xi, w = s.vset(0)
    for c in range(9):
        rho = 1.0 + a * s.mesh.xc[c, 0]
        s.g[c], s.h[c] = _bimaxwell(xi, rho, u, v, Ta, Tb, Tz, th, R)
    f = s.fields()
    sig = np.array([mlp.cell_stress(xi, w, s.g[c], f[c, 0], f[c, 1:3], f[c, 3], R) for c in range(9)])
    grad = mlp.cell_gradient(s.mesh, f[:, 0])
    F = mlp.features(f[:, 0], f[:, 1], f[:, 2], f[:, 3], f[:, 4], f[:, 5], sig[:, 0], sig[:, 1], grad,
                     s.mesh.vol, R, p.T_ref, s.mu(f[:, 3]))[4]        # the centre cell
    rho = 1.0 + a * 0.5
    T = (Ta + Tb + Tz) / 3.0
    Pxx = rho * R * (Ta * math.cos(th) ** 2 + Tb * math.sin(th) ** 2)
    Pxy = rho * R * (Ta - Tb) * math.sin(th) * math.cos(th)
    pres = rho * R * T
    mu = s.mu_ref * T ** 0.81
    lam = mu / pres * math.sqrt(math.pi * R * T / 2.0)
    dx = 1.0 / 3.0
    want = [math.log(rho), u / math.sqrt(R), v / math.sqrt(R), math.log(T), 0.0, 0.0,
            Pxx / pres - 1.0, Pxy / pres, math.log(1.0 + dx * a / rho), math.log10(lam / dx)]
    assert np.allclose(F, want, rtol=1e-11, atol=1e-12)
    # the stress terms are not trivially zero, the gradient not the one-sided one
    assert abs(want[6]) > 0.05 and abs(want[7]) > 0.05
    assert grad[4] == pytest.approx(a, rel=1e-11)


# ---------------------------------------------------------------------------
# chi = (g_S, h_S) in the compatibility correction
# ---------------------------------------------------------------------------
def _coarse_shakhov():
    x, wx = newton_cotes_1d(9, 3.2)
    xi, w = tensor_grid(x, wx)
    R, Pr, K = 0.5, 2.0 / 3.0, 0
    rho, u, T, q = 1.2, np.array([0.35, -0.2]), 0.9, np.array([0.05, 0.02])
    gS, hS = kin.shakhov(xi, rho, u, T, q, R, Pr, K)
    return xi, w, gS, hS, rho, u, T, q, R, Pr, K


def _span_residual(basis, r, mask):
    coef, *_ = np.linalg.lstsq(basis[mask], r[mask], rcond=None)
    return float(np.max(np.abs(basis[mask] @ coef - r[mask]))) / float(np.max(np.abs(r[mask])))


def test_compat4_weighting_is_the_model_distribution():
    xi, w, gS, hS, rho, u, T, q, R, Pr, K = _coarse_shakhov()
    g4, h4, a = kin.compat_correct4(xi, w, gS, hS, rho, u, T, R, K)
    mask = (np.abs(gS) > 1e-6 * np.max(np.abs(gS))) & (np.abs(hS) > 1e-6 * np.max(np.abs(hS)))
    r = g4[mask] / gS[mask] - 1.0
    x2 = np.sum(xi * xi, axis=1)
    Exi = 0.5 * ((3 - 2 + K) * R * T + x2)
    basis = np.column_stack([np.ones_like(x2), xi[:, 0], xi[:, 1], Exi])[mask]
    assert np.max(np.abs(r)) > 1e-4                      # a real correction on this coarse grid
    assert _span_residual(basis, r, np.ones(len(r), bool)) < 1e-10
    assert np.max(np.abs(h4[mask] / hS[mask] - 1.0 - r)) < 1e-12 * np.max(np.abs(r)) + 1e-15
    # the additive form (chi = 1) would put g* - g_S, not the ratio, in the span
    d = g4[mask] - gS[mask]
    assert _span_residual(basis, d, np.ones(len(d), bool)) > 1e-3


def test_compat8_weighting_is_the_model_distribution():
    xi, w, gS, hS, rho, u, T, q, R, Pr, K = _coarse_shakhov()
    g8, h8, a = kin.compat_correct8(xi, w, gS, hS, rho, u, T, (1 - Pr) * q, R, K)
    mask = (np.abs(gS) > 1e-6 * np.max(np.abs(gS))) & (np.abs(hS) > 1e-6 * np.max(np.abs(hS)))
    r = g8[mask] / gS[mask] - 1.0
    x2 = np.sum(xi * xi, axis=1)
    c = xi - u[None, :]
    c2 = np.sum(c * c, axis=1)
    cK = (3 - 2 + K) * R * T
    basis = np.column_stack([np.ones_like(x2), xi[:, 0], xi[:, 1], 0.5 * (cK + x2), 0.5 * (cK + c2) * c[:, 0],
                             0.5 * (cK + c2) * c[:, 1], c[:, 0] ** 2 - c[:, 1] ** 2, c[:, 0] * c[:, 1]])[mask]
    assert np.max(np.abs(r)) > 1e-4
    assert _span_residual(basis, r, np.ones(len(r), bool)) < 1e-10
    assert np.max(np.abs(h8[mask] / hS[mask] - 1.0 - r)) < 1e-12 * np.max(np.abs(r)) + 1e-15


# ---------------------------------------------------------------------------
# the positivity band of the exponential fallback
# ---------------------------------------------------------------------------
def test_positivity_band_both_sides():
    p = W.periodic_box(2, 2, Lx=1.0, Ly=1.0, Kn=0.05, nv=12, vmax=4.0, kind="uniform")
    s = Solver(p, compat=4, positivity="exp")
    lev = s.levels[0]
    xi, wts = lev.xi, lev.w
    gp, hp = kin.maxwell(xi, 1.0, np.array([0.1, 0.0]), 1.0, p.R, p.K)
    top = np.max(gp)
    tgt = lv.moments4(xi, wts, gp, hp)
    band = s.POS_EPS * top
    k = int(np.argmin(gp))
    for depth, takes in ((0.5, False), (2.0, True)):
        gs = gp.copy()
        gs[k] = -depth * band                    # a linear result that dips below zero
        s.exp_count = 0
        ge, he = s.positivity_fallback(lev, gp, hp, gs, hp.copy(), tgt)
        assert (s.exp_count == 1) == takes
        assert (ge is gs) != takes
    # a provisional state a little below zero still counts as nonnegative
    # inside the band, not beyond it
    for depth, takes in ((0.5, True), (2.0, False)):
        gq = gp.copy()
        gq[k] = -depth * band
        gs = gq.copy()
        gs[(k + 1) % len(gs)] = -10 * band
        s.exp_count = 0
        s.positivity_fallback(lev, gq, hp, gs, hp.copy(), tgt)
        assert (s.exp_count == 1) == takes


def _mirror_problem():
    """A periodic box on the 28-point Gauss-Hermite grid whose state is mirror
    symmetric about the horizontal mid-line (rho, u, T even in y, v odd)."""
    import dataclasses
    import math
    p = W.periodic_box(6, 8, Lx=1.0, Ly=1.0, Kn=0.05, nv=28)
    yc = (np.arange(p.nj) + 0.5) / p.nj
    xc = (np.arange(p.ni) + 0.5) / p.ni
    Yc, Xc = np.meshgrid(yc, xc, indexing="ij")
    return dataclasses.replace(p, vel_kind="gh", gh_scale_T=1.0,
                               rho0=1.0 + 0.3 * np.cos(2 * math.pi * Yc) + 0.1 * np.sin(2 * math.pi * Xc),
                               u0=0.2 * np.cos(2 * math.pi * Yc), v0=0.15 * np.sin(2 * math.pi * Yc),
                               T0=1.0 + 0.2 * np.cos(2 * math.pi * Yc))


def test_merged_points_on_a_symmetry_axis_keep_the_mirror_symmetry():
    # Reading R34.  The 4x4 blocks of nodes 12..15 straddle xi_y = 0 on the
    # 28-point Gauss-Hermite grid, so their merged points lie on the axis; a
    # state mirror-symmetric in y then stays symmetric to round-off (the
    # reflected cell at the reflected velocity), which it does not if the sign
    # of the mean's rounding residue picks the upwind side at xi . n = 0.
    from oracle.solver import Solver
    p = _mirror_problem()
    o = Solver(p, compat=4)
    nb = p.nv // 2
    k = np.zeros((nb, nb), np.uint8)
    k[6:8, 0:4] = 2                      # quads qy = 3, qx = 0, 1 (blocks by 6..7)
    k[6:8, 10:14] = 2                    # quads qy = 3, qx = 5, 6
    kap = k.ravel()
    lev = lv.Level(o.base, kap)
    axis = [q for q in range(lev.N) if len(lev.members[q]) == 16]
    assert len(axis) == 4 and all(lev.xi[q, 1] == 0.0 for q in axis)
    # the mirror image of every level point is a level point
    key = {(round(x, 12), round(y, 12)): q for q, (x, y) in enumerate(lev.xi)}
    mirror = np.array([key[(round(x, 12), round(-y + 0.0, 12))] for x, y in lev.xi])
    o.set_levels([kap], np.zeros(p.n_cells, np.int64))
    for _ in range(3):
        o.step()
    ni, nj = p.ni, p.nj
    scale = max(np.max(np.abs(g)) for g in o.g)
    worst = 0.0
    for j in range(nj):
        for i in range(ni):
            a, b = i + ni * j, i + ni * (nj - 1 - j)
            worst = max(worst, np.max(np.abs(o.g[a] - o.g[b][mirror])) / scale)
    assert worst < 1e-13, worst
