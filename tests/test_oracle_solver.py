"""Pins of the oracle's DUGKS step (uniform and multi-level velocity spaces).

Pinned against: the exact collisionless solution of the discrete-velocity
system (free-molecular limit, tau -> infinity), the exact Euler Riemann
solution for the near-continuum Sod tube (plausibility), the fixed point of
a uniform equilibrium, mass conservation in a closed cavity, conservation to
round-off across levels (Sec. 3.4) and the runtime-model fit of Sec. 4.6.
"""
import math
import os

import numpy as np
import pytest
from scipy.special import erfc

import workloads as W
from oracle import costmodel
from oracle import kinetic as kin
from oracle import levels as lv
from oracle.solver import AdaptParams, Solver

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_uniform_equilibrium_is_fixed_point():
    # BGK (Pr = 1): the compatibility-corrected Maxwellian is its own collision
    # target and a uniform state has zero flux divergence
    p = W.periodic_box(4, 3, Lx=1.0, Ly=0.75, Kn=0.05, nv=13, vmax=4.0, kind="uniform", Pr=1.0)
    s = Solver(p, compat=4)
    g0 = [x.copy() for x in s.g]
    for _ in range(3):
        s.step()
    err = max(np.max(np.abs(a - b)) for a, b in zip(s.g, g0))
    assert err < 1e-13


def test_closed_cavity_conserves_mass():
    p = W.cavity(6, nv=12, Kn=0.1)
    s = Solver(p, compat=4)
    t0 = s.totals()
    for _ in range(4):
        s.step()
    t1 = s.totals()
    assert abs(t1[0] - t0[0]) < 1e-13
    assert abs(t1[1] - t0[1]) > 1e-8       # the moving lid does transfer momentum


def test_periodic_totals_round_off():
    p = W.perturb(W.periodic_box(6, 4, Lx=1.0, Ly=0.5, Kn=0.02, nv=13, vmax=4.0, kind="sine"), seed=3)
    s = Solver(p, compat=4)
    t0 = s.totals()
    for _ in range(4):
        s.step()
    assert np.max(np.abs(s.totals() - t0)) < 1e-13


def _free_molecular(ncell, t_end):
    p = W.sod_1d(ncell, Kn=1e8, nv=41, vmax=5.0)
    s = Solver(p, compat=0)
    nsteps = int(round(t_end / s.dt))
    s.dt = t_end / nsteps
    for _ in range(nsteps):
        s.step()
    x = s.mesh.xc[:, 0]
    xi = s.xi_base_D[:, 0]
    w = s.base.w
    # exact solution of the discrete-velocity free transport: f(x, xi, t) = f0(x - xi t, xi)
    rho = np.zeros(ncell)
    for rl, Tl, side in ((1.0, 1.0, 1), (0.125, 0.8, -1)):
        g0, _ = kin.maxwell(xi[:, None], rl, np.zeros(1), Tl, 1.0, 0)
        # cell average of the indicator of the upstream state
        for c in range(ncell):
            xl, xr = x[c] - 0.5 / ncell, x[c] + 0.5 / ncell
            a = (xl - xi * t_end - 0.5) * side
            b = (xr - xi * t_end - 0.5) * side
            frac = np.clip((np.minimum(-a, 0) - np.minimum(-b, 0)) / (1.0 / ncell), 0, 1) if side == 1 else None
            lo = xl - xi * t_end
            hi = xr - xi * t_end
            if side == 1:
                frac = np.clip((np.minimum(hi, 0.5) - np.minimum(lo, 0.5)) / (hi - lo), 0, 1)
            else:
                frac = np.clip((np.maximum(hi, 0.5) - np.maximum(lo, 0.5)) / (hi - lo), 0, 1)
            rho[c] += np.sum(w * g0 * frac)
    num = s.fields()[:, 0]
    return np.mean(np.abs(num - rho))


@pytest.mark.slow
def test_free_molecular_limit_converges():
    e1 = _free_molecular(50, 0.05)
    e2 = _free_molecular(100, 0.05)
    assert e2 < 0.7 * e1
    assert e2 < 5e-3


def _euler_exact(x, t, gamma, L, R_):
    """Textbook exact Riemann solver (two-rarefaction/shock Newton on p*)."""
    rl, ul, pl = L
    rr, ur, pr = R_
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)

    def fk(p, rk, pk, ck):
        if p > pk:
            A, B = 2 / ((gamma + 1) * rk), (gamma - 1) / (gamma + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2 * ck / (gamma - 1) * ((p / pk) ** ((gamma - 1) / (2 * gamma)) - 1)

    lo, hi = 1e-8, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fk(mid, rl, pl, cl) + fk(mid, rr, pr, cr) + ur - ul > 0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (fk(ps, rr, pr, cr) - fk(ps, rl, pl, cl))
    out = np.zeros((len(x), 3))
    for k, xx in enumerate(x):
        S = (xx - 0.5) / t
        if S < us:
            if ps <= pl:
                shl = ul - cl
                rsl = rl * (ps / pl) ** (1 / gamma)
                csl = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                stl = us - csl
                if S < shl:
                    out[k] = L
                elif S > stl:
                    out[k] = (rsl, us, ps)
                else:
                    u = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * ul + S)
                    c = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - S))
                    r = rl * (c / cl) ** (2 / (gamma - 1))
                    out[k] = (r, u, pl * (c / cl) ** (2 * gamma / (gamma - 1)))
            else:
                raise NotImplementedError
        else:
            rsr = rr * ((ps / pr + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * ps / pr + 1))
            Ss = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
            out[k] = R_ if S > Ss else (rsr, us, ps)
    return out


@pytest.mark.slow
def test_sod_near_continuum_matches_euler():
    p = W.sod_1d(200, Kn=1e-3, nv=101, vmax=10.0)
    s = Solver(p, compat=0)
    nsteps = 400                                   # t = 0.1
    for _ in range(nsteps):
        s.step()
    t = nsteps * s.dt
    f = s.fields()
    ex = _euler_exact(s.mesh.xc[:, 0], t, 5.0 / 3.0, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    err = np.mean(np.abs(f[:, 0] - ex[:, 0])) / np.mean(ex[:, 0])
    assert err < 0.03


def _mlvs_problem():
    return W.periodic_box(8, 2, Lx=1.0, Ly=0.25, Kn=0.05, nv=24, vmax=5.0, kind="sine", amp=0.5)


def test_mlvs_with_no_merging_equals_uvs_exactly():
    p = _mlvs_problem()
    a = Solver(p, compat=4)
    b = Solver(p, compat=4, adapt=AdaptParams(1e-2, 0.0, 0.0, 0.05, False, 2))
    for _ in range(3):
        a.step()
        b.step()
    assert all(np.array_equal(x, y) for x, y in zip(a.g, b.g))
    assert len(b.levels) == 1


def test_mlvs_multilevel_conserves_to_round_off():
    p = _mlvs_problem()
    b = Solver(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 1e-3, 0.02, True, 2))
    t0 = b.totals()
    for _ in range(4):
        b.step()
    assert len(b.levels) >= 2
    assert np.max(np.abs(b.totals() - t0)) < 1e-13


def test_cross_level_native_fluxes_share_moments():
    p = _mlvs_problem()
    b = Solver(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 1e-3, 0.02, True, 2))
    b.adapt()
    b.cell_stage()
    b.slope_stage()
    m = b.mesh
    found = 0
    for f in range(m.n_faces):
        L, R = m.fL[f], m.fR[f]
        if b.cell_level[L] == b.cell_level[R]:
            continue
        acc = {L: [np.zeros_like(b.g[L]), np.zeros_like(b.h[L])],
               R: [np.zeros_like(b.g[R]), np.zeros_like(b.h[R])]}
        b.cross_face(f, acc)
        A, B = b.levels[b.cell_level[L]], b.levels[b.cell_level[R]]
        mL = lv.moments4(A.xi, A.w, acc[L][0], acc[L][1])
        mR = -lv.moments4(B.xi, B.w, acc[R][0], acc[R][1])
        assert np.allclose(mL, mR, rtol=1e-13, atol=1e-15)
        found += 1
    assert found > 0


def test_tau_one_gives_a_single_shared_level():
    p = _mlvs_problem()
    b = Solver(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 0.0, 1.0, False, 100))
    b.step()
    assert len(b.levels) == 1
    c = Solver(p, compat=4)
    c.set_levels([b.levels[0].kappa], np.zeros(p.n_cells, np.int64))
    c.step()
    assert all(np.allclose(x, y, rtol=0, atol=1e-15) for x, y in zip(b.g, c.g))


def test_interval_zero_adapts_only_when_asked():
    # reading R23: with interval 0 the steps never adapt by themselves; the
    # result equals the same steps without adaptation parameters
    p = _mlvs_problem()
    a = Solver(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 0.0, 0.05, False, 0))
    b = Solver(p, compat=4)
    for _ in range(2):
        a.step()
        b.step()
    assert len(a.levels) == 1 and a.step_count == 2
    assert all(np.array_equal(x, y) for x, y in zip(a.g, b.g))
    a.adapt()
    assert any(L.N < a.base.N for L in a.levels)


def test_runtime_model_fit_reproduces_paper():
    rows = np.loadtxt(os.path.join(GOLD, "h9_threshold.txt"))
    tau, nrep, nbar, ncross, meas, model = rows.T
    lam, c, r2 = costmodel.fit_runtime_model(nbar, ncross, meas, 7921, 10176, 10767.19)
    assert abs(lam - 0.30264) < 5e-5 and abs(c - 0.03917) < 5e-5 and abs(r2 - 0.925) < 1e-3
    est = costmodel.model_time(nbar, ncross, 7921, 10176, 10767.19, 0.30264, 0.03917)
    assert np.allclose(est, model, atol=0.15)
    wins, thr = costmodel.multilevel_wins(714.698 / 7921, 1033 / 7921, 537 / 10176, 0.30264)
    assert wins and abs(thr - 0.133) < 1e-3


def test_exponential_positivity_fallback_on_level_switches_and_neighbour_rows():
    """Positivity mode "exp": level switches whose linear correction turns a
    nonnegative g negative take the exponential correction instead; the
    switched state is then nonnegative, the conserved totals stay exact to
    round-off, and mode "keep" on the same switch leaves negative values."""
    p = W.perturb(W.periodic_box(10, 4, Lx=1.0, Ly=0.4, Kn=0.05, nv=24, vmax=5.0, kind="sine", amp=0.5), seed=2)
    nb = p.nv // 2
    kap = [np.zeros(nb * nb, np.uint8)] + [W.random_kappa(nb, nb, 7 + k) for k in range(2)]
    cl = W.striped_levels(p.ni, p.nj, 3, 1)
    keep = Solver(p, compat=4, positivity="keep")
    keep.set_levels(kap, cl)
    assert keep.neg_count > 0 and min(np.min(g) for g in keep.g) < 0
    o = Solver(p, compat=4, positivity="exp")
    t0 = o.totals()
    o.set_levels(kap, cl)
    assert o.exp_count > 0 and o.exp_fail == 0
    assert min(np.min(g) / np.max(g) for g in o.g) >= -o.POS_EPS
    assert np.max(np.abs(o.totals() - t0)) < 1e-14 * np.max(np.abs(t0))
    n0 = o.exp_count
    o.step()                                   # neighbour rows mapped across levels
    assert o.exp_count > n0
    assert np.max(np.abs(o.totals() - t0)) < 1e-14 * np.max(np.abs(t0))
    with pytest.raises(ValueError):
        Solver(p, compat=4, positivity="exp", map_moments=9)
