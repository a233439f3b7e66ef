"""GPU parity of the uniform-velocity-space DUGKS step (FP64) against the oracle.

Both sides start from the same seeded macroscopic state; each side builds its
own quadrature, equilibrium and geometry.  Per step the whole g~, h~ state is
compared: max|gpu - oracle| / max|oracle| <= 1e-12.
"""
import numpy as np
import pytest

import workloads as W
from oracle.solver import Solver as Oracle
from tests.parity import state_error

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _gpu(p, **kw):
    import paper_2609_35258_amd as m
    return m.Solver.from_problem(p, **kw)


def _run_parity(p, steps, compat=4, face_compat=True):
    print("case", p.name, p.ni, p.nj, p.nv, "compat", compat, flush=True)
    o = Oracle(p, compat=compat, face_compat=face_compat)
    g = _gpu(p, compat=compat, face_compat=face_compat)
    assert abs(g.dt - o.dt) <= 1e-14 * o.dt
    st = g.get_state()
    e0 = state_error(st, o.g, o.h)
    assert max(e0) < TOL, ("initial", e0)
    worst = 0.0
    for k in range(steps):
        o.step()
        g.step(1)
        e = state_error(g.get_state(), o.g, o.h)
        worst = max(worst, *e)
        assert max(e) < TOL, (k, e)
    t_o, t_g = o.totals(), g.totals()
    # totals near zero (a symmetric momentum component) carry only rounding of
    # the order of the largest total times machine epsilon
    assert np.allclose(t_g, t_o, rtol=1e-12, atol=1e-14 * np.max(np.abs(t_o)))
    f_o, f_g = o.fields(), g.moments()
    assert np.allclose(f_g, f_o, rtol=1e-10, atol=1e-12)
    g.close()
    return worst


def test_sod_1d_plain_all_steps():
    # 1-D Sod, 200 cells, 101 Boole points on [-10, 10], BGK, correction off, 100 steps
    _run_parity(W.sod_1d(200, Kn=1e-3), 100, compat=0)


def test_sod_1d_kn01_compat():
    _run_parity(W.sod_1d(64, Kn=0.1, nv=41, vmax=8.0), 10, compat=4)


def test_cavity_gauss_hermite():
    _run_parity(W.cavity(12, Kn=0.075, nv=12), 5)


def test_cavity_ragged_newton_cotes():
    # odd velocity grid with xi = 0 rows/columns (zero normal velocity on faces)
    _run_parity(W.cavity(9, Kn=0.5, nv=17, vel_kind="nc", vmax=4.0), 4)


def test_cylinder_ogrid():
    _run_parity(W.cylinder(24, 10, Kn=0.1, nv=21, vmax=10.0), 4)


def test_cylinder_velocity_chunks(monkeypatch):
    # 441 points in chunks of 64: the reconstruction and update split every
    # row into 7 chunks whose partial moments are added in chunk order
    monkeypatch.setenv("MLVS_CHUNK", "64")
    _run_parity(W.cylinder(24, 10, Kn=0.1, nv=21, vmax=10.0), 3)


def test_jet_slot():
    _run_parity(W.jet(20, 12, Kn_jet=0.01, nv=21, vmax=7.0), 3)


def test_periodic_sine_no_face_compat():
    p = W.perturb(W.periodic_box(10, 6, Lx=1.0, Ly=0.6, Kn=0.02, nv=15, vmax=4.0, kind="sine"), seed=11)
    _run_parity(p, 5, face_compat=False)


@pytest.mark.parametrize("case", ["cavity", "cylinder", "periodic"])
def test_eight_moment_compat(case):
    # eight-moment compatibility correction of the cell and face targets:
    # heat flux (1 - Pr) q and zero deviatoric stress imposed as well
    if case == "cavity":
        p = W.cavity(12, Kn=0.075, nv=12)
    elif case == "cylinder":
        p = W.cylinder(24, 10, Kn=0.1, nv=21, vmax=10.0)
    else:
        p = W.perturb(W.periodic_box(10, 6, Lx=1.0, Ly=0.6, Kn=0.02, nv=15, vmax=4.0, kind="sine"), seed=11)
    _run_parity(p, 4, compat=8)


def test_periodic_totals_round_off_gpu():
    p = W.perturb(W.periodic_box(16, 8, Lx=1.0, Ly=0.5, Kn=0.02, nv=17, vmax=4.0, kind="sine"), seed=5)
    g = _gpu(p)
    t0 = g.totals()
    g.step(20)
    assert np.max(np.abs(g.totals() - t0)) < 1e-13
    g.close()


@pytest.mark.parametrize("ni,nj,nv", [(1, 1, 6), (2, 1, 8), (1, 3, 10), (3, 2, 7)])
def test_degenerate_meshes_and_short_rows(ni, nj, nv):
    # a single periodic cell (its own neighbour on every side), meshes one or
    # two cells wide, and velocity rows shorter than a wavefront (36 to 100
    # points, odd and even)
    p = W.perturb(W.periodic_box(ni, nj, Lx=0.2 * ni, Ly=0.2 * nj, Kn=0.05, nv=nv, vmax=4.0, kind="sine"), seed=ni + nj)
    _run_parity(p, 3)


def test_stress_matches_oracle():
    # deviatoric stress of the cavity after a few steps, against the oracle's
    # state (P_ab = sum w c_a c_b g, minus p on the diagonal)
    p = W.cavity(12, Kn=0.075, nv=12)
    o = Oracle(p, compat=4)
    g = _gpu(p)
    for _ in range(5):
        o.step()
    g.step(5)
    ref = np.zeros((p.n_cells, 3))
    for c in range(p.n_cells):
        xi, w = o.vset(o.cell_level[c])
        rho, u, T = o.macro(xi, w, o.g[c], o.h[c])
        cc = xi - u[None, :]
        pr = rho * p.R * T
        ref[c] = [np.sum(w * cc[:, 0] ** 2 * o.g[c]) - pr, np.sum(w * cc[:, 0] * cc[:, 1] * o.g[c]),
                  np.sum(w * cc[:, 1] ** 2 * o.g[c]) - pr]
    got = g.stress()
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref)) + 1e-14
    assert np.max(np.abs(ref[:, 1])) > 1e-6          # the lid shears the cavity
    g.close()
