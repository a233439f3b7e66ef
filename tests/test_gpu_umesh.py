"""GPU parity of the unstructured-mesh path (triangles and quadrilaterals,
least-squares slopes with Venkatakrishnan's limiter) against the oracle.

* Two-cavity expansion (1000:1 density jump, mixed triangles and channel
  quadrilaterals) and a lid-driven cavity cut into triangles: FP64 UVS steps,
  <= 1e-12 of the largest value, in velocity chunks of 64 (staged step) and
  whole rows (fused step).
* Multi-level FP64: a fixed catalogue from the oracle's criterion and
  grouping on a perturbed state (four- and nine-moment mapping, four- and
  eight-moment compatibility), and criterion adaptation inside the step
  loop.
* FP32 storage: fields within 1e-5 relative L2 after a few steps.
* Degenerate meshes: one triangle with boundary faces only, two triangles, a
  quadrilateral beside a triangle; the cylinder O-grid taken as an
  unstructured mesh (seam closed by shared nodes).
* Full size (two-cavity at lattice spacing 1/48: 9504 cells, 101^2 velocity
  points, FP32, UVS and MLVS), from seeded inputs only (the initial state with
  a seeded perturbation; for MLVS the base grid and the oracle's criterion
  masks of a few seeded single-cell states, on seeded squares of the plane):
  sampled cells against an oracle step of the two-neighbour-ring patch around
  each (a cell's update reads its faces' upwind cells and their face
  neighbours only), <= 1e-6 of the largest value;
  the base-grid criterion masks of the sampled cells bit for bit (threshold
  ties excepted); the oracle's own time step from the full mesh equals the
  GPU's.
"""
import numpy as np
import pytest

import workloads as W
from oracle import levels as lv
from oracle.solver import AdaptParams
from oracle.solver import Solver as Oracle
from tests.parity import rel_l2, state_error

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _gpu(p, **kw):
    import paper_2609_35258_amd as m
    return m.Solver.from_problem(p, **kw)


def _tri_cavity(n=8, nv=12):
    p = W.perturb(W.cavity(n, Kn=0.05, nv=nv, vel_kind="nc", vmax=5.0), seed=4, amp=0.05)
    return W.as_unstructured(p, split="random", seed=5)


@pytest.mark.parametrize("chunk", ["64", None])
@pytest.mark.parametrize("case", ["two_cavity", "tri_cavity"])
def test_uvs_fp64(case, chunk, monkeypatch):
    if chunk:
        monkeypatch.setenv("MLVS_CHUNK", chunk)
    else:
        monkeypatch.delenv("MLVS_CHUNK", raising=False)
    p = W.two_cavity(16, nv=16, vmax=7.0) if case == "two_cavity" else _tri_cavity()
    print("case uvs", case, chunk, p.n_cells, flush=True)
    o = Oracle(p, compat=4)
    g = _gpu(p, compat=4)
    assert abs(g.dt - o.dt) < 1e-15 * o.dt
    t0 = g.totals()
    for k in range(3):
        o.step()
        g.step(1)
        e = state_error(g.get_state(), o.g, o.h)
        assert max(e) < TOL, (k, e)
    assert abs(g.totals()[0] - t0[0]) < 1e-13 * t0[0]
    g.close()


@pytest.mark.parametrize("mode", ["uvs", "mlvs"])
def test_o_grid_with_least_squares_slopes_fp64(mode):
    # the body-fitted cylinder O-grid taken as an unstructured mesh: least
    # squares + Venkatakrishnan in place of van Leer per index direction
    p = W.perturb(W.cylinder(16, 8, Kn=0.1, nv=32, vmax=10.0), seed=3, amp=0.1)
    q = W.as_unstructured(p)
    print("case o-grid unstructured", mode, flush=True)
    o = Oracle(q, compat=4)
    g = _gpu(q, compat=4)
    if mode == "mlvs":
        o1 = Oracle(q, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 1e-3, 0.02, True, 100))
        kap, cl = lv.cluster_masks(o1.criterion_masks(), 0.02)
        assert len(kap) >= 2
        o.set_levels(kap, cl)
        g.set_levels(np.stack(kap), cl)
    for k in range(3):
        o.step()
        g.step(1)
        e = state_error(g.get_state(), o.g, o.h)
        assert max(e) < TOL, (k, e)
    g.close()


def _tiny(polys, nodes, bedges, rho):
    n = len(polys)
    ptr = np.concatenate([[0], np.cumsum([len(q) for q in polys])]).astype(np.int32)
    return W.UProblem("tiny", np.asarray(nodes, float), ptr, np.array([v for q in polys for v in q], np.int32),
                      np.asarray(bedges, np.int32).reshape(-1, 3), [W.BC(W.WALL, T=1.0), W.BC(W.WALL, u=0.1, T=1.2)],
                      np.asarray(rho, float), np.full(n, 0.05), np.zeros(n), np.ones(n), R=0.5, Pr=2.0 / 3.0, K=0,
                      omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0, Kn=0.1, cfl=0.5, vel_kind="nc", nv=12, vmax=5.0)


@pytest.mark.parametrize("case", ["one_triangle", "two_triangles", "quad_and_triangle"])
def test_degenerate_small_meshes_fp64(case):
    # a cell whose faces are all boundary faces (least squares from the
    # mirror ghosts alone), a two-cell mesh, and a mixed quad/triangle pair
    if case == "one_triangle":
        p = _tiny([(0, 1, 2)], [(0, 0), (1, 0), (0.3, 0.8)], [(0, 1, 0), (1, 2, 1), (2, 0, 0)], [1.0])
    elif case == "two_triangles":
        p = _tiny([(0, 1, 2), (0, 2, 3)], [(0, 0), (1, 0), (1, 1), (0, 1)],
                  [(0, 1, 0), (1, 2, 0), (2, 3, 1), (3, 0, 0)], [1.0, 0.5])
    else:
        p = _tiny([(0, 1, 4, 3), (1, 2, 4)], [(0, 0), (1, 0), (1.6, 0.2), (0, 1), (1, 1)],
                  [(0, 1, 0), (1, 2, 0), (2, 4, 1), (4, 3, 1), (3, 0, 0)], [1.0, 0.7])
    print("case tiny", case, flush=True)
    o = Oracle(p, compat=4)
    g = _gpu(p, compat=4)
    t0 = g.totals()
    for k in range(3):
        o.step()
        g.step(1)
        e = state_error(g.get_state(), o.g, o.h)
        assert max(e) < TOL, (case, k, e)
    assert abs(g.totals()[0] - t0[0]) < 1e-13 * t0[0]
    g.close()


def _perturbed(ratio=0.05):
    return W.perturb(W.two_cavity(16, nv=16, vmax=7.0, ratio=ratio), seed=3, amp=0.3)


@pytest.mark.parametrize("map_moments,compat", [(4, 4), (9, 8)])
def test_mlvs_fixed_catalog_fp64(map_moments, compat, monkeypatch):
    # catalogue from the oracle's criterion + grouping on a perturbed state
    monkeypatch.setenv("MLVS_CHUNK", "64")
    p = _perturbed()
    print("case mlvs fixed", map_moments, compat, flush=True)
    o1 = Oracle(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 1e-3, 0.02, True, 100))
    kap, cl = lv.cluster_masks(o1.criterion_masks(), 0.02)
    assert len(kap) >= 3
    o = Oracle(p, compat=compat, map_moments=map_moments)
    g = _gpu(p, compat=compat, map_moments=map_moments)
    o.set_levels(kap, cl)
    g.set_levels(np.stack(kap), cl)
    e = state_error(g.get_state(), o.g, o.h)
    assert max(e) < TOL, ("remap", e)
    _, _, ncross = g.level_info()
    assert ncross > 0
    t0 = g.totals()
    for k in range(3):
        o.step()
        g.step(1)
        e = state_error(g.get_state(), o.g, o.h)
        assert max(e) < TOL, (k, e)
    assert abs(g.totals()[0] - t0[0]) < 1e-13 * t0[0]       # walls exchange momentum and energy only
    g.close()


def test_mlvs_criterion_adaptation_fp64():
    p = _perturbed()
    print("case mlvs adapt", flush=True)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.02, flux_test=True, interval=2)
    o = Oracle(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 1e-3, 0.02, True, 2))
    g = _gpu(p, compat=4, adapt=ap)
    for k in range(3):
        o.step()
        g.step(1)
        assert np.array_equal(g.cell_levels(), o.cell_level), k
        e = state_error(g.get_state(), o.g, o.h)
        assert max(e) < TOL, (k, e)
    npts, _, ncross = g.level_info()
    print("levels", list(npts), "cross", ncross, flush=True)
    assert len(npts) >= 2
    g.close()


def test_fp32_two_cavity_fields():
    p = W.two_cavity(16, nv=16, vmax=7.0)
    print("case fp32", flush=True)
    o = Oracle(p, compat=4)
    g = _gpu(p, compat=4, precision=32)
    for _ in range(3):
        o.step()
    g.step(3)
    fo, fg = o.fields(), g.moments()
    for k in (0, 1, 3):
        e = rel_l2(fg[:, k], fo[:, k], o.mesh.vol)
        assert e < 1e-5, (k, e)
    g.close()


def _nearest(p, pts):
    xc = p.centroids()
    return [int(np.argmin(np.sum((xc - np.asarray(q)) ** 2, axis=1))) for q in pts]


# left cavity, channel entrance, jump, channel exit, right cavity, a wall corner
SAMPLE_POINTS = [(-1.0, 0.2), (-0.51, 0.01), (0.0, 0.0), (0.02, -0.05), (0.52, 0.03), (1.2, -0.3), (1.49, 0.49)]


@pytest.mark.parametrize("mode", ["uvs", "mlvs"])
def test_two_cavity_full_size_sampled_cells(mode, tmp_path):
    from oracle.solver import base_grid
    from oracle.umesh import UMesh
    from paper_2609_35258_amd import autotune
    from tests.parity import near_threshold
    import torch
    p = W.perturb(W.two_cavity(48, nv=101, vmax=7.0), seed=51, amp=0.1)
    print("case two-cavity 9504 cells 101^2 fp32", mode, flush=True)
    xi, _, _, _ = base_grid(p)
    dt = p.cfl * UMesh(p).hmin / float(np.max(np.sqrt(np.sum(xi * xi, axis=1))))
    ap = dict(C_split=0.01, C_merge=0.005, eps_merge=2e-5, tau_clust=0.05, flux_test=True, interval=0)
    g = _gpu(p, precision=32, compat=4, adapt=ap, graph=True)
    assert abs(g.dt - dt) <= 1e-14 * dt
    centres = _nearest(p, SAMPLE_POINTS)
    if mode == "uvs":
        # the criterion on the base grid, from the same seeded state
        masks = g.criterion()
        for c in centres:
            q, cells = W.upatch(p, c, hops=2)
            o = Oracle(q, compat=4, dt=dt)
            ko = lv.criterion(o.levels[0], o.g[0], o.h[0], ap["C_split"], ap["C_merge"], ap["eps_merge"], True)
            amb = near_threshold(o, ap["C_split"], ap["C_merge"], ap["eps_merge"], cells=[0])[0]
            diff = (masks[c] != ko) & ~amb
            print("criterion cell", c, "kappa max", int(ko.max()), "ties", int(amb.sum()), flush=True)
            assert not diff.any(), (c, int(diff.sum()))
    else:
        from tests.parity import oracle_catalogue
        kap = oracle_catalogue(p, 5, 51, ap["C_split"], ap["C_merge"], ap["eps_merge"])
        levels = W.point_levels(p.centroids(), len(kap), 51, h=0.125)
        g.set_levels(kap, levels)
        npts, _, ncross = g.level_info()
        print("levels", list(npts), "cross", ncross, flush=True)
        assert len(npts) == len(kap) >= 2 and ncross > 0
        # plus a cell beside a cross-level face in the channel
        nbr = W.cell_neighbours(p)
        xc = p.centroids()
        chan = [c for c in range(len(levels)) if abs(xc[c][0]) < 0.45 and any(levels[n] != levels[c] for n in nbr[c])]
        assert chan, "no cross-level face in the channel"
        centres = centres + chan[:1]
    autotune.autotune(g, 32, cache=str(tmp_path / "t.json"))
    g.step(1)
    for c in centres:
        q, cells = W.upatch(p, c, hops=2)
        o = Oracle(q, compat=4, dt=dt)
        if mode == "mlvs":
            o.set_levels(list(kap), levels[cells])
        o.step()
        ga, ha = g.get_cell(c)
        eg = np.max(np.abs(ga - o.g[0])) / np.max(np.abs(o.g[0]))
        eh = np.max(np.abs(ha - o.h[0])) / np.max(np.abs(o.h[0]))
        print("cell", c, "points", len(ga), "patch", len(cells), "error", eg, eh, flush=True)
        assert max(eg, eh) < 1e-6, (c, eg, eh)
    g.close()
    del g
    torch.cuda.empty_cache()
