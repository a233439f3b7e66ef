"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (graph-captured steps, autotuned launch variants,
velocity chunks chosen per level set, tiled traversal).

* Cavity 64x64, 28^2 Gauss-Hermite, FP64, MLVS with the benchmark's
  adaptation settings: after the warm-up and the adaptation at step 100, one
  GPU step against one oracle step from the same state and level catalogue,
  every cell, <= 1e-12 of the largest value.
* Cylinder 256x128 O-grid, 101^2 Newton-Cotes, FP32, UVS and MLVS (the
  benchmark's base-grid warm-up, then criterion levels), and the slot jet
  512x256, 161^2 Newton-Cotes (25921 points, about 110 GB of device state in
  the UVS form), FP32, UVS and MLVS: sampled cells.  The oracle steps the
  5x5-cell patch of the mesh around each sampled cell from the GPU's state,
  with the GPU's time step.  A cell's update reads nothing farther than two
  cells away (the upwind neighbour's slope), so the patch's own boundary does
  not reach the centre; the centre after one step agrees to 1e-6 of its
  largest value (FP32 storage against FP64).
"""
import numpy as np
import pytest

import workloads as W
from oracle.solver import Solver as Oracle
from tests.parity import state_error

pytestmark = pytest.mark.gpu


def _m():
    import paper_2609_35258_amd as m
    return m


def test_cavity_full_size_bench_configuration(tmp_path):
    from paper_2609_35258_amd import autotune
    m = _m()
    p = W.cavity(64, Kn=0.075, nv=28)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=5e-5, tau_clust=0.05, flux_test=True, interval=100)
    print("case cavity 64x64 fp64 mlvs", flush=True)
    g = m.Solver.from_problem(p, precision=64, compat=4, adapt=ap, graph=True)
    g.step(100)
    autotune.autotune(g, 64, cache=str(tmp_path / "t.json"))
    g.step(1)                                   # adapted at step 100
    npts, ncells, _ = g.level_info()
    kap = np.stack([g.level_kappa(k) for k in range(len(npts))])
    cl = g.cell_levels()
    st = g.get_state()
    o = Oracle(p, compat=4, dt=g.dt)
    o.set_levels(list(kap), cl)
    o.g = [x[0].copy() for x in st]
    o.h = [x[1].copy() for x in st]
    o.step()
    g.step(1)
    e = state_error(g.get_state(), o.g, o.h)
    print("levels", list(npts), "error", e, flush=True)
    assert max(e) < 1e-12, e
    t_o, t_g = o.totals(), g.totals()
    assert np.allclose(t_g, t_o, rtol=1e-12, atol=1e-14 * np.max(np.abs(t_o)))
    g.close()


# sampled cells (i, j) of the O-grid: near the wall, in the shock layer, in the
# wake and in the far field, away from the periodic seam
SAMPLES = [(40, 2), (128, 3), (5, 17), (200, 40), (100, 77), (250, 125)]
# of the jet: at the slot, in the jet, at the side and far walls
JET_SAMPLES = [(2, 128), (3, 127), (5, 131), (7, 120), (2, 2), (509, 253)]


def _sampled_parity(p, mode, samples, warm):
    from paper_2609_35258_amd import autotune
    import torch
    m = _m()
    ap = dict(C_split=0.01, C_merge=0.005, eps_merge=2e-5, tau_clust=0.05, flux_test=True, interval=0)
    g = m.Solver.from_problem(p, precision=32, compat=4, adapt=ap if mode == "mlvs" else None, graph=True)
    g.step(warm)                                # base-grid warm-up
    if mode == "mlvs":
        g.adapt()
    g.step(2)
    autotune.autotune(g, 32, cache=None)
    ni = p.ni
    if mode == "mlvs":
        npts, _, ncross = g.level_info()
        kap = np.stack([g.level_kappa(k) for k in range(len(npts))])
        levels = g.cell_levels()
        assert len(npts) >= 2 and ncross > 0
        # plus the first cell (away from the mesh edges) with a cross-level
        # face towards +i and the first with one towards +j
        Lg = levels.reshape(p.nj, ni)
        inner = np.zeros_like(Lg, bool)
        inner[2:-3, 2:-3] = True
        for d in (1, 0):
            cross = inner & (Lg != np.roll(Lg, -1, axis=d))
            jj, ii = np.nonzero(cross)
            assert len(ii) > 0, "no cross-level face along axis %d" % d
            samples = list(samples) + [(int(ii[0]), int(jj[0]))]
    patches = {}
    for (i, j) in samples:
        i0, j0 = i - 2, max(j - 2, 0)
        i0, j0 = min(max(i0, 0), ni - 5), min(j0, p.nj - 5)
        cells = [(i0 + a) + ni * (j0 + b) for b in range(5) for a in range(5)]
        patches[(i, j)] = (i0, j0, cells, [g.get_cell(c) for c in cells])
    g.step(1)
    for (i, j), (i0, j0, cells, before) in patches.items():
        q = W.patch(p, i0, j0)
        o = Oracle(q, compat=4, dt=g.dt)
        if mode == "mlvs":
            o.set_levels(list(kap), levels[cells])
        o.g = [x[0].copy() for x in before]
        o.h = [x[1].copy() for x in before]
        o.step()
        k = (i - i0) + 5 * (j - j0)
        ga, ha = g.get_cell(i + ni * j)
        eg = np.max(np.abs(ga - o.g[k])) / np.max(np.abs(o.g[k]))
        eh = np.max(np.abs(ha - o.h[k])) / np.max(np.abs(o.h[k]))
        print("cell", (i, j), "points", len(ga), "error", eg, eh, flush=True)
        assert max(eg, eh) < 1e-6, ((i, j), eg, eh)
    g.close()
    del g
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["uvs", "mlvs"])
def test_cylinder_full_size_sampled_cells(mode):
    print("case cylinder 256x128 fp32", mode, flush=True)
    _sampled_parity(W.cylinder(256, 128, Kn=0.1, nv=101, vmax=10.0), mode, SAMPLES, 100)


@pytest.mark.parametrize("mode", ["uvs", "mlvs"])
def test_jet_full_size_sampled_cells(mode):
    print("case jet 512x256 161^2 fp32", mode, flush=True)
    _sampled_parity(W.jet(512, 256, Kn_jet=1e-3, nv=161, vmax=7.0), mode, JET_SAMPLES, 100)
