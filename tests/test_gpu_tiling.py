"""Traversal tiles of structured meshes: retiling reorders the state rows on the
device without changing a value, later steps give the same state bit for bit
whatever the tiles (each face and cell is computed on its own, the fluxes
into a cell are added in a fixed face order), and the tile tuner runs and
caches its choice."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _gpu(p, **kw):
    import paper_2609_35258_amd as m
    return m.Solver.from_problem(p, **kw)


def _same(sa, sb):
    return all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) for x, y in zip(sa, sb))


@pytest.mark.parametrize("precision,graph", [(64, False), (32, True)])
def test_tiles_reorder_rows_and_leave_results_unchanged(precision, graph):
    p = W.perturb(W.periodic_box(20, 12, Lx=1.0, Ly=0.6, Kn=0.05, nv=20, vmax=5.0, kind="sine", amp=0.5), seed=7)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.02, flux_test=True, interval=3)
    a = _gpu(p, precision=precision, adapt=ap, graph=graph)
    b = _gpu(p, precision=precision, adapt=ap, graph=graph)
    assert a.tiling() == (16, 8)
    tiles = [(4, 4), (0, 0), (7, 3), (32, 8), (16, 8)]
    for k in range(10):
        if k % 2 == 0:
            s0 = b.get_state()
            b.set_tiling(*tiles[(k // 2) % len(tiles)])
            assert b.tiling() == tiles[(k // 2) % len(tiles)]
            assert _same(b.get_state(), s0), k          # a row copy, values unchanged
        a.step(1)
        b.step(1)
        assert _same(a.get_state(), b.get_state()), k
    assert b.counters()["adaptations"] >= 3
    a.close()
    b.close()


def test_tiles_persistent_step_and_errors():
    import paper_2609_35258_amd as m
    p = W.perturb(W.periodic_box(12, 6, Lx=1.0, Ly=0.5, Kn=0.05, nv=16, vmax=5.0, kind="sine", amp=0.4), seed=2)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.02, flux_test=True, interval=2)
    a = _gpu(p, precision=64, adapt=ap, graph=True)
    b = _gpu(p, precision=64, adapt=ap, graph=True)
    b.set_persistent(True)
    for k in range(5):
        b.set_tiling(*[(3, 2), (0, 0), (12, 6), (5, 5), (16, 8)][k])
        a.step(1)
        b.step(1)
        assert _same(a.get_state(), b.get_state()), k
    assert b.graph_info()["error"] == 0
    for bad in [(-1, 4), (4, 0), (0, 4), (5000, 2)]:
        with pytest.raises(m.MLVSError, match="bad tiles"):
            b.set_tiling(*bad)
    a.close()
    b.close()
    u = _gpu(W.two_cavity(16, nv=12, vmax=7.0, ratio=0.05), precision=64)
    assert u.tiling() == (0, 0)
    with pytest.raises(m.MLVSError, match="structured"):
        u.set_tiling(16, 8)
    u.close()


def test_tile_tuner_picks_and_caches(tmp_path):
    import paper_2609_35258_amd.autotune as at
    p = W.cylinder(32, 16, Kn=0.1, nv=21, vmax=10.0)
    s = _gpu(p, precision=32, graph=True)
    s.step(2)
    ref = _gpu(p, precision=32, graph=True)
    ref.step(2)
    cache = str(tmp_path / "t.json")
    r = at.autotune_tiles(s, 32, candidates=((16, 8), (8, 4), (0, 0)), reps=2, cache=cache)
    assert not r["from_cache"] and tuple(r["tiles"]) in {(16, 8), (8, 4), (0, 0)} and len(r["all_ms"]) == 3
    assert s.tiling() == tuple(r["tiles"])
    s.set_tiling(0, 0)
    r2 = at.autotune_tiles(s, 32, candidates=((16, 8), (8, 4), (0, 0)), reps=2, cache=cache)
    assert r2["from_cache"] and s.tiling() == tuple(r["tiles"])
    s.step(3)
    ref.step(3)
    assert _same(s.get_state(), ref.get_state())
    s.close()
    ref.close()
    u = _gpu(W.two_cavity(16, nv=12, vmax=7.0, ratio=0.05), precision=32)
    assert at.autotune_tiles(u, 32, cache=cache) == {}
    u.close()
