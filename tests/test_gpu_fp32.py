"""FP32-storage path: fields within 1e-3 relative L2 of the FP64 oracle, totals
conserved to FP32 round-off, on uniform and multi-level runs."""
import numpy as np
import pytest

import workloads as W
from oracle.solver import Solver as Oracle
from tests.parity import rel_l2

pytestmark = pytest.mark.gpu


def _gpu(p, **kw):
    import paper_2609_35258_amd as m
    return m.Solver.from_problem(p, **kw)


def _check_fields(o, g, tol=1e-3):
    fo, fg = o.fields(), g.moments()
    vol = o.mesh.vol
    out = {}
    for k, name in ((0, "rho"), (1, "u"), (2, "v"), (3, "T")):
        ref = fo[:, k]
        if np.max(np.abs(ref)) < 1e-8:
            continue
        out[name] = rel_l2(fg[:, k], ref, vol)
    p = fo[:, 0] * fo[:, 3]
    out["p"] = rel_l2(fg[:, 0] * fg[:, 3], p, vol)
    print("fp32 rel L2", out, flush=True)
    for name, e in out.items():
        assert e < tol, (name, e)
    return out


def test_fp32_cavity_fields():
    p = W.cavity(16, Kn=0.075, nv=28)
    o = Oracle(p, compat=4)
    g = _gpu(p, precision=32, compat=4)
    for _ in range(20):
        o.step()
    g.step(20)
    _check_fields(o, g)
    g.close()


def test_fp32_cylinder_fields_and_heat_flux():
    p = W.cylinder(24, 10, Kn=0.1, nv=41, vmax=10.0)
    o = Oracle(p, compat=4)
    g = _gpu(p, precision=32, compat=4)
    for _ in range(6):
        o.step()
    g.step(6)
    _check_fields(o, g)
    qo = o.fields()[:, 4:6]
    qg = g.moments()[:, 4:6]
    scale = np.max(np.abs(qo))
    assert np.max(np.abs(qg - qo)) < 2e-3 * scale
    g.close()


def test_fp32_cylinder_eight_moment_compat():
    p = W.cylinder(24, 10, Kn=0.1, nv=41, vmax=10.0)
    o = Oracle(p, compat=8)
    g = _gpu(p, precision=32, compat=8)
    for _ in range(6):
        o.step()
    g.step(6)
    _check_fields(o, g)
    g.close()


def test_fp32_multilevel_conservation():
    p = W.perturb(W.periodic_box(12, 6, Lx=1.0, Ly=0.5, Kn=0.05, nv=24, vmax=5.0, kind="sine", amp=0.5), seed=3)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.02, flux_test=True, interval=5)
    g = _gpu(p, precision=32, compat=4, adapt=ap)
    t0 = g.totals()
    g.step(20)
    t1 = g.totals()
    npts, ncells, ncross = g.level_info()
    assert len(npts) >= 2 and ncross > 0
    rel = np.abs(t1 - t0) / np.maximum(np.abs(t0), 1.0)
    # FP32 storage: drift at the level of float rounding per step
    assert np.max(rel) < 20 * 20 * np.finfo(np.float32).eps, rel
    g.close()
