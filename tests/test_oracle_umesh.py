"""Pins of the oracle's unstructured-mesh path (geometry, least-squares
slopes with Venkatakrishnan's limiter, the step on triangles and
quadrilaterals).

Pinned against: exact areas and perimeters of the two-cavity domain, the
structured geometry of the same quadrilaterals, exact gradients of linear
fields, closed-form values of Venkatakrishnan's function, the limiter's
bound at the face centres (eps = 0), the first-order step of the structured
solver on the same quadrilaterals, and mass conservation in the closed
two-cavity domain.
"""
import numpy as np
import pytest

import workloads as W
from oracle import solver as S
from oracle import umesh as um
from oracle.mesh import Mesh
from oracle.umesh import UMesh, lsq_limited_slope, venkat


def _cavity_with_jump(n=8, nv=12, rho_r=1e-3):
    p = W.cavity(n, Kn=1e-3, nv=nv, vel_kind="nc", vmax=7.0)
    xc = 0.5 * (p.X[:-1, :-1] + p.X[:-1, 1:])
    p.rho0 = np.where(xc < 0.5, 1.0, rho_r)
    return p


def test_two_cavity_geometry():
    p = W.two_cavity(16)
    m = UMesh(p)
    # two unit squares and a 1 x 1/8 channel
    assert abs(m.vol.sum() - 2.125) < 1e-12
    # perimeter: 2 * 4 - 2 * 1/8 (the channel mouths) + 2 * 1 (channel sides)
    assert abs(m.ba.sum() - 9.75) < 1e-12
    sizes = np.diff(p.cell_ptr)
    assert int(sizes.sum()) == 2 * m.n_faces + m.n_bfaces
    assert m.n_cells == 2 * 2 * 16 * 16 + 16 * 2
    # every cell is closed: sum of outward A n over its faces vanishes
    for c in range(m.n_cells):
        s = np.zeros(2)
        for kind, f in m.edges[c]:
            if kind == "f":
                s += (1.0 if m.fL[f] == c else -1.0) * m.fa[f] * m.fn[f]
            else:
                s += m.ba[f] * m.bn[f]
        assert np.max(np.abs(s)) < 1e-15
    # the normal of an interior face points from L to R
    d = m.xc[m.fR] - m.xc[m.fL]
    assert np.all(np.sum(d * m.fn, axis=1) > 0)
    assert np.all(np.sum(m.bd * m.bn, axis=1) > 0)


def test_quadrilaterals_match_structured_geometry():
    p = W.cavity(7, nv=8)
    m, ms = UMesh(W.as_unstructured(p)), Mesh(p)
    assert np.allclose(m.vol, ms.vol, rtol=0, atol=1e-15)
    assert np.allclose(m.xc, ms.xc, rtol=0, atol=1e-15)
    assert m.n_faces == ms.n_faces and m.n_bfaces == ms.n_bfaces
    key = lambda L, R: (min(L, R), max(L, R))
    a = {key(L, R): A for L, R, A in zip(m.fL, m.fR, m.fa)}
    b = {key(L, R): A for L, R, A in zip(ms.fL, ms.fR, ms.fa)}
    assert a.keys() == b.keys()
    assert max(abs(a[k] - b[k]) for k in a) < 1e-15
    assert abs(m.hmin - ms.hmin) < 1e-15


@pytest.mark.parametrize("split", ["none", "random"])
def test_least_squares_exact_for_linear_fields(split):
    p = W.as_unstructured(W.cavity(6, nv=8), split=split, seed=3)
    m = UMesh(p)
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=3), rng.normal(size=(3, 2))
    for c in range(m.n_cells):
        if any(nb < 0 for nb, _, _ in m.cell_faces[c]):
            continue                     # the zero-gradient ghost is not linear
        phi = lambda x: a + b @ x
        fc = phi(m.xc[c])
        nv = [phi(m.xc[nb]) for nb, _, _ in m.cell_faces[c]]
        sig = lsq_limited_slope(m, c, fc, nv, eps2=1e300)      # limiter inactive
        assert np.allclose(sig, b, rtol=0, atol=1e-12)


def test_unlimited_least_squares_gradient_exact_for_linear_fields():
    p = W.two_cavity(16)
    m = UMesh(p)
    b = np.array([0.4, -1.3])
    for c in range(0, m.n_cells, 5):
        if any(nb < 0 for nb, _, _ in m.cell_faces[c]):
            continue
        fc = np.array([2.0 + b @ m.xc[c]])
        nv = [np.array([2.0 + b @ m.xc[nb]]) for nb, _, _ in m.cell_faces[c]]
        assert np.allclose(um.lsq_gradient(m, c, fc, nv), b[None, :], rtol=0, atol=1e-12)


def test_venkatakrishnan_closed_forms():
    d = np.array([1e-3, 0.5, 3.0])
    # V(d+, d-) = (y^2 + 2y)/(y^2 + y + 2) with y = d+/d- when eps = 0
    for y, v in ((0.0, 0.0), (1.0, 0.75), (2.0, 1.0), (4.0, 24.0 / 22.0)):
        assert np.allclose(venkat(y * d, d, 0.0), v, rtol=1e-15)
        assert np.allclose(venkat(-y * d, -d, 0.0), v, rtol=1e-15)
    assert np.all(venkat(d, 0.0 * d, 0.0) == 1.0)               # no extrapolation, no constraint
    assert np.allclose(venkat(0.0 * d, d, 1e300), 1.0)           # eps dominates
    # eps^2 enters as written: V(0, d) = eps^2 / (2 d^2 + eps^2)
    assert np.allclose(venkat(0.0 * d, d, 0.25), 0.25 / (2 * d * d + 0.25), rtol=1e-15)


def test_limited_reconstruction_stays_within_neighbours():
    p = W.two_cavity(16)
    m = UMesh(p)
    rng = np.random.default_rng(7)
    vals = rng.uniform(0.0, 1.0, size=(m.n_cells, 32))
    for c in range(0, m.n_cells, 7):
        nv = [None if nb < 0 else vals[nb] for nb, _, _ in m.cell_faces[c]]
        sig = lsq_limited_slope(m, c, vals[c], nv, eps2=0.0)
        lo = np.min([vals[c]] + [v for v in nv if v is not None], axis=0)
        hi = np.max([vals[c]] + [v for v in nv if v is not None], axis=0)
        for nb, fo, _ in m.cell_faces[c]:
            rec = vals[c] + sig @ fo
            assert np.all(rec >= lo - 1e-14) and np.all(rec <= hi + 1e-14)


def test_linear_field_unlimited_on_uniform_quads():
    # on a uniform quadrilateral mesh a linear field has d+ = 2 d- at every
    # face, where V = 1 exactly: the limiter keeps the exact gradient
    p = W.as_unstructured(W.cavity(6, nv=8))
    m = UMesh(p)
    b = np.array([0.3, -0.7])
    for c in range(m.n_cells):
        if any(nb < 0 for nb, _, _ in m.cell_faces[c]):
            continue
        fc = np.array([1.0 + b @ m.xc[c]])
        nv = [np.array([1.0 + b @ m.xc[nb]]) for nb, _, _ in m.cell_faces[c]]
        assert np.allclose(lsq_limited_slope(m, c, fc, nv), b[None, :], rtol=0, atol=1e-12)


def test_first_order_step_matches_structured(monkeypatch):
    # with every slope zero both paths are the first-order DUGKS on the same
    # quadrilaterals: faces, normals, boundary faces and the update agree
    monkeypatch.setattr(S, "van_leer", lambda a, b: np.zeros_like(a))
    monkeypatch.setattr(S, "lsq_limited_slope", lambda m, c, fc, nv, eps2=None: np.zeros((len(fc), 2)))
    p = W.perturb(_cavity_with_jump(6, nv=10, rho_r=0.3), seed=2, amp=0.05)
    a, b = S.Solver(p, compat=4), S.Solver(W.as_unstructured(p), compat=4)
    assert a.dt == b.dt
    for _ in range(3):
        a.step()
        b.step()
    err = max(np.max(np.abs(x - y)) for x, y in zip(a.g + a.h, b.g + b.h))
    assert err < 1e-13


def test_o_grid_as_quadrilaterals_matches_structured(monkeypatch):
    # the periodic seam of an O-grid closes by shared nodes; geometry and the
    # first-order step agree with the structured solver
    p = W.perturb(W.cylinder(16, 6, Kn=0.1, nv=10, vmax=10.0), seed=1, amp=0.05)
    m, ms = UMesh(W.as_unstructured(p)), Mesh(p)
    assert m.n_faces == ms.n_faces and m.n_bfaces == ms.n_bfaces
    assert np.allclose(m.vol, ms.vol, rtol=0, atol=1e-15)
    monkeypatch.setattr(S, "van_leer", lambda a, b: np.zeros_like(a))
    monkeypatch.setattr(S, "lsq_limited_slope", lambda m_, c, fc, nv, eps2=None: np.zeros((len(fc), 2)))
    a, b = S.Solver(p, compat=4), S.Solver(W.as_unstructured(p), compat=4)
    for _ in range(2):
        a.step()
        b.step()
    assert max(np.max(np.abs(x - y)) for x, y in zip(a.g + a.h, b.g + b.h)) < 1e-13


def test_first_order_differs_from_limited():
    # guard for the test above: the slopes do matter on this input
    p = W.perturb(_cavity_with_jump(6, nv=10, rho_r=0.3), seed=2, amp=0.05)
    a, b = S.Solver(p, compat=4), S.Solver(W.as_unstructured(p), compat=4)
    a.step(); b.step()
    assert max(np.max(np.abs(x - y)) for x, y in zip(a.g, b.g)) > 1e-6


def test_two_cavity_conserves_mass_and_stays_positive():
    p = W.two_cavity(16, nv=12, vmax=7.0)
    s = S.Solver(p, compat=4)
    t0 = s.totals()
    for _ in range(4):
        s.step()
    t1 = s.totals()
    assert abs(t1[0] - t0[0]) < 1e-13 * t0[0]
    f = s.fields()
    assert np.all(f[:, 0] > 0) and np.all(f[:, 3] > 0)
    # gas has entered the channel's right half
    right = np.array([x[0] > 0 for x in s.mesh.xc])
    assert np.max(f[right, 0]) > 1.5e-3


def test_absolute_eps_breaks_on_the_density_jump(monkeypatch):
    # why eps is relative: with the classic absolute eps^2 = (K h)^3 the tails
    # of a 1000:1 jump reconstruct negative and the face temperature fails
    orig = um.lsq_limited_slope

    def absolute(m, c, fc, nv, eps2=None):
        return orig(m, c, fc, nv, eps2=(um.VENKAT_K * np.sqrt(m.vol[c])) ** 3)

    monkeypatch.setattr(S, "lsq_limited_slope", absolute)
    s = S.Solver(W.as_unstructured(_cavity_with_jump(8, nv=12)), compat=4)
    with np.errstate(all="ignore"):
        for _ in range(2):
            s.step()
        f = s.fields()
    assert not np.all(f[:, 3] > 0)
