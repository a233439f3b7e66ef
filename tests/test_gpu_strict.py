"""Strict mode through the C ABI (Sec. 3.3: the positivity check after every
correction, made an error instead of a count): a state with T <= 0 set from
the host, a state that turns non-finite, a positivity violation in the
neighbour mapping, and a healthy run that strict mode leaves bit for bit
unchanged."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

E_NUMERIC = -5


def _m():
    import paper_2609_35258_amd as m
    return m


def _status(fn, *args):
    m = _m()
    st = fn(*args)
    return st, m.lib().mlvs_last_error().decode()


def test_strict_rejects_host_set_nonpositive_temperature():
    m = _m()
    p = W.cavity(8, nv=12, Kn=0.1)
    g = m.Solver.from_problem(p, compat=4)
    g.step(2)
    st = g.get_state()
    gs = [a.copy() for a, _ in st]
    hs = [b.copy() for _, b in st]
    vx, vw = m.gauss_hermite(12, p.R, 1.0)
    xi2 = (vx[:, None] ** 2 + vx[None, :] ** 2).ravel()
    # cell 13: h so negative that rho E < rho u^2 / 2, i.e. T < 0
    hs[13] = -(xi2 + 5.0) * gs[13]
    g.set_state(gs, hs)
    g.set_strict(1)
    code, msg = _status(m.lib().mlvs_step, g.h, 1)
    print("strict:", code, msg, flush=True)
    assert code == E_NUMERIC
    assert "before the first step" in msg and "cell 13" in msg
    # the same state without strict mode: the call succeeds (only counted)
    g.set_strict(0)
    assert m.lib().mlvs_step(g.h, 1) == 0
    g.close()


def test_strict_catches_the_step_that_goes_bad():
    # a time step 40 times the CFL limit: the explicit transport overshoots and
    # some cell's density or temperature leaves the positive range within a
    # few steps; strict mode names that step
    m = _m()
    p = W.perturb(W.cavity(8, nv=12, Kn=0.1), seed=3, amp=0.3)
    dt0 = m.Solver.from_problem(p, compat=4).dt
    g = m.Solver.from_problem(p, compat=4, dt=40 * dt0)
    g.set_strict(1)
    with pytest.raises(m.MLVSError) as ei:
        g.step(50)
    print(ei.value, flush=True)
    assert "mlvs error %d" % E_NUMERIC in str(ei.value) and "after step" in str(ei.value)
    g.close()


def test_strict_positivity_bit():
    m = _m()
    p = W.perturb(W.periodic_box(10, 4, Lx=1.0, Ly=0.4, Kn=0.05, nv=24, vmax=5.0, kind="sine", amp=0.5), seed=2)
    nb = p.nv // 2
    kap = np.stack([np.zeros(nb * nb, np.uint8)] + [W.random_kappa(nb, nb, 7 + k) for k in range(2)])
    cl = W.striped_levels(p.ni, p.nj, 3, 1)
    g = m.Solver.from_problem(p, compat=4)
    g.set_levels(kap, cl)
    n0 = g.neg_count()
    g.set_strict(2)
    with pytest.raises(m.MLVSError) as ei:
        g.step(1)
    print(ei.value, flush=True)
    assert "mlvs error %d" % E_NUMERIC in str(ei.value) and g.neg_count() > n0
    g.close()


def test_strict_mode_leaves_a_healthy_run_unchanged():
    m = _m()
    p = W.perturb(W.periodic_box(8, 4, Lx=1.0, Ly=0.5, Kn=0.05, nv=16, vmax=4.0, kind="sine"), seed=1)
    a = m.Solver.from_problem(p, compat=4)
    b = m.Solver.from_problem(p, compat=4)
    b.set_strict(1)
    a.step(4)
    b.step(4)
    for (ga, ha), (gb, hb) in zip(a.get_state(), b.get_state()):
        assert np.array_equal(ga, gb) and np.array_equal(ha, hb)
    with pytest.raises(m.MLVSError):
        b.set_strict(4)
    a.close()
    b.close()
