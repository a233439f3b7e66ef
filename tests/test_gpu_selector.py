"""Learned level selector on the GPU: network forward/backward against the FP64
oracle, BF16 inference, features and criterion-judged labels against the
oracle, and a learned adaptation run (trained on solver snapshots, judged by the
criterion, conservation kept)."""
import time

import numpy as np
import pytest

import workloads as W
from oracle import levels as lv
from oracle import mlp
from oracle.solver import AdaptParams
from oracle.solver import Solver as Oracle
from tests.parity import near_threshold

pytestmark = pytest.mark.gpu


def _m():
    import paper_2609_35258_amd as m
    return m


def _net(K=4, B=257, seed=3):
    th = W.mlp_init_params(K, seed)
    rng = np.random.default_rng(seed + 1)
    X = rng.normal(size=(B, 10))
    y = rng.integers(0, K, size=B)
    th[-20:-10] = rng.normal(size=10) * 0.1
    th[-10:] = rng.uniform(0.5, 2.0, size=10)
    return th, X, y


@pytest.mark.parametrize("K,B", [(4, 257), (16, 1), (2, 33), (16, 4100)])
def test_network_forward_backward_matches_oracle(K, B):
    # ragged batches (not a multiple of the 16-sample workgroup pass), one
    # sample, 2 and 16 classes, and more passes than partial gradients (4100
    # samples: 257 passes on 256 workgroups, one of which takes two)
    th, X, y = _net(K, B=B)
    th32 = th.astype(np.float32)
    probs, grad, loss = _m().mlp_eval(th32, K, X.astype(np.float32), y)
    lo, go, po = mlp.loss_and_grad(th32.astype(np.float64), X.astype(np.float32).astype(np.float64), y, K)
    assert np.allclose(probs, po, rtol=1e-4, atol=1e-6)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    assert np.max(np.abs(grad - go)) <= 1e-4 * np.max(np.abs(go))


def test_bf16_inference_agrees_with_fp32():
    K = 5
    th, X, y = _net(K, B=2000, seed=9)
    c32, p32 = _m().mlp_predict(th, K, X, bf16=False)
    c16, p16 = _m().mlp_predict(th, K, X, bf16=True)
    _, po, _ = mlp.forward(th.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64), K)
    top2 = np.sort(po, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 1e-4
    assert np.all(c32[clear] == np.argmax(po, axis=1)[clear])
    assert np.mean(c16 == c32) > 0.97
    assert np.max(np.abs(p16 - p32)) < 0.05


@pytest.mark.parametrize("K,B", [(2, 33), (5, 2001), (16, 1000)])
def test_inference_matches_oracle(K, B):
    # FP32 evaluation against the FP64 forward; BF16 matrix-core inference
    # against the oracle's BF16 forward (same roundings, exact sums).  Ragged
    # batches (not a multiple of the 16-sample tile) and 2 to 16 classes.
    th, X, _ = _net(K, B=B, seed=11 + K)
    th32 = th.astype(np.float32)
    X32 = X.astype(np.float32)
    c32, p32 = _m().mlp_predict(th32, K, X32, bf16=False)
    c16, p16 = _m().mlp_predict(th32, K, X32, bf16=True)
    t64 = th32.astype(np.float64)
    z, po, _ = mlp.forward(t64, X32.astype(np.float64), K)
    assert np.allclose(p32, po, rtol=0, atol=1e-5)
    top2 = np.sort(z, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 1e-4
    assert np.all(c32[clear] == np.argmax(z, axis=1)[clear])
    zb, pb = mlp.forward_bf16(t64, X32, K)
    err = np.abs(p16 - pb)
    # FP32 accumulation order differs; a hidden activation that lands on the
    # other side of a bfloat16 rounding boundary moves a probability by ~1e-4
    print("K", K, "B", B, "bf16 prob error max", err.max(), "median", np.median(err), flush=True)
    assert err.max() < 2e-3 and np.median(err) < 1e-5
    top2 = np.sort(zb, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 1e-2
    assert clear.mean() > 0.9
    assert np.all(c16[clear] == np.argmax(zb, axis=1)[clear])


def test_features_match_oracle():
    p = W.perturb(W.cylinder(16, 8, Kn=0.1, nv=24, vmax=10.0), seed=5, amp=0.1)
    o = Oracle(p, compat=4)
    g = _m().Solver.from_problem(p, compat=4)
    o.step(); g.step(1)
    f = o.fields()
    xi, w = o.vset(0)
    sig = np.array([mlp.cell_stress(xi, w, o.g[c], f[c, 0], f[c, 1:3], f[c, 3], p.R) for c in range(p.n_cells)])
    grad = mlp.cell_gradient(o.mesh, f[:, 0])
    ref = mlp.features(f[:, 0], f[:, 1], f[:, 2], f[:, 3], f[:, 4], f[:, 5], sig[:, 0], sig[:, 1], grad,
                       o.mesh.vol, p.R, p.T_ref, o.mu(f[:, 3]))
    got = g.features()
    assert np.allclose(got, ref, rtol=2e-5, atol=2e-6)
    g.close()


def test_features_match_oracle_unstructured():
    # the density gradient by least squares over the face neighbours
    p = W.perturb(W.two_cavity(16, nv=16, vmax=7.0, ratio=0.3), seed=6, amp=0.1)
    o = Oracle(p, compat=4)
    g = _m().Solver.from_problem(p, compat=4)
    o.step(); g.step(1)
    f = o.fields()
    xi, w = o.vset(0)
    sig = np.array([mlp.cell_stress(xi, w, o.g[c], f[c, 0], f[c, 1:3], f[c, 3], p.R) for c in range(p.n_cells)])
    grad = mlp.cell_gradient(o.mesh, f[:, 0])
    ref = mlp.features(f[:, 0], f[:, 1], f[:, 2], f[:, 3], f[:, 4], f[:, 5], sig[:, 0], sig[:, 1], grad,
                       o.mesh.vol, p.R, p.T_ref, o.mu(f[:, 3]))
    got = g.features()
    assert np.allclose(got, ref, rtol=2e-5, atol=2e-6)
    g.close()


def _catalogue_problem(seed=4):
    p = W.perturb(W.periodic_box(12, 6, Lx=1.0, Ly=0.5, Kn=0.05, nv=32, vmax=5.0, kind="sine", amp=0.5), seed=seed)
    o1 = Oracle(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 1e-3, 0.03, True, 100))
    kap, cl = lv.cluster_masks(o1.criterion_masks(), 0.03)
    return p, kap, cl


def test_labels_match_oracle():
    p, kap, cl = _catalogue_problem()
    o = Oracle(p, compat=4, adapt=AdaptParams(5e-3, 2.5e-3, 1e-3, 0.03, True, 100))
    o.set_levels(kap, cl)
    g = _m().Solver.from_problem(p, compat=4, adapt=dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3,
                                                         tau_clust=0.03, flux_test=True, interval=0))
    g.set_levels(np.stack(kap), cl)
    ko = o.criterion_masks()
    lab_o = mlp.label_from_masks(ko, np.stack(kap), [L.N for L in o.levels])
    lab_g = g.labels()
    # labels are integers: equal on every cell whose mask rests on no tie of an
    # indicator or transport error with a threshold
    amb = near_threshold(o, 5e-3, 2.5e-3, 1e-3).any(axis=1)
    diff = (lab_g != lab_o) & ~amb
    assert not diff.any(), (np.nonzero(diff)[0], lab_g[diff], lab_o[diff])
    assert amb.mean() < 0.05, amb.mean()
    g.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_tail_check_matches_oracle(precision):
    # the tail-mass check of a seeded proposed level per cell against the
    # oracle's; base grid 21^2 (one full and one partial 16-point tile per
    # axis, and an odd edge row and column outside every 2x2 block), a
    # catalogue of seeded masks with 8x8, 4x4 and 2x2 merges, C_split at the
    # median of the oracle's largest block indicators so that both outcomes
    # occur; cells whose indicator ties with C_split are excepted
    p = W.perturb(W.cylinder(16, 8, Kn=0.1, nv=21, vmax=10.0), seed=6, amp=0.1)
    nb = 21 // 2
    kap = np.stack([np.zeros(nb * nb, np.uint8)] + [W.random_kappa(nb, nb, seed=s) for s in (1, 2, 3, 4)])
    cl = W.block_levels(16, 8, len(kap), seed=6, block=4)
    o = Oracle(p, compat=4)
    o.set_levels(list(kap), cl)
    n = p.n_cells
    prop = np.random.default_rng(7).integers(0, len(kap), size=n)
    res = [lv.tail_check(o.levels[o.cell_level[c]], o.g[c], o.h[c], kap[prop[c]], 1.0) for c in range(n)]
    imax = np.array([r[1] for r in res])
    C = float(np.median(imax[np.isfinite(imax)]))
    ok_o = imax <= C
    g = _m().Solver.from_problem(p, precision=precision, compat=4,
                                 adapt=dict(C_split=C, C_merge=C / 2, eps_merge=1e-3, tau_clust=0.03,
                                            flux_test=True, interval=0))
    g.set_levels(kap, cl)
    ok_g = g.selector_check(prop)
    tie = np.abs(imax - C) <= (1e-9 if precision == 64 else 1e-5) * C
    print("precision", precision, "accepted", ok_g.mean(), "ties", int(tie.sum()), flush=True)
    assert 0.2 < ok_o.mean() < 0.8
    diff = (ok_g != ok_o) & ~tie
    assert not diff.any(), (np.nonzero(diff)[0], imax[diff], C)
    with pytest.raises(_m().MLVSError):
        g.selector_check(np.full(n, len(kap)))
    g.close()


def test_adam_steps_match_oracle():
    # two full-batch training steps on the device (forward, backward, Adam)
    # against the oracle's gradient and Adam update from the same start
    K = 3
    th, X, y = _net(K, B=512, seed=5)
    X = X.astype(np.float32)
    lr = 1e-2
    P, rep = _m().mlp_train(th.astype(np.float32), K, X, y, epochs=2, batch=len(y), lr=lr, val_frac=0.0, seed=7)
    assert rep["steps"] == 2
    t = th.astype(np.float32).astype(np.float64)
    X64 = X.astype(np.float64)
    # the device sets the standardisation block from the training samples first
    mu = X64.mean(axis=0)
    sd = np.sqrt(((X64 - mu) ** 2).mean(axis=0))
    t[-20:-10] = mu.astype(np.float32)
    t[-10:] = sd.astype(np.float32)
    m1 = np.zeros_like(t)
    v1 = np.zeros_like(t)
    gmin = np.full_like(t, np.inf)
    for step in (1, 2):
        _, gr, _ = mlp.loss_and_grad(t, X64, y, K)
        gmin = np.minimum(gmin, np.abs(gr) / np.max(np.abs(gr)))
        t, m1, v1 = mlp.adam_step(t, gr, m1, v1, step, lr=lr)
    n_tr = len(t) - 20
    err = np.abs(P[:n_tr] - t[:n_tr])
    # each Adam step moves a weight by about lr sign(g); where the gradient is
    # not tiny (Adam's eps and FP32 rounding decide there) the two sides agree
    # to a small fraction of that (FP32 against FP64 gradients)
    clear = gmin[:n_tr] > 1e-5
    assert clear.mean() > 0.9
    assert np.max(err[clear]) < 2e-3 * lr, np.max(err[clear])
    assert np.max(err) <= 2.0 * lr * (1 + 1e-6)
    assert np.allclose(P[n_tr:], t[n_tr:], rtol=1e-6, atol=0)


def test_selector_trained_from_context_snapshots():
    """The context-bound selector calls: record snapshots of the context's own
    state, train on them, switch learned adaptation on and off."""
    m = _m()
    p = W.perturb(W.periodic_box(24, 8, Lx=1.0, Ly=1.0 / 3, Kn=0.05, nv=32, vmax=5.0, kind="sine", amp=0.5), seed=8)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.05, flux_test=True, interval=0)
    g = m.Solver.from_problem(p, compat=4, adapt=ap)
    g.step(2)
    g.adapt()
    K = len(g.level_info()[0])
    assert K >= 2
    with pytest.raises(m.MLVSError):
        g.selector_train(epochs=1)                 # nothing recorded yet
    with pytest.raises(m.MLVSError):
        g.selector_enable(True)                    # no network
    n = 0
    for snap in range(12):
        g.step(5)
        n = g.selector_snapshot(reset=(snap == 0))
    assert n == 12 * g.n_cells
    rep = g.selector_train(epochs=40, batch=256, lr=3e-3, val_frac=0.2, seed=1)
    print("training", rep, flush=True)
    assert rep["loss_last"] < rep["loss_first"] and rep["val_acc"] > 0.6
    P, Kp = g.selector_params()
    assert Kp == K and len(P) == m.mlp_nparams(K) and np.all(np.isfinite(P))
    t0 = g.totals()
    g.selector_enable(True)
    r1 = g.adapt()
    assert r1["n_unique"] == -1 and r1["n_fallback"] < g.n_cells
    g.step(3)
    assert np.max(np.abs(g.totals() - t0)) < 1e-12
    g.selector_enable(False)
    assert g.adapt()["n_unique"] >= 1
    g.close()


def test_learned_adaptation_run():
    m = _m()
    p = W.perturb(W.periodic_box(24, 8, Lx=1.0, Ly=1.0 / 3, Kn=0.05, nv=32, vmax=5.0, kind="sine", amp=0.5), seed=8)
    # adaptation only when called: one full adaptation builds the catalogue, which
    # then stays frozen while snapshots are collected and during learned adaptation
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.05, flux_test=True, interval=0)
    g = m.Solver.from_problem(p, compat=4, adapt=ap)
    g.step(2)
    g.adapt()
    K = len(g.level_info()[0])
    assert K >= 2
    X, Y = [], []
    for snap in range(12):                      # snapshots in time order
        g.step(5)
        X.append(g.features())
        Y.append(g.labels())
    X = np.concatenate(X)
    Y = np.concatenate(Y)
    ok = Y >= 0
    params, rep = m.mlp_train(W.mlp_init_params(K, 0), K, X[ok], Y[ok], epochs=40, batch=256, lr=3e-3,
                              val_frac=0.2, seed=1)
    print("training", rep, flush=True)
    assert rep["loss_last"] < rep["loss_first"]
    assert rep["val_acc"] > 0.6
    t0 = g.totals()
    g.selector_set(params, K)
    reps = []
    for _ in range(3):
        t = time.perf_counter()
        reps.append(g.adapt())
        g.step(5)
    print("learned adaptations", reps, flush=True)
    assert np.max(np.abs(g.totals() - t0)) < 1e-12
    assert all(r["n_fallback"] < g.n_cells for r in reps)
    g.close()


def test_learned_adaptation_run_unstructured():
    # the learned path on the two-cavity mesh: train on snapshots, then adapt
    m = _m()
    p = W.perturb(W.two_cavity(16, nv=16, vmax=7.0, ratio=0.05), seed=3, amp=0.3)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.02, flux_test=True, interval=0)
    g = m.Solver.from_problem(p, compat=4, adapt=ap)
    g.step(2)
    g.adapt()
    K = len(g.level_info()[0])
    assert 2 <= K <= 16, K
    X, Y = [], []
    for snap in range(8):
        g.step(5)
        X.append(g.features())
        Y.append(g.labels())
    X = np.concatenate(X)
    Y = np.concatenate(Y)
    ok = Y >= 0
    params, rep = m.mlp_train(W.mlp_init_params(K, 0), K, X[ok], Y[ok], epochs=30, batch=256, lr=3e-3,
                              val_frac=0.2, seed=1)
    print("training", rep, flush=True)
    assert rep["loss_last"] < rep["loss_first"]
    t0 = g.totals()
    g.selector_set(params, K)
    reps = [g.adapt() for _ in range(2)]
    g.step(3)
    print("learned adaptations", reps, flush=True)
    assert abs(g.totals()[0] - t0[0]) < 1e-12 * t0[0]
    assert all(r["n_fallback"] < g.n_cells for r in reps)
    g.close()


def test_learned_gain_over_criterion():
    """What the network gains: from the same state and catalogue, a learned
    adaptation runs the criterion only on the cells the tail-mass check rejects
    (the criterion adaptation runs it on every cell), with few misclassified
    cells, and the run stays close to the criterion-adapted run."""
    m = _m()
    p = W.perturb(W.periodic_box(24, 8, Lx=1.0, Ly=1.0 / 3, Kn=0.05, nv=32, vmax=5.0, kind="sine", amp=0.5), seed=8)
    ap = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=1e-3, tau_clust=0.05, flux_test=True, interval=0)
    crit = m.Solver.from_problem(p, compat=4, adapt=ap)
    crit.step(2)
    crit.adapt()
    K = len(crit.level_info()[0])
    X, Y = [], []
    for _ in range(12):
        crit.step(5)
        X.append(crit.features())
        Y.append(crit.labels())
    X, Y = np.concatenate(X), np.concatenate(Y)
    ok = Y >= 0
    params, rep = m.mlp_train(W.mlp_init_params(K, 0), K, X[ok], Y[ok], epochs=40, batch=256, lr=3e-3,
                              val_frac=0.2, seed=1)
    lrn = m.Solver.from_problem(p, compat=4, adapt=ap)
    lrn.set_levels(np.stack([crit.level_kappa(k) for k in range(K)]), crit.cell_levels())
    st = crit.get_state()
    lrn.set_state([g for g, _ in st], [h for _, h in st])
    lrn.selector_set(params, K)
    n = p.n_cells
    fb, mis = [], []
    for _ in range(3):
        lab = lrn.labels()
        pred, _ = m.mlp_predict(params, K, lrn.features(), bf16=True)
        mis.append(np.mean(pred[lab >= 0] != lab[lab >= 0]))
        t0 = time.perf_counter()
        crit.adapt()
        t1 = time.perf_counter()
        r = lrn.adapt()
        t2 = time.perf_counter()
        fb.append(r["n_fallback"] / n)
        crit.step(5)
        lrn.step(5)
        print("adapt ms criterion %.2f learned %.2f, criterion cells %d of %d, misclassified %.3f"
              % (1e3 * (t1 - t0), 1e3 * (t2 - t1), r["n_fallback"], n, mis[-1]), flush=True)
    assert max(fb) < 0.2, fb
    assert np.mean(mis) < 0.15, mis
    fc, fl = crit.moments(), lrn.moments()
    for k in (0, 3):
        assert np.sqrt(np.sum((fl[:, k] - fc[:, k]) ** 2) / np.sum(fc[:, k] ** 2)) < 1e-3
    crit.close()
    lrn.close()
