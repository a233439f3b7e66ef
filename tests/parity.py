"""Helpers shared by the GPU parity tests (method arithmetic only through the oracle)."""
import numpy as np

from oracle import levels as lv


def state_error(gpu_state, oracle_g, oracle_h):
    """max|g_gpu - g_orc| / max|g_orc| over all cells (and the same for h);
    infinite when either side holds a NaN."""
    for a, b, c in zip(gpu_state, oracle_g, oracle_h):
        if not (np.all(np.isfinite(a[0])) and np.all(np.isfinite(a[1])) and np.all(np.isfinite(b))
                and np.all(np.isfinite(c))):
            return float("inf"), float("inf")
    eg = max(float(np.max(np.abs(a[0] - b))) for a, b in zip(gpu_state, oracle_g))
    eh = max(float(np.max(np.abs(a[1] - b))) for a, b in zip(gpu_state, oracle_h))
    sg = max(float(np.max(np.abs(b))) for b in oracle_g)
    sh = max(float(np.max(np.abs(b))) for b in oracle_h)
    return eg / sg, eh / sh


def rel_l2(a, b, vol):
    """Volume-weighted relative L2 difference."""
    return float(np.sqrt(np.sum(vol * (a - b) ** 2) / np.sum(vol * b ** 2)))


def near_threshold(o, C_split, C_merge, eps_merge=None, rel=1e-9, cells=None):
    """Per cell and 2x2 block of V_base: True where the criterion's decision
    rests on a tie, i.e. a block containing it has an indicator I_B within rel
    of C_split or C_merge, or (eps_merge given) a transport error eps_B within
    rel of eps_merge (oracle side, Sec. 3.2).  cells: the oracle cells to
    examine (default all), one row each."""
    out = []
    base = o.base
    for c in (range(o.mesh.n_cells) if cells is None else cells):
        L = o.levels[o.cell_level[c]]
        gb, hb = lv.refine_to_base(L, o.g[c], o.h[c])
        M1, M2 = lv.indicators(base, gb, hb)
        S = lv.flux_scale(base, gb, hb) if eps_merge else None
        amb = np.zeros(base.Nb, bool)
        for s in (1, 2, 3):
            n = 1 << (s - 1)
            for by in range(base.nby // n):
                for bx in range(base.nbx // n):
                    I = lv.block_indicator(base, M1, M2, s, bx, by)
                    tie = any(abs(I - C) <= rel * C for C in (C_split, C_merge))
                    if eps_merge and not tie:
                        e = lv.block_flux_error(base, gb, hb, S, s, bx, by)
                        tie = abs(e - eps_merge) <= rel * eps_merge
                    if tie:
                        amb[base.block_children2(s, bx, by)] = True
        out.append(amb)
    return np.array(out)


def oracle_catalogue(p, n_masks, seed, C_split, C_merge, eps_merge, amp=0.5):
    """A level catalogue for the full-size tests from seeded inputs and the
    oracle alone: the base grid (kappa = 0) followed by the distinct masks the
    oracle's criterion (Sec. 3.2, with the flux test) gives on `n_masks` single
    cells of the problem's initial state under a seeded perturbation of
    amplitude `amp`.  Masks of real distributions keep the velocity space fine
    where the distribution is large, so every level carries a usable state."""
    import workloads as W
    from oracle.solver import Solver as Oracle
    q = W.perturb(p, seed, amp)
    rng = np.random.default_rng(seed)
    nb = int(q.nv) // 2
    out = [np.zeros(nb * nb, np.uint8)]
    for c in rng.choice(int(p.n_cells), size=n_masks, replace=False):
        if getattr(q, "unstructured", False):
            cell = W.upatch(q, int(c), hops=0)[0]
        else:
            cell = W.patch(q, int(c) % q.ni, int(c) // q.ni, 1, 1)
        o = Oracle(cell, compat=4)
        k = lv.criterion(o.levels[0], o.g[0], o.h[0], C_split, C_merge, eps_merge, True)
        if not any(np.array_equal(k, m) for m in out):
            out.append(k)
    return np.stack(out)


def oracle_sensitivity(make, steps, eps=1e-15, trials=2, seed=0):
    """Per step, the largest change (relative to the largest |g|) of the
    oracle's state when its initial g~, h~ carry relative noise of size eps:
    the spread the result has anyway under rounding.  make() returns a fresh
    oracle at the starting state.  Where a configuration is ill-conditioned
    (a cell whose mass sits almost all in one merged point makes its
    correction systems nearly singular) this exceeds the usual 1e-12 bound,
    and a GPU result can differ from the oracle by as much without either
    being wrong."""
    ref = make()
    out = np.zeros(steps)
    runs = []
    for t in range(trials):
        o = make()
        rng = np.random.default_rng(seed + t)
        o.g = [x * (1.0 + eps * rng.uniform(-1, 1, x.shape)) for x in o.g]
        o.h = [x * (1.0 + eps * rng.uniform(-1, 1, x.shape)) for x in o.h]
        runs.append(o)
    for k in range(steps):
        ref.step()
        scale = max(np.max(np.abs(x)) for x in ref.g)
        for o in runs:
            o.step()
            out[k] = max(out[k], max(np.max(np.abs(a - b)) for a, b in zip(o.g, ref.g)) / scale)
    return out
