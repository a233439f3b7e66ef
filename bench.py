"""Benchmark: MLVS-DUGKS cell-velocity updates/s on one MI355X, MLVS vs UVS.

Workload (synthetic, deterministic): 2-D lid-driven cavity, 64 x 64 uniform
cells on [0,1]^2, lid Mach 0.16, Kn 0.075, Shakhov Pr 2/3, 28 x 28
Gauss-Hermite base velocity grid, FP64.  MLVS: criterion C_split 5e-3,
C_merge 2.5e-3, transport-error test eps 5e-5, tau_clust 0.05, adaptation
every 100 steps (levels built from the distributions); UVS: the same run on
the fixed base grid.  A step is one pass of the whole hot path (adaptation at
its interval, cell stage, neighbour mapping, same-level / boundary /
cross-level faces, update).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6

ADAPT = dict(C_split=5e-3, C_merge=2.5e-3, eps_merge=5e-5, tau_clust=0.05, flux_test=True, interval=100)


def workload(args):
    return W.cavity(args.n, Kn=0.075, nv=args.nv)


def run_gpu(p, steps, warmup, precision, adapt, graph=True, tune=True):
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=adapt, graph=graph)
    s.step(warmup)
    if tune:
        s.tuned = autotune.autotune(s, precision)
    torch.cuda.synchronize()
    c0 = s.counters()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = s.counters()
    return s, t1 - t0, c1["cell_updates"] - c0["cell_updates"], c1["iface_points"] - c0["iface_points"]


def stage_profile(s, reps=20):
    """Mean ms per launch of each stage the step launches (HIP events on the context stream)."""
    out = {}
    for st in s.step_stages():
        items, pts = s.stage_size(st)
        if items == 0:
            continue
        out[st] = {"ms": s.time_stage(st, reps), "items": items, "points": pts}
    return out


# algorithmic bytes per velocity point of each stage (FP64 values, 8 B; FP32, 4 B):
#   cell:        read g~,h~ + write phi_bar+ g,h                         -> 4 values
#   face_rec:    read phi_bar+ g,h of the upwind cell + write phi_bar_f  -> 4 values
#   face_target: per-face records only (ALU: the target's moment pass)    -> 0 values
#   update:      read g~,h~ and phi_bar+ g,h, the cell's face rows (each shared
#                by two cells: 4 faces x 2 / 2) + write g~,h~             -> 10 values
#   xface:       per V_int point, read both sides' phi_bar+ (2x2) + write one native row (2) -> 6 values
#   ghost:       read source phi_bar+ + write mapped row                 -> 4 values
#   face (fused face_rec + face_target)                                  -> 4 values
#   update_cell (fused update + next cell stage): the update's 10 + write the
#                new phi_bar+ g,h (the new state is the update's own output) -> 12 values
ALG_VALUES = {"cell": 4, "face_rec": 4, "face_target": 0, "update": 10, "xface": 6, "ghost": 4, "face": 4,
              "update_cell": 12}


def cpu_baseline(p, sample_steps=2, sample_cells=256):
    """The oracle as it stands on the same workload: full-size steps from the
    initial state plus the criterion on a sample of cells (scaled to the whole
    mesh), the adaptation amortised over its interval."""
    from oracle import levels as lv
    from oracle.solver import Solver as Oracle
    o = Oracle(p, compat=4)
    t0 = time.perf_counter()
    for c in range(min(sample_cells, o.mesh.n_cells)):
        lv.criterion(o.levels[0], o.g[c], o.h[c], ADAPT["C_split"], ADAPT["C_merge"], ADAPT["eps_merge"],
                     ADAPT["flux_test"])
    t_crit = (time.perf_counter() - t0) * o.mesh.n_cells / min(sample_cells, o.mesh.n_cells)
    t0 = time.perf_counter()
    for _ in range(sample_steps):
        o.step()
    t_step = (time.perf_counter() - t0) / sample_steps
    pts = float(o.mesh.n_cells * o.levels[0].N)
    rate = pts / (t_step + t_crit / ADAPT["interval"])
    return {"value": rate, "unit": "cell-velocity updates/s", "cores": 1, "kind": "oracle",
            "sample": "%dx%d cavity, %d-point base grid: %d oracle steps (%.2f s/step) + criterion on %d cells "
                      "(scaled to %d cells: %.1f s), adaptation amortised over %d steps"
                      % (p.ni, p.nj, o.levels[0].N, sample_steps, t_step, sample_cells, o.mesh.n_cells,
                         t_crit, ADAPT["interval"])}


LEARNED_ADAPT = dict(C_split=0.01, C_merge=0.005, eps_merge=2e-5, tau_clust=0.05, flux_test=True, interval=0)


def learned_vs_criterion(precision=32, n_theta=256, n_r=128, nv=101, warm=100, snaps=32, every=10, rounds=6):
    """Learned vs criterion adaptation on the same GPU.

    Supersonic cylinder (Ma 3, Kn 0.1, Shakhov), n_theta x n_r cells and an
    nv^2 Newton-Cotes base grid (by default the full-size case: 32 snapshots of
    32768 cells, about 1e6 samples).  A criterion run builds the catalogue (one
    full adaptation after `warm` base-grid steps) and collects (features,
    criterion label) snapshots every `every` steps; the network is trained on
    the GPU on the earlier 80% of the snapshots.  A second solver starts from the same
    state and levels with the selector on.  Both then run `rounds` rounds of
    `every` steps plus one adaptation: full criterion adaptation (the paper's
    method, catalogue rebuilt) vs learned adaptation (frozen catalogue, tail-mass
    check, criterion on rejected cells only)."""
    import torch
    import paper_2609_35258_amd as m
    p = W.cylinder(n_theta, n_r, Kn=0.1, nv=nv, vmax=10.0)
    crit = m.Solver.from_problem(p, precision=precision, compat=4, adapt=LEARNED_ADAPT)
    crit.step(warm)
    crit.adapt()
    K = len(crit.level_info()[0])
    X, Y = [], []
    for _ in range(snaps):
        crit.step(every)
        X.append(crit.features())
        Y.append(crit.labels())
    X = np.concatenate(X)
    Y = np.concatenate(Y)
    ok = Y >= 0
    params, trep = m.mlp_train(W.mlp_init_params(K, 0), K, X[ok], Y[ok], epochs=30, batch=1024, lr=3e-3,
                               val_frac=0.2, seed=0)
    lrn = m.Solver.from_problem(p, precision=precision, compat=4, adapt=LEARNED_ADAPT)
    lrn.set_levels(np.stack([crit.level_kappa(k) for k in range(K)]), crit.cell_levels())
    st = crit.get_state()
    lrn.set_state([g for g, _ in st], [h for _, h in st])
    lrn.selector_set(params, K)
    n = p.n_cells
    out = {"workload": "cylinder %dx%d, Ma 3, Kn 0.1, %dx%d Newton-Cotes on [-10,10]^2, fp%d, C_split 0.01, "
                       "C_merge 0.005, eps_merge 2e-5, tau_clust 0.05" % (n_theta, n_r, nv, nv, precision),
           "K": K, "samples": int(ok.sum()), "train": {k: trep[k] for k in ("loss_first", "loss_last", "train_acc",
                                                                           "val_acc", "ms")}}
    mis, fb, t_c, t_l, run_c, run_l = [], [], [], [], 0.0, 0.0
    for _ in range(rounds):
        feats, lab = lrn.features(), lrn.labels()
        pred, _ = m.mlp_predict(params, K, feats, bf16=True)
        v = lab >= 0
        mis.append(float(np.mean(pred[v] != lab[v])))
        for s, acc, tl in ((crit, t_c, "c"), (lrn, t_l, "l")):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = s.adapt()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s.step(every)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            acc.append(1e3 * (t1 - t0))
            if tl == "c":
                run_c += t2 - t0
            else:
                run_l += t2 - t0
                fb.append(rep["n_fallback"] / n)
    fc, fl = crit.moments(), lrn.moments()
    err = {}
    for k, name in ((0, "rho"), (1, "u"), (3, "T")):
        err[name] = float(np.sqrt(np.sum((fl[:, k] - fc[:, k]) ** 2) / np.sum(fc[:, k] ** 2)))
    npc, ncc, _ = crit.level_info()
    npl, ncl, _ = lrn.level_info()
    out.update({"misclassification": float(np.mean(mis)), "fallback_rate": float(np.mean(fb)),
                "criterion_adapt_ms": float(np.median(t_c)), "learned_adapt_ms": float(np.median(t_l)),
                "adapt_speedup": float(np.median(t_c) / np.median(t_l)),
                "end_to_end_s": {"criterion": run_c, "learned": run_l},
                "nbar": {"criterion": float(np.sum(npc * ncc) / n), "learned": float(np.sum(npl * ncl) / n)},
                "learned_vs_criterion_rel_l2": err})
    crit.close()
    lrn.close()
    return out


CYL_ADAPT = dict(C_split=0.01, C_merge=0.005, eps_merge=2e-5, tau_clust=0.05, flux_test=True, interval=0)
CYL_INTERVAL = 100


def jet_case(steps=100, warmup=100, precision=32, mode="both"):
    """Under-expanded slot jet into near vacuum at full size (512 x 256 cells,
    161^2 = 25921-point Newton-Cotes base grid on [-7,7]^2, about 110 GB of
    device state in the UVS form, FP32 storage), MLVS against UVS.  Both take
    `warmup` untimed base-grid steps from the initial state; the MLVS run then
    adapts (criterion levels) at the start of the timed steps, adaptation
    included in the timing.  Graph-captured steps, autotuned variants."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.jet(512, 256, Kn_jet=1e-3, nv=161, vmax=7.0)
    if mode == "uvs":
        u, t_u, upd_u, _ = run_gpu(p, steps, warmup + 2, precision, None)
        prof_u = stage_profile(u, reps=3)
        var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
        u.close()
        return {"uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                        "roofline": roofline(prof_u, precision, var_u,
                                             "jet512x256-nc161-fp32-uvs" if precision == 32 else None)}}
    s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=CYL_ADAPT, graph=True)
    s.step(warmup)
    s.adapt()
    s.step(2)
    autotune.autotune(s, precision)
    torch.cuda.synchronize()
    c0 = s.counters()
    t0 = time.perf_counter()
    s.adapt()
    s.step(steps)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    upd = s.counters()["cell_updates"] - c0["cell_updates"]
    npts, ncells, ncross = s.level_info()
    f_m = s.moments()
    mem_m = s.memory()
    prof = stage_profile(s, reps=3)
    s.close()
    del s
    torch.cuda.empty_cache()
    if mode == "mlvs":
        return {"value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "nbar": float(np.sum(npts * ncells) / np.sum(ncells)),
                "roofline": roofline(prof, precision)}
    u, t_u, upd_u, _ = run_gpu(p, steps, warmup + 2, precision, None)
    f_u = u.moments()
    mem_u = u.memory()
    prof_u = stage_profile(u, reps=3)
    var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
    u.close()
    del u
    torch.cuda.empty_cache()
    err = {name: float(np.sqrt(np.sum((f_m[:, k] - f_u[:, k]) ** 2) / np.sum(f_u[:, k] ** 2)))
           for k, name in ((0, "rho"), (1, "u"), (3, "T"))}
    return {"workload": "slot jet 512x256 on [0,32]x[-8,8], sonic slot |y| <= 0.5, background rho 0.01, Kn_jet "
                        "1e-3, Shakhov Pr 2/3, 161x161 Newton-Cotes on [-7,7]^2, fp%d; %d base-grid steps, then %d "
                        "timed steps; MLVS C_split 0.01 C_merge 0.005 eps 2e-5 tau 0.05" % (precision, warmup, steps),
            "value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "levels": len(npts),
            "level_points": [int(x) for x in npts], "level_cells": [int(x) for x in ncells],
            "nbar": float(np.sum(npts * ncells) / np.sum(ncells)), "n_cross": int(ncross),
            "roofline": roofline(prof, precision),
            "uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                    "roofline": roofline(prof_u, precision, var_u,
                                         "jet512x256-nc161-fp32-uvs" if precision == 32 else None),
                    "device_bytes": int(mem_u), "time_to_solution_ratio": t_u / t_m, "memory_ratio": mem_u / mem_m,
                    "mlvs_vs_uvs_rel_l2": err}}


TC_ADAPT = dict(C_split=0.01, C_merge=0.005, eps_merge=2e-5, tau_clust=0.05, flux_test=True, interval=5)


def two_cavity_case(steps=200, warmup=100, precision=32, mode="both", interval=5):
    """Gas expansion between two cavities joined by a channel at full size
    (unstructured: 9216 triangles + 288 quadrilaterals, lattice spacing 1/48;
    101^2 Newton-Cotes base grid on [-7,7]^2; 1000:1 density jump at x = 0;
    FP32 storage), MLVS against UVS.  Both run `warmup` untimed then `steps`
    timed steps from the initial state; the MLVS run adapts at step 0 and every
    `interval` steps (the paper's 5), adaptation included in the timing."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.two_cavity(48, nv=101, vmax=7.0)
    wl = "twocavity48-nc101-fp32-uvs" if precision == 32 else None
    # the update reads each cell's face rows: 3.03 faces per cell on this mesh
    nf = float(np.sum(np.diff(p.cell_ptr))) / p.n_cells
    alg = {"update": 6 + nf, "update_cell": 8 + nf}
    if mode == "uvs":
        u, t_u, upd_u, _ = run_gpu(p, steps, warmup, precision, None)
        prof_u = stage_profile(u, reps=5)
        var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
        u.close()
        return {"uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                        "roofline": roofline(prof_u, precision, var_u, wl, alg, 1)}}
    ap = dict(TC_ADAPT, interval=interval)
    s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=ap, graph=True)
    s.step(warmup)
    autotune.autotune(s, precision)
    torch.cuda.synchronize()
    c0 = s.counters()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    upd = s.counters()["cell_updates"] - c0["cell_updates"]
    npts, ncells, ncross = s.level_info()
    f_m = s.moments()
    mem_m = s.memory()
    prof = stage_profile(s, reps=5)
    s.close()
    del s
    torch.cuda.empty_cache()
    if mode == "mlvs":
        return {"value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "nbar": float(np.sum(npts * ncells) / np.sum(ncells)),
                "roofline": roofline(prof, precision, None, None, alg, 1)}
    u, t_u, upd_u, _ = run_gpu(p, steps, warmup, precision, None)
    f_u = u.moments()
    mem_u = u.memory()
    prof_u = stage_profile(u, reps=5)
    var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
    u.close()
    del u
    torch.cuda.empty_cache()
    vol = cell_areas(p)
    rl2 = lambda a, b: float(np.sqrt(np.sum(vol * (a - b) ** 2) / np.sum(vol * b ** 2)))
    err = {"rho": rl2(f_m[:, 0], f_u[:, 0]), "p": rl2(f_m[:, 0] * f_m[:, 3], f_u[:, 0] * f_u[:, 3]),
           "u": float(np.sqrt(np.sum(vol[:, None] * (f_m[:, 1:3] - f_u[:, 1:3]) ** 2)
                              / np.sum(vol[:, None] * f_u[:, 1:3] ** 2))),
           "T": rl2(f_m[:, 3], f_u[:, 3])}
    return {"workload": "two-cavity expansion, unstructured 9504 cells (9216 triangles + 288 quadrilaterals, "
                        "spacing 1/48), 1000:1 density jump, Kn_left 1e-3, Shakhov Pr 2/3, 101x101 Newton-Cotes "
                        "on [-7,7]^2, fp%d; %d untimed then %d timed steps from the initial state; MLVS C_split "
                        "0.01 C_merge 0.005 eps 2e-5 tau 0.05, adaptation every %d steps" % (
                            precision, warmup, steps, interval),
            "value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "levels": len(npts),
            "level_points": [int(x) for x in npts], "level_cells": [int(x) for x in ncells],
            "nbar": float(np.sum(npts * ncells) / np.sum(ncells)), "n_cross": int(ncross),
            "roofline": roofline(prof, precision, None, None, alg, 1),
            "uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                    "roofline": roofline(prof_u, precision, var_u, wl, alg, 1),
                    "device_bytes": int(mem_u), "time_to_solution_ratio": t_u / t_m, "memory_ratio": mem_u / mem_m,
                    "mlvs_vs_uvs_rel_l2": err}}


def two_cavity_to_time(t_end=4.0, precision=32, interval=5, map_moments=4, tau_clust=0.05, scale=1.0):
    """The two-cavity expansion run to dimensionless time t_end (the paper
    compares MLVS and UVS at t = 4), both forms timed over the whole run from
    the initial state (MLVS adaptation every `interval` steps included), with
    the area-weighted field differences and the level configuration at t_end."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.two_cavity(48, nv=101, vmax=7.0)
    vol = cell_areas(p)
    out = {}
    for mode in ("mlvs", "uvs"):
        s = m.Solver.from_problem(p, precision=precision, compat=4, map_moments=map_moments,
                                  adapt=dict(TC_ADAPT, interval=interval, tau_clust=tau_clust,
                                             C_split=scale * TC_ADAPT["C_split"], C_merge=scale * TC_ADAPT["C_merge"],
                                             eps_merge=scale * TC_ADAPT["eps_merge"]) if mode == "mlvs" else None,
                                  graph=True)
        n = int(round(t_end / s.dt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(10)
        autotune.autotune(s, precision)
        done = 10
        while done < n:
            k = min(1000, n - done)
            s.step(k)
            done += k
            torch.cuda.synchronize()
            print("two-cavity %s step %d of %d, %.1f s" % (mode, done, n, time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
        t = time.perf_counter() - t0
        npts, ncells, _ = s.level_info()
        out[mode] = {"seconds": t, "steps": n, "fields": s.moments(), "memory": s.memory(),
                     "levels": [int(x) for x in npts], "cells": [int(x) for x in ncells],
                     "nbar": float(np.sum(npts * ncells) / np.sum(ncells))}
        s.close()
        del s
        torch.cuda.empty_cache()
    fm, fu = out["mlvs"]["fields"], out["uvs"]["fields"]
    rl2 = lambda a, b: float(np.sqrt(np.sum(vol[:, None] * (a - b) ** 2) / np.sum(vol[:, None] * b ** 2)))
    err = {"rho": rl2(fm[:, :1], fu[:, :1]), "p": rl2((fm[:, 0] * fm[:, 3])[:, None], (fu[:, 0] * fu[:, 3])[:, None]),
           "u": rl2(fm[:, 1:3], fu[:, 1:3]), "T": rl2(fm[:, 3:4], fu[:, 3:4]), "q": rl2(fm[:, 4:6], fu[:, 4:6])}
    return {"workload": "two-cavity expansion to t = %g (%d steps), 9504 unstructured cells, 101^2, fp%d, MLVS "
                        "adaptation every %d steps, %d-moment mapping, tau_clust %g, criterion thresholds x %g; whole "
                        "runs timed" % (t_end, out["uvs"]["steps"], precision, interval, map_moments, tau_clust, scale),
            "mlvs_seconds": out["mlvs"]["seconds"], "uvs_seconds": out["uvs"]["seconds"],
            "speedup": out["uvs"]["seconds"] / out["mlvs"]["seconds"],
            "memory_ratio": out["uvs"]["memory"] / out["mlvs"]["memory"],
            "levels": out["mlvs"]["levels"], "level_cells": out["mlvs"]["cells"], "nbar": out["mlvs"]["nbar"],
            "mlvs_vs_uvs_rel_l2": err}


def long_run(kind="cylinder", steps=10000, warmup=100, precision=32, map_moments=4):
    """A whole run of the cylinder (10,000 steps, about one flow-through) or the
    jet (2,000 steps) from the freestream or background state, MLVS against
    UVS, each timed over the whole run: `warmup` base-grid steps, then the
    MLVS run adapts at the start of every block of 100 steps (adaptation
    included).  Field differences at the end."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = (W.cylinder(256, 128, Kn=0.1, nv=101, vmax=10.0) if kind == "cylinder"
         else W.jet(512, 256, Kn_jet=1e-3, nv=161, vmax=7.0))
    out = {}
    for mode in ("mlvs", "uvs"):
        s = m.Solver.from_problem(p, precision=precision, compat=4, map_moments=map_moments,
                                  adapt=CYL_ADAPT if mode == "mlvs" else None, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(10)
        autotune.autotune(s, precision)
        s.step(warmup - 10)
        done = warmup
        while done < steps:
            if mode == "mlvs":
                s.adapt()
            k = min(CYL_INTERVAL, steps - done)
            s.step(k)
            done += k
            if done % 500 == 0 or done == steps:
                torch.cuda.synchronize()
                print("%s %s step %d of %d, %.1f s" % (kind, mode, done, steps, time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        npts, ncells, ncross = s.level_info()
        out[mode] = {"seconds": t, "fields": s.moments(), "memory": s.memory(), "levels": [int(x) for x in npts],
                     "nbar": float(np.sum(npts * ncells) / np.sum(ncells)), "n_cross": int(ncross)}
        s.close()
        del s
        torch.cuda.empty_cache()
    fm, fu = out["mlvs"]["fields"], out["uvs"]["fields"]
    rl2 = lambda a, b: float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))
    err = {"rho": rl2(fm[:, 0], fu[:, 0]), "u": rl2(fm[:, 1:3], fu[:, 1:3]), "T": rl2(fm[:, 3], fu[:, 3]),
           "q": rl2(fm[:, 4:6], fu[:, 4:6])}
    return {"workload": "%s, %d steps (%d on the base grid first), fp%d, MLVS adaptation every %d steps, %d-moment "
                        "mapping; whole runs timed" % (kind, steps, warmup, precision, CYL_INTERVAL, map_moments),
            "mlvs_seconds": out["mlvs"]["seconds"], "uvs_seconds": out["uvs"]["seconds"],
            "speedup": out["uvs"]["seconds"] / out["mlvs"]["seconds"],
            "memory_ratio": out["uvs"]["memory"] / out["mlvs"]["memory"], "levels": out["mlvs"]["levels"],
            "nbar": out["mlvs"]["nbar"], "n_cross": out["mlvs"]["n_cross"], "mlvs_vs_uvs_rel_l2": err}


def tau_sweep(steps=2000, warmup=100, taus=(1.0, 0.07, 0.05, 0.04, 0.035), precision=32):
    """Clustering-threshold sweep on the full cylinder (the paper's threshold
    study): for each tau_clust an MLVS run of `steps` steps (`warmup` on the
    base grid, then adaptation every 100 steps), timed whole, against one UVS
    run of the same steps; levels, cross faces and field differences at the
    end, and the cheapest setting within 1e-3 on rho and T."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.cylinder(256, 128, Kn=0.1, nv=101, vmax=10.0)

    def run(adapt):
        s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=adapt, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(10)
        autotune.autotune(s, precision)
        s.step(warmup - 10)
        done = warmup
        while done < steps:
            if adapt is not None:
                s.adapt()
            k = min(CYL_INTERVAL, steps - done)
            s.step(k)
            done += k
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        npts, ncells, ncross = s.level_info()
        r = {"seconds": t, "fields": s.moments(), "levels": len(npts),
             "nbar": float(np.sum(npts * ncells) / np.sum(ncells)), "n_cross": int(ncross)}
        s.close()
        del s
        torch.cuda.empty_cache()
        return r

    ref = run(None)
    print("tau sweep: UVS %.1f s" % ref["seconds"], file=sys.stderr, flush=True)
    fu = ref["fields"]
    rl2 = lambda a, b: float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))
    rows = []
    for tau in taus:
        r = run(dict(CYL_ADAPT, tau_clust=tau))
        fm = r.pop("fields")
        r.update(tau_clust=tau, speedup=ref["seconds"] / r["seconds"],
                 rel_l2={"rho": rl2(fm[:, 0], fu[:, 0]), "u": rl2(fm[:, 1:3], fu[:, 1:3]), "T": rl2(fm[:, 3], fu[:, 3]),
                         "q": rl2(fm[:, 4:6], fu[:, 4:6])})
        print("tau %g: %.1f s, %d levels" % (tau, r["seconds"], r["levels"]), file=sys.stderr, flush=True)
        rows.append(r)
    ok = [r for r in rows if r["rel_l2"]["rho"] <= 1e-3 and r["rel_l2"]["T"] <= 1e-3]
    best = min(ok, key=lambda r: r["seconds"])["tau_clust"] if ok else None
    return {"workload": "cylinder 256x128, 101^2, fp%d, %d steps (%d on the base grid), adaptation every %d steps"
                        % (precision, steps, warmup, CYL_INTERVAL),
            "uvs_seconds": ref["seconds"], "runs": rows, "cheapest_within_1e-3_rho_T": best}


def cell_areas(p):
    """Shoelace areas of an unstructured problem's cells (weights of the field differences)."""
    out = np.zeros(p.n_cells)
    for c in range(p.n_cells):
        v = p.nodes[p.cell_node[p.cell_ptr[c]:p.cell_ptr[c + 1]]]
        x, y = v[:, 0], v[:, 1]
        out[c] = 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(np.roll(x, -1), y))
    return out


# launch variant index -> (velocity points per lane per load batch, minimum waves per SIMD)
VARIANTS = {0: (1, 4), 1: (2, 4), 2: (4, 2), 3: (4, 4), 4: (1, 2)}
# kernels instantiated per compatibility order carry it as a template argument,
# and the face kernels the mesh kind (0 structured, 1 unstructured) after it
STAGE_CM = ("cell", "face_target", "face", "update_cell")
STAGE_MK = ("face_rec", "face", "xface")
STAGE_KERNEL = {"face": "k_face_full", "update_cell": "k_update_cell",
                "cell": "k_cell_prep", "face_rec": "k_face_rec", "face_target": "k_face_target",
                "update": "k_update", "xface": "k_xface"}


def measured_traffic(workload, stage, precision, variant, mk=0):
    """HBM-side bytes per dispatch of the stage's kernel from profiles/traffic.txt
    (FETCH_SIZE and WRITE_SIZE runs, copy-calibrated), or None when absent or
    when the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    src = os.path.join(ROOT, "paper_2609_35258_amd", "csrc", "kernels.hip")
    if stage not in STAGE_KERNEL or variant is None or not os.path.exists(path):
        return None
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    u, w = VARIANTS[variant]
    if mk and stage in STAGE_MK:
        u, w = VARIANTS[0]                 # unstructured face kernels: the (1, 4) pair for every variant
    name = "mlvs::%s<%s,%d,%d%s%s>" % (STAGE_KERNEL[stage], "double" if precision == 64 else "float", u, w,
                                       ",4" if stage in STAGE_CM else "", ",%d" % mk if stage in STAGE_MK else "")
    for line in open(path):
        f = line.split()
        if len(f) == 4 and not line.startswith("#") and f[0] == h and f[1] == workload and f[2] == name:
            return float(f[3])
    return None


def roofline(prof, precision, variants=None, workload=None, alg=None, mk=0):
    """Roofline entry for the dominant stage: algorithmic bytes / mean launch time.
    alg: per-stage overrides of ALG_VALUES; mk: mesh kind (1 unstructured)."""
    av = dict(ALG_VALUES, **(alg or {}))
    evsz = 8 if precision == 64 else 4
    # cross-level faces run on a second stream beside the face stages, off the
    # step's critical path: they are not the dominant kernel even when their
    # lone launch is long
    dom = max((k for k in prof if av[k] > 0 and (k != "xface" or len(prof) == 1)), key=lambda k: prof[k]["ms"])
    d = prof[dom]
    achieved = d["points"] * av[dom] * evsz / (d["ms"] * 1e-3) / 1e9
    t = measured_traffic(workload, dom, precision, (variants or {}).get(dom), mk) if workload else None
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": t,
            "algorithmic_bytes": d["points"] * av[dom] * evsz,
            "stage_ms": {k: round(v["ms"], 5) for k, v in prof.items()}}


def cylinder_case(steps=200, warmup=100, precision=32, mode="both"):
    """Supersonic cylinder at full size (256 x 128 O-grid, Ma 3, Kn 0.1, 101^2
    Newton-Cotes base grid, FP32 storage), MLVS against UVS.  Both start from
    the freestream and take `warmup` untimed steps on the base grid (an
    impulsive Ma 3 start is not resolved by levels built from the uniform
    freestream); then the MLVS run adapts (criterion levels) at the start of
    every block of 100 steps, adaptation time included in the timed steps."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.cylinder(256, 128, Kn=0.1, nv=101, vmax=10.0)
    uvs_wl = "cylinder256x128-nc101-fp32-uvs" if precision == 32 else None
    if mode == "uvs":
        u, t_u, upd_u, _ = run_gpu(p, steps, warmup + 2, precision, None)
        prof_u = stage_profile(u, reps=5)
        var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
        u.close()
        return {"uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                        "roofline": roofline(prof_u, precision, var_u, uvs_wl)}}
    s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=CYL_ADAPT, graph=True)
    s.step(warmup)
    s.adapt()
    s.step(2)
    autotune.autotune(s, precision)
    torch.cuda.synchronize()
    c0 = s.counters()
    t0 = time.perf_counter()
    for _ in range(steps // CYL_INTERVAL):
        s.adapt()
        s.step(CYL_INTERVAL)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    upd = s.counters()["cell_updates"] - c0["cell_updates"]
    npts, ncells, ncross = s.level_info()
    f_m = s.moments()
    mem_m = s.memory()
    prof = stage_profile(s, reps=5)
    s.close()
    if mode == "mlvs":
        return {"value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "nbar": float(np.sum(npts * ncells) / np.sum(ncells)),
                "roofline": roofline(prof, precision)}
    u, t_u, upd_u, _ = run_gpu(p, steps, warmup + 2, precision, None)
    f_u = u.moments()
    mem_u = u.memory()
    prof_u = stage_profile(u, reps=5)
    var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
    u.close()
    err = {name: float(np.sqrt(np.sum((f_m[:, k] - f_u[:, k]) ** 2) / np.sum(f_u[:, k] ** 2)))
           for k, name in ((0, "rho"), (1, "u"), (3, "T"))}
    return {"workload": "cylinder O-grid 256x128, Ma 3, Kn 0.1, Shakhov Pr 2/3, 101x101 Newton-Cotes on "
                        "[-10,10]^2, fp%d; %d base-grid steps from a freestream start, then %d timed steps; MLVS "
                        "C_split 0.01 C_merge 0.005 eps 2e-5 tau 0.05, adaptation every %d steps"
                        % (precision, warmup, steps, CYL_INTERVAL),
            "value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "levels": len(npts),
            "level_points": [int(x) for x in npts], "level_cells": [int(x) for x in ncells],
            "nbar": float(np.sum(npts * ncells) / np.sum(ncells)), "n_cross": int(ncross),
            "roofline": roofline(prof, precision),
            "uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                    "roofline": roofline(prof_u, precision, var_u, uvs_wl),
                    "time_to_solution_ratio": t_u / t_m, "memory_ratio": mem_u / mem_m,
                    "mlvs_vs_uvs_rel_l2": err}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nv", type=int, default=28)
    ap.add_argument("--precision", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-uvs", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-cylinder", action="store_true")
    ap.add_argument("--no-jet", action="store_true")
    ap.add_argument("--tau-sweep", action="store_true", help="only the clustering-threshold sweep on the cylinder")
    ap.add_argument("--long-map", type=int, default=4, choices=[4, 9], help="mapping order of the --long runs")
    ap.add_argument("--long", choices=("cylinder", "jet"), default=None,
                    help="only a whole run of that case, MLVS against UVS (10,000 cylinder or 2,000 jet steps)")
    ap.add_argument("--no-two-cavity", action="store_true")
    ap.add_argument("--two-cavity-only", action="store_true", help="only the two-cavity comparison")
    ap.add_argument("--tc-mode", default="both", choices=["both", "uvs", "mlvs"])
    ap.add_argument("--tc-interval", type=int, default=5)
    ap.add_argument("--tc-map", type=int, default=4, choices=[4, 9])
    ap.add_argument("--tc-tau", type=float, default=0.05)
    ap.add_argument("--tc-scale", type=float, default=1.0, help="factor on C_split, C_merge and eps_merge")
    ap.add_argument("--tc-t-end", type=float, default=0.0,
                    help="with --two-cavity-only: run both forms to this time instead (the paper's t = 4)")
    ap.add_argument("--jet-only", action="store_true", help="only the full-size jet comparison (profiling runs)")
    ap.add_argument("--jet-mode", choices=("both", "mlvs", "uvs"), default="both")
    ap.add_argument("--cylinder-only", action="store_true",
                    help="only the full-size cylinder comparison (profiling runs)")
    ap.add_argument("--cylinder-steps", type=int, default=200)
    ap.add_argument("--cylinder-mode", choices=("both", "mlvs", "uvs"), default="both")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}))
        return
    if args.jet_only:
        print(json.dumps({"jet": jet_case(mode=args.jet_mode)}), flush=True)
        return
    if args.tau_sweep:
        print(json.dumps({"tau_sweep": tau_sweep()}), flush=True)
        return
    if args.long:
        print(json.dumps({"long_run": long_run(args.long, 10000 if args.long == "cylinder" else 2000,
                                               map_moments=args.long_map)}), flush=True)
        return
    if args.two_cavity_only:
        if args.tc_t_end > 0:
            print(json.dumps({"two_cavity_to_time": two_cavity_to_time(args.tc_t_end, interval=args.tc_interval,
                                                                       map_moments=args.tc_map,
                                                                       tau_clust=args.tc_tau,
                                                                       scale=args.tc_scale)}), flush=True)
            return
        print(json.dumps({"two_cavity": two_cavity_case(mode=args.tc_mode, interval=args.tc_interval)}), flush=True)
        return
    if args.cylinder_only:
        print(json.dumps({"cylinder": cylinder_case(steps=args.cylinder_steps, mode=args.cylinder_mode)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    p = workload(args)
    s, t_mlvs, upd, ipts = run_gpu(p, args.steps, args.warmup, args.precision, ADAPT, not args.no_graph,
                                   not args.no_tune)
    value = upd / t_mlvs
    npts, ncells, ncross = s.level_info()
    nbar = float(np.sum(npts * ncells) / np.sum(ncells))
    fields_m = s.moments()
    mem_m = s.memory()
    prof = stage_profile(s)
    variants = {k: v["variant"] for k, v in getattr(s, "tuned", {}).items()}
    roof = roofline(prof, args.precision, variants,
                    "cavity64-gh28-fp64-mlvs" if (args.n, args.nv, args.precision) == (64, 28, 64) else None)
    out = {"metric": "DUGKS cell-velocity updates/s (MLVS-DUGKS hot path, adaptation included)",
           "value": value, "unit": "cell-velocity updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_mlvs / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == 64 else "f32",
           "data": "synthetic",
           "config": {"workload": "lid-driven cavity %dx%d, Kn 0.075, lid Ma 0.16, Shakhov Pr 2/3, %dx%d "
                                  "Gauss-Hermite base grid, MLVS (criterion levels, interval 100)"
                                  % (args.n, args.n, args.nv, args.nv),
                      "n_cells": p.n_cells, "base_points": args.nv * args.nv, "levels": len(npts),
                      "level_points": [int(x) for x in npts], "level_cells": [int(x) for x in ncells],
                      "nbar": nbar, "n_cross": int(ncross), "iface_points_per_s": ipts / t_mlvs,
                      "graph": not args.no_graph,
                      "variants": {k: v["variant"] for k, v in getattr(s, "tuned", {}).items()}},
           "roofline": roof}
    s.close()
    if not args.no_uvs:
        u, t_uvs, upd_u, _ = run_gpu(p, args.steps, args.warmup, args.precision, None, not args.no_graph,
                                     not args.no_tune)
        fields_u = u.moments()
        mem_u = u.memory()
        vol = np.ones(p.n_cells)
        err = {}
        for k, name in ((0, "rho"), (1, "u"), (3, "T")):
            a, b = fields_m[:, k], fields_u[:, k]
            err[name] = float(np.sqrt(np.sum(vol * (a - b) ** 2) / np.sum(vol * b ** 2)))
        out["uvs"] = {"value": upd_u / t_uvs, "ms_per_step": 1e3 * t_uvs / args.steps,
                      "time_to_solution_ratio": t_uvs / t_mlvs, "memory_ratio": mem_u / mem_m,
                      "mlvs_vs_uvs_rel_l2": err}
        u.close()
    if not args.no_cylinder:
        out["cylinder"] = cylinder_case(steps=args.cylinder_steps)
    if not args.no_jet:
        out["jet"] = jet_case()
    if not args.no_two_cavity:
        out["two_cavity"] = two_cavity_case()
    if not args.no_learned:
        out["learned"] = learned_vs_criterion()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
