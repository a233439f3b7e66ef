"""Benchmark: MLVS-DUGKS cell-velocity updates/s on one MI355X, MLVS vs UVS.

Headline workload (synthetic, deterministic): the under-expanded slot jet
into near vacuum, 512 x 256 uniform cells on [0,32] x [-8,8], sonic slot
|y| <= 0.5 at x = 0, background density 0.01 (pressure ratio 100), Kn_jet
1e-3, Shakhov Pr 2/3, 161 x 161 Newton-Cotes base grid on [-7,7]^2 (25921
points), FP32 storage.  MLVS: criterion C_split 0.01, C_merge 0.005,
transport-error test 2e-5, tau_clust 0.05, adaptation every 5 steps.  The
solver first takes 100 untimed steps on the base grid from the initial state
(levels built from a uniform background would not resolve the jet), then
--warmup untimed and --steps timed MLVS steps, adaptation (criterion,
grouping, remap) inside the timed window.  UVS: the same steps on the fixed
base grid.  A step is one pass of the whole hot path.  Prints one JSON line.
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


def run_gpu(p, steps, warmup, precision, adapt, graph=True, tune=True):
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=adapt, graph=graph)
    s.step(warmup)
    if tune:
        s.tiles = autotune.autotune_tiles(s, precision)
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


LEARNED_ADAPT = dict(C_split=0.01, C_merge=0.005, eps_merge=2e-5, tau_clust=0.05, flux_test=True, interval=0)


def learned_vs_criterion(precision=32, n_theta=256, n_r=128, nv=101, warm=100, snaps=32, every=10, rounds=6):
    """Learned vs criterion adaptation on the same GPU.

    Supersonic cylinder (Ma 3, Kn 0.1, Shakhov), n_theta x n_r cells and an
    nv^2 Newton-Cotes base grid (by default the full-size case: 32 snapshots of
    32768 cells, about 1e6 samples).  A criterion run builds the catalogue (one
    full adaptation after `warm` base-grid steps) and records (features,
    criterion label) snapshots every `every` steps in the context; the context
    trains its network on the GPU on the earlier 80% of the snapshots.  A second solver starts from the same
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
    for k in range(snaps):
        crit.step(every)
        n_samples = crit.selector_snapshot(reset=(k == 0))
    trep = crit.selector_train(epochs=30, batch=1024, lr=3e-3, val_frac=0.2, seed=0)
    params, _ = crit.selector_params()
    lrn = m.Solver.from_problem(p, precision=precision, compat=4, adapt=LEARNED_ADAPT)
    lrn.set_levels(np.stack([crit.level_kappa(k) for k in range(K)]), crit.cell_levels())
    st = crit.get_state()
    lrn.set_state([g for g, _ in st], [h for _, h in st])
    lrn.selector_set(params, K)
    n = p.n_cells
    out = {"workload": "cylinder %dx%d, Ma 3, Kn 0.1, %dx%d Newton-Cotes on [-10,10]^2, fp%d, C_split 0.01, "
                       "C_merge 0.005, eps_merge 2e-5, tau_clust 0.05" % (n_theta, n_r, nv, nv, precision),
           "K": K, "samples": int(trep["n_train"] + trep["n_val"]), "snapshot_rows": int(n_samples),
           "train": {k: trep[k] for k in ("loss_first", "loss_last", "train_acc", "val_acc", "ms")}}
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
# thresholds 0.03 times the above: the cylinder's MLVS fields then stay within
# the 1e-3 rel-L2 gate of UVS on rho and T (the near-vacuum wake decides T)
CYL_ADAPT_GATE = dict(CYL_ADAPT, C_split=3e-4, C_merge=1.5e-4, eps_merge=6e-7)


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
    if mode == "uvs":
        u, t_u, upd_u, _ = run_gpu(p, steps, warmup, precision, None)
        prof_u = stage_profile(u, reps=5)
        var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
        u.close()
        return {"uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                        "roofline": method_roofline(prof_u, precision, upd_u / steps, 1e3 * t_u / steps)}}
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
                "roofline": method_roofline(prof, precision, upd / steps, 1e3 * t_m / steps)}
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
            "roofline": method_roofline(prof, precision, upd / steps, 1e3 * t_m / steps),
            "uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                    "roofline": method_roofline(prof_u, precision, upd_u / steps, 1e3 * t_u / steps),
                    "device_bytes": int(mem_u), "time_to_solution_ratio": t_u / t_m, "memory_ratio": mem_u / mem_m,
                    "mlvs_vs_uvs_rel_l2": err, "meets_1e-3_gate_rho_T": _gate(err)}}


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
            "mlvs_vs_uvs_rel_l2": err, "meets_1e-3_gate_rho_T": _gate(err)}


def long_run(kind="cylinder", steps=10000, warmup=100, precision=32, map_moments=4, scale=1.0):
    """A whole run of the cylinder (10,000 steps, about one flow-through) or the
    jet (2,000 steps) from the freestream or background state, MLVS against
    UVS, each timed over the whole run: `warmup` base-grid steps, then the
    MLVS run adapts at the start of every block of 100 steps (adaptation
    included).  Field differences at the end.  `scale` multiplies C_split,
    C_merge and eps_merge."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = (W.cylinder(256, 128, Kn=0.1, nv=101, vmax=10.0) if kind == "cylinder"
         else W.jet(512, 256, Kn_jet=1e-3, nv=161, vmax=7.0))
    ap = dict(CYL_ADAPT, C_split=CYL_ADAPT["C_split"] * scale, C_merge=CYL_ADAPT["C_merge"] * scale,
              eps_merge=CYL_ADAPT["eps_merge"] * scale)
    out = {}
    for mode in ("mlvs", "uvs"):
        s = m.Solver.from_problem(p, precision=precision, compat=4, map_moments=map_moments,
                                  adapt=ap if mode == "mlvs" else None, graph=True)
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
                        "mapping, C_split %g C_merge %g eps_merge %g; whole runs timed"
                        % (kind, steps, warmup, precision, CYL_INTERVAL, map_moments, ap["C_split"], ap["C_merge"],
                           ap["eps_merge"]),
            "mlvs_seconds": out["mlvs"]["seconds"], "uvs_seconds": out["uvs"]["seconds"],
            "speedup": out["uvs"]["seconds"] / out["mlvs"]["seconds"],
            "memory_ratio": out["uvs"]["memory"] / out["mlvs"]["memory"], "levels": out["mlvs"]["levels"],
            "nbar": out["mlvs"]["nbar"], "n_cross": out["mlvs"]["n_cross"], "mlvs_vs_uvs_rel_l2": err,
            "meets_1e-3_gate_rho_T": _gate(err)}


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


def measured_traffic(workload, stage, precision, variant, mk=0, crit=False):
    """HBM-side bytes per dispatch of the stage's kernel from profiles/traffic.txt
    (FETCH_SIZE and WRITE_SIZE runs, copy-calibrated), or None when absent or
    when the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    src = os.path.join(ROOT, "paper_2609_35258_amd", "csrc", "kernels.hip")
    if not os.path.exists(path) or (not crit and (stage not in STAGE_KERNEL or variant is None)):
        return None
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if crit:
        name = "mlvs::k_criterion<%s>" % ("double" if precision == 64 else "float")
    else:
        u, w = VARIANTS[variant]
        if mk and stage in STAGE_MK:
            u, w = VARIANTS[0]             # unstructured face kernels: the (1, 4) pair for every variant
        name = "mlvs::%s<%s,%d,%d%s%s>" % (STAGE_KERNEL[stage], "double" if precision == 64 else "float", u, w,
                                           ",4" if stage in STAGE_CM else "", ",%d" % mk if stage in STAGE_MK else "")
    for line in open(path):
        f = line.split()
        if len(f) == 4 and not line.startswith("#") and f[0] == h and f[1] == workload and f[2] == name:
            return float(f[3])
    return None


def cylinder_case(steps=200, warmup=100, precision=32, mode="both", Kn=0.1, adapt=None):
    """Supersonic cylinder at full size (256 x 128 O-grid, Ma 3, Kn 0.1 or 1, 101^2
    Newton-Cotes base grid, FP32 storage), MLVS against UVS.  Both start from
    the freestream and take `warmup` untimed steps on the base grid (an
    impulsive Ma 3 start is not resolved by levels built from the uniform
    freestream); then the MLVS run adapts (criterion levels) at the start of
    every block of 100 steps, adaptation time included in the timed steps."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.cylinder(256, 128, Kn=Kn, nv=101, vmax=10.0)
    uvs_wl = "cylinder256x128-nc101-fp32-uvs" if precision == 32 and Kn == 0.1 else None
    if mode == "uvs":
        u, t_u, upd_u, _ = run_gpu(p, steps, warmup + 2, precision, None)
        prof_u = stage_profile(u, reps=5)
        var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
        u.close()
        return {"uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                        "roofline": method_roofline(prof_u, precision, upd_u / steps, 1e3 * t_u / steps, uvs_wl,
                                                    var_u)}}
    ap = CYL_ADAPT if adapt is None else adapt
    s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=ap, graph=True)
    s.step(warmup)
    s.adapt()
    s.step(2)
    autotune.autotune_tiles(s, precision)
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
                "roofline": method_roofline(prof, precision, upd / steps, 1e3 * t_m / steps)}
    u, t_u, upd_u, _ = run_gpu(p, steps, warmup + 2, precision, None)
    f_u = u.moments()
    mem_u = u.memory()
    prof_u = stage_profile(u, reps=5)
    var_u = {k: v["variant"] for k, v in getattr(u, "tuned", {}).items()}
    u.close()
    err = {name: float(np.sqrt(np.sum((f_m[:, k] - f_u[:, k]) ** 2) / np.sum(f_u[:, k] ** 2)))
           for k, name in ((0, "rho"), (1, "u"), (3, "T"))}
    return {"workload": "cylinder O-grid 256x128, Ma 3, Kn %g, Shakhov Pr 2/3, 101x101 Newton-Cotes on "
                        "[-10,10]^2, fp%d; %d base-grid steps from a freestream start, then %d timed steps; MLVS "
                        "C_split %g C_merge %g eps %g tau %g, adaptation every %d steps"
                        % (Kn, precision, warmup, steps, ap["C_split"], ap["C_merge"], ap["eps_merge"],
                           ap["tau_clust"], CYL_INTERVAL),
            "value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "levels": len(npts),
            "level_points": [int(x) for x in npts], "level_cells": [int(x) for x in ncells],
            "nbar": float(np.sum(npts * ncells) / np.sum(ncells)), "n_cross": int(ncross),
            "roofline": method_roofline(prof, precision, upd / steps, 1e3 * t_m / steps),
            "uvs": {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps,
                    "roofline": method_roofline(prof_u, precision, upd_u / steps, 1e3 * t_u / steps, uvs_wl, var_u),
                    "time_to_solution_ratio": t_u / t_m, "memory_ratio": mem_u / mem_m,
                    "mlvs_vs_uvs_rel_l2": err, "meets_1e-3_gate_rho_T": _gate(err)}}


def persistent_ab(steps=100, interval=5, precision=32, pure_steps=20):
    """The staged (or fused) step against the persistent single-launch step on
    the full-size cylinder (Ma 3, after 100 base-grid steps) and two-cavity
    (from the initial state) MLVS runs.  Per mode: ms per step with adaptation
    every `interval` steps inside the timed window, the graph captures and
    graph launches those steps took, and ms per step without adaptation; the
    relative L2 difference of the final fields between the two modes."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    cases = {"cylinder256x128-nc101": (lambda: W.cylinder(256, 128, Kn=0.1, nv=101, vmax=10.0), CYL_ADAPT, 100),
             "two_cavity9504-nc101": (lambda: W.two_cavity(48, nv=101, vmax=7.0), TC_ADAPT, 0)}
    out = {}
    for name, (make, base_ap, warm) in cases.items():
        p = make()
        res, fields = {}, {}
        for mode in ("staged", "persistent"):
            s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=dict(base_ap, interval=0), graph=True)
            s.step(warm)
            s.adapt()
            s.set_persistent(mode == "persistent")
            s.step(2)
            tuned = autotune.autotune(s, precision)
            s.set_adapt(dict(base_ap, interval=interval))
            torch.cuda.synchronize()
            g0, c0 = s.graph_info(), s.counters()
            t0 = time.perf_counter()
            s.step(steps)
            torch.cuda.synchronize()
            t_ad = time.perf_counter() - t0
            g1, c1 = s.graph_info(), s.counters()
            s.set_adapt(dict(base_ap, interval=0))
            s.step(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(pure_steps)
            torch.cuda.synchronize()
            t_pure = time.perf_counter() - t0
            npts, ncells, _ = s.level_info()
            res[mode] = {"ms_per_step_with_adaptation": 1e3 * t_ad / steps,
                         "ms_per_step_no_adaptation": 1e3 * t_pure / pure_steps,
                         "adaptations": c1["adaptations"] - c0["adaptations"],
                         "graph_captures": g1["captures"] - g0["captures"],
                         "graph_launches": g1["launches"] - g0["launches"],
                         "stages": s.step_stages(), "grid": g1["grid"], "barrier_error": g1["error"],
                         "variants": {k: v["variant"] for k, v in tuned.items()},
                         "levels": len(npts), "nbar": float(np.sum(npts * ncells) / np.sum(ncells))}
            fields[mode] = s.moments()
            print("persistent_ab %s %s: %s" % (name, mode, json.dumps(res[mode])), file=sys.stderr, flush=True)
            s.close()
            del s
            torch.cuda.empty_cache()
        a, b = fields["staged"], fields["persistent"]
        res["fields_rel_l2"] = {nm: float(np.sqrt(np.sum((b[:, k] - a[:, k]) ** 2) / np.sum(a[:, k] ** 2)))
                                for k, nm in ((0, "rho"), (1, "u"), (3, "T"))}
        out[name] = res
    return {"workload": "fp%d; %d timed steps with adaptation every %d steps, then %d steps without" % (
        precision, steps, interval, pure_steps), "cases": out}


JET_ADAPT = dict(C_split=0.01, C_merge=0.005, eps_merge=2e-5, tau_clust=0.05, flux_test=True, interval=5)
JET_BASE_STEPS = 100
JET_WL = "jet512x256-nc161-fp32"
# the method's own bytes per cell-velocity update: read and write g~, h~ once
# (4 values), and the design floor with the second read the two velocity
# reductions force (6 values)
METHOD_VALUES, FLOOR_VALUES = 4, 6


def method_roofline(prof, precision, updates_per_step, step_ms, workload=None, variants=None, interval=0,
                    crit_cells=0, crit_blocks=0):
    """Roofline of the timed window's dominant kernel (the largest share of a
    step: the criterion counts 1/interval of its launch time).  Algorithmic
    bytes per launch, by the method's own figures: a step kernel is credited
    with the step's 16 B per FP32 (32 B per FP64) cell-velocity update (read
    and write g~, h~ once), the criterion with reading the state once (8 B per
    FP32, 16 B per FP64 point) and writing one kappa byte per cell and 2x2
    block.  achieved = those bytes over the kernel's mean launch time; the
    whole step against the same 16 B and the 24 B floor beside it.  traffic:
    the copy-calibrated FETCH_SIZE and WRITE_SIZE bytes per launch of that
    kernel from profiles/traffic.txt (null when the kernels changed since)."""
    evsz = 8 if precision == 64 else 4
    per_step = {}
    for k, v in prof.items():
        if k == "criterion" and not interval:
            continue
        if k == "xface" and len(prof) > 1:
            continue                        # second stream, beside the face stages
        per_step[k] = v["ms"] * ((1.0 / interval) if k == "criterion" else 1.0)

    def alg_of(k):
        if k == "criterion":
            return 2 * evsz * updates_per_step + crit_blocks * crit_cells
        return METHOD_VALUES * evsz * updates_per_step

    def basis_of(k):
        if k == "criterion":
            return ("%d B per cell-velocity point (read g~, h~ once) x %.4g points + one kappa byte per cell and 2x2 "
                    "block (%d x %d), over the mean launch time of criterion" % (2 * evsz, updates_per_step,
                                                                                crit_cells, crit_blocks))
        return ("%d B per cell-velocity update (read and write g~, h~ once) x %.4g updates per step, over the mean "
                "launch time of %s" % (METHOD_VALUES * evsz, updates_per_step, k))

    dom = max(per_step, key=per_step.get)
    alg = alg_of(dom)
    achieved = alg / (prof[dom]["ms"] * 1e-3) / 1e9
    var = (variants or {}).get(dom)
    t = measured_traffic(workload, dom, precision, var, crit=(dom == "criterion")) if workload else None
    step_alg = METHOD_VALUES * evsz * updates_per_step
    # every stage's launch time and share of a step; achieved and frac only
    # where the method gives the kernel a figure of its own (the step's
    # longest streaming kernel carries the step's bytes, the criterion its read)
    kernels = {}
    for k in per_step:
        kernels[k] = {"ms": round(prof[k]["ms"], 5), "ms_per_step": round(per_step[k], 5)}
        if k in (dom, "criterion"):
            a = alg_of(k)
            kernels[k].update({"algorithmic_bytes": a, "achieved_GBs": round(a / (prof[k]["ms"] * 1e-3) / 1e9, 1),
                               "frac": round(a / (prof[k]["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": t, "algorithmic_bytes": alg, "basis": basis_of(dom),
            "step": {"ms": step_ms, "achieved": step_alg / (step_ms * 1e-3) / 1e9,
                     "frac": step_alg / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "floor_frac": FLOOR_VALUES * evsz * updates_per_step / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "kernels": kernels}


def _gate(err):
    """The metric's accuracy gate: MLVS against UVS within 1e-3 relative L2 on rho and T."""
    return bool(err["rho"] <= 1e-3 and err["T"] <= 1e-3)


def _fields_error(fa, fb, vol=None):
    """Relative L2 (volume-weighted) of rho, u (vector), T, p and q (vector) of fa against fb."""
    vol = np.ones(len(fa)) if vol is None else vol
    rl2 = lambda a, b: float(np.sqrt(np.sum(vol[:, None] * (a - b) ** 2) / np.sum(vol[:, None] * b ** 2)))
    pa, pb = (fa[:, 0] * fa[:, 3])[:, None], (fb[:, 0] * fb[:, 3])[:, None]
    return {"rho": rl2(fa[:, :1], fb[:, :1]), "u": rl2(fa[:, 1:3], fb[:, 1:3]), "T": rl2(fa[:, 3:4], fb[:, 3:4]),
            "p": rl2(pa, pb), "q": rl2(fa[:, 4:6], fb[:, 4:6])}


def jet_headline(steps, warmup, interval=5, precision=32, with_uvs=True, tune=True, with_mlvs=True):
    """The headline: full-size jet, MLVS with adaptation every `interval`
    steps inside the timed window, against UVS over the same steps."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.jet(512, 256, Kn_jet=1e-3, nv=161, vmax=7.0)
    if not with_mlvs:
        return {"uvs": _jet_uvs(p, steps, warmup, precision, tune)[0]}
    s = m.Solver.from_problem(p, precision=precision, compat=4, adapt=dict(JET_ADAPT, interval=0), graph=True)
    s.step(JET_BASE_STEPS)
    s.set_adapt(dict(JET_ADAPT, interval=interval))
    s.step(max(warmup, 1))
    tiles = autotune.autotune_tiles(s, precision) if tune else {}
    tuned = autotune.autotune(s, precision) if tune else {}
    torch.cuda.synchronize()
    c0 = s.counters()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    c1 = s.counters()
    upd = c1["cell_updates"] - c0["cell_updates"]
    n_adapt = c1["adaptations"] - c0["adaptations"]
    print("jet MLVS: %d steps, %d adaptations, %.3f s" % (steps, n_adapt, t_m), file=sys.stderr, flush=True)
    npts, ncells, ncross = s.level_info()
    f_m = s.moments()
    mem_m = s.memory()
    prof = stage_profile(s, reps=3)
    prof["criterion"] = {"ms": s.time_stage("criterion", 2), "items": p.n_cells, "points": upd / max(steps, 1)}
    # adaptation cost (criterion, grouping, level install), timed as whole calls
    t_ad, split = [], []
    for _ in range(3):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = s.adapt()
        torch.cuda.synchronize()
        t_ad.append(1e3 * (time.perf_counter() - ta))
        split.append({k: round(r[k], 3) for k in ("ms_criterion", "ms_dedupe", "ms_cluster", "ms_install")}
                     | {"n_unique": r["n_unique"], "n_changed": r["n_changed"]})
    variants = {k: v["variant"] for k, v in tuned.items()}
    s.close()
    del s
    torch.cuda.empty_cache()
    ups = upd / steps
    out = {"value": upd / t_m, "ms_per_step": 1e3 * t_m / steps, "updates_per_step": ups,
           "adaptations_timed": int(n_adapt), "adapt_ms": t_ad, "adapt_split": split, "levels": len(npts),
           "level_points": [int(x) for x in npts], "level_cells": [int(x) for x in ncells],
           "nbar": float(np.sum(npts * ncells) / np.sum(ncells)), "n_cross": int(ncross), "device_bytes": int(mem_m),
           "variants": variants, "tiles": _tiles_summary(tiles),
           "roofline": method_roofline(prof, precision, ups, 1e3 * t_m / steps,
                                       JET_WL + "-mlvs" if precision == 32 else None, variants, interval,
                                       crit_cells=p.n_cells, crit_blocks=(p.nv // 2) ** 2)}
    if with_uvs:
        out["uvs"], f_u, mem_u, t_u = _jet_uvs(p, steps, warmup, precision, tune)
        err = _fields_error(f_m, f_u)
        out["uvs"].update({"time_to_solution_ratio": t_u / t_m, "memory_ratio": mem_u / mem_m,
                           "mlvs_vs_uvs_rel_l2": err,
                           "meets_1e-3_gate_rho_T": _gate(err)})
    return out


def _tiles_summary(t):
    """The tile tuner's choice and its step time per candidate (ms)."""
    if not t:
        return None
    return {"chosen": t["tiles"], "from_cache": t["from_cache"],
            "step_ms": {"%dx%d" % tuple(c): round(ms, 3) for c, ms in zip(t.get("candidates", []), t["all_ms"])}}


def _jet_uvs(p, steps, warmup, precision, tune):
    """The UVS form of the headline over the same steps: (result, fields, bytes, seconds)."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    u = m.Solver.from_problem(p, precision=precision, compat=4, adapt=None, graph=True)
    u.step(JET_BASE_STEPS + max(warmup, 1))
    tiles_u = autotune.autotune_tiles(u, precision) if tune else {}
    tuned_u = autotune.autotune(u, precision) if tune else {}
    torch.cuda.synchronize()
    c0 = u.counters()
    t0 = time.perf_counter()
    u.step(steps)
    torch.cuda.synchronize()
    t_u = time.perf_counter() - t0
    upd_u = u.counters()["cell_updates"] - c0["cell_updates"]
    f_u = u.moments()
    mem_u = u.memory()
    prof_u = stage_profile(u, reps=3)
    var_u = {k: v["variant"] for k, v in tuned_u.items()}
    u.close()
    del u
    torch.cuda.empty_cache()
    res = {"value": upd_u / t_u, "ms_per_step": 1e3 * t_u / steps, "device_bytes": int(mem_u), "variants": var_u,
           "tiles": _tiles_summary(tiles_u),
           "roofline": method_roofline(prof_u, precision, upd_u / steps, 1e3 * t_u / steps,
                                       JET_WL + "-uvs" if precision == 32 else None, var_u)}
    return res, f_u, mem_u, t_u


CPU_WINDOW = dict(i0=0, j0=122, size=12, levels=6, seed=11, amp=0.2, p8=0.55, p4=0.45, p2=0.6)


def _cpu_window():
    """The CPU baseline's sample, from seeded inputs only: the 12 x 12 cells of
    the jet at its slot (initial state with a seeded perturbation), six seeded
    random coarsening masks on the 80 x 80 blocks of the 161^2 grid (about 4000
    points each, the headline's mean level size), and cells assigned to them
    in seeded 4 x 4-cell blocks, so the window holds cross-level faces."""
    w = CPU_WINDOW
    p = W.jet(512, 256, Kn_jet=1e-3, nv=161, vmax=7.0)
    q = W.perturb(W.patch(p, w["i0"], w["j0"], w["size"], w["size"]), seed=w["seed"], amp=w["amp"])
    nb = p.nv // 2
    kap = [W.random_kappa(nb, nb, w["seed"] + k, p8=w["p8"], p4=w["p4"], p2=w["p2"]) for k in range(w["levels"])]
    rng = np.random.default_rng(w["seed"])
    nblk = w["size"] // 4
    blk = rng.integers(0, w["levels"], size=(nblk, nblk))
    cl = np.repeat(np.repeat(blk, 4, axis=0), 4, axis=1).ravel().astype(np.int32)
    return q, kap, cl


def _oracle_patch_work(args):
    """One CPU worker: an oracle MLVS step of the seeded window plus the
    criterion on `n_crit` of its cells.  Returns (seconds of the step, seconds
    per criterion cell, cell-velocity updates of the step, mean level size)."""
    n_crit, = args
    from oracle import levels as lv_
    from oracle.solver import AdaptParams, Solver as Oracle
    q, kap, cl = _cpu_window()
    o = Oracle(q, compat=4, adapt=AdaptParams(JET_ADAPT["C_split"], JET_ADAPT["C_merge"], JET_ADAPT["eps_merge"],
                                              JET_ADAPT["tau_clust"], True, 0))
    o.set_levels(kap, cl)
    ap = o.adapt_params
    t0 = time.perf_counter()
    for c in range(n_crit):
        lv_.criterion(o.levels[o.cell_level[c]], o.g[c], o.h[c], ap.C_split, ap.C_merge, ap.eps_merge, True)
    t_crit = (time.perf_counter() - t0) / max(n_crit, 1)
    t0 = time.perf_counter()
    o.step_count = 1                     # no adaptation inside the timed step
    o.adapt_params = None
    o.step()
    t_step = time.perf_counter() - t0
    n = float(sum(len(g) for g in o.g))
    return t_step, t_crit, n, n / len(o.g)


def _host_cpu():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(interval=5, n_crit=4, max_workers=16):
    """The oracle as it stands, timed on the host: an MLVS step of a 12 x 12-cell
    window of the jet from seeded inputs (`_cpu_window`) plus the criterion on a
    few of its cells, amortised over the adaptation interval; once on one core
    and once on every core of the process's CPU share (the same task in each of
    min(16, available) worker processes)."""
    import multiprocessing as mp
    host = _host_cpu()
    ctx = mp.get_context("spawn")
    # one thread per worker process (numpy's BLAS would otherwise start its own)
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    os.environ.update({k: "1" for k in saved})
    try:
        with ctx.Pool(1) as pool:
            t1, c1, n1, nbar = pool.map(_oracle_patch_work, [(n_crit,)])[0]
        P = max(1, min(max_workers, host["nproc"] or 1))
        t0 = time.perf_counter()
        with ctx.Pool(P) as pool:
            res = pool.map(_oracle_patch_work, [(n_crit,)] * P)
        wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    w = CPU_WINDOW
    ncell = w["size"] ** 2
    rate1 = n1 / (t1 + c1 * ncell / interval)
    # all cores: every worker did the same step and criterion cells
    tP = max(r[0] for r in res)
    cP = max(r[1] for r in res)
    rateP = P * n1 / (tP + cP * ncell / interval)
    return {"value": rateP, "unit": "cell-velocity updates/s", "cores": P, "kind": "oracle",
            "sample": "oracle MLVS step of the 12x12 cells (%d..%d, %d..%d) of the jet at its slot, from seeded "
                      "inputs: initial state perturbed (seed %d, amplitude %g), %d seeded random levels (mean %.0f "
                      "points) on seeded 4x4-cell blocks; %.4g cell-velocity updates; plus the criterion on %d cells, "
                      "amortised over %d steps; %d worker processes each running that task (one oracle and one BLAS "
                      "thread per process), slowest worker's times" % (
                          w["i0"], w["i0"] + 11, w["j0"], w["j0"] + 11, w["seed"], w["amp"], w["levels"], nbar, n1,
                          n_crit, interval, P),
            "host": host,
            "single_core": {"value": rate1, "cores": 1, "step_s": t1, "criterion_s_per_cell": c1},
            "all_cores": {"value": rateP, "cores": P, "step_s": tP, "criterion_s_per_cell": cP, "wall_s": wall}}


def fp32_vs_fp64(steps=200, warmup=100):
    """FP32 storage against the FP64 path at full size (the cylinder, 256 x 128,
    101^2, Ma 3, Kn 0.1): both from the freestream, `warmup` base-grid steps,
    then the FP64 run adapts once and the FP32 run takes the same catalogue and
    cell levels (so only the precision differs), then `steps` more steps; the
    per-field relative L2 of the FP32 fields against the FP64 ones at the end,
    UVS and MLVS, and the drift of the conserved totals."""
    import torch
    import paper_2609_35258_amd as m
    p = W.cylinder(256, 128, Kn=0.1, nv=101, vmax=10.0)
    out = {}
    for mode in ("uvs", "mlvs"):
        runs = {}
        cat = None
        for prec in (64, 32):
            s = m.Solver.from_problem(p, precision=prec, compat=4, adapt=CYL_ADAPT if mode == "mlvs" else None,
                                      graph=True)
            t0 = s.totals()
            s.step(warmup)
            if mode == "mlvs":
                if cat is None:
                    s.adapt()
                    npts = s.level_info()[0]
                    cat = (np.stack([s.level_kappa(k) for k in range(len(npts))]), s.cell_levels())
                else:
                    s.set_levels(*cat)
            s.step(steps)
            runs[prec] = (s.moments(), s.totals(), t0)
            s.close()
            del s
            torch.cuda.empty_cache()
        f64, f32 = runs[64][0], runs[32][0]
        tot32, t032 = runs[32][1], runs[32][2]
        out[mode] = {"rel_l2": _fields_error(f32, f64),
                     "mass_drift_fp32": float(abs(tot32[0] - t032[0]) / abs(t032[0]))}
    out["workload"] = ("cylinder 256x128, 101^2, Ma 3, Kn 0.1: %d base-grid steps, then %d steps (MLVS: the FP64 "
                       "run's catalogue installed in both)" % (warmup, steps))
    return out


def sod_case(steps=100):
    """Configuration 1: the 1-D Sod tube, 200 cells, 101-point Boole grid, BGK,
    plain UVS-DUGKS in FP64 (no compatibility correction), Kn 1e-3 and 1e-1."""
    import torch
    import paper_2609_35258_amd as m
    out = {}
    for Kn in (1e-3, 1e-1):
        p = W.sod_1d(200, Kn=Kn, nv=101, vmax=10.0)
        s = m.Solver.from_problem(p, precision=64, compat=0, face_compat=False, graph=True)
        s.step(5)
        torch.cuda.synchronize()
        c0 = s.counters()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out["Kn=%g" % Kn] = {"value": (s.counters()["cell_updates"] - c0["cell_updates"]) / t,
                             "ms_per_step": 1e3 * t / steps}
        s.close()
    out["note"] = "2.0e4 cell-velocity points per step: launch-bound"
    return out


def cavity_case(steps=200, warmup=100):
    """Configuration 2: the 64 x 64 lid-driven cavity, 28^2 Gauss-Hermite, FP64,
    MLVS with criterion levels (adaptation every 100 steps) and with a fixed
    three-level catalogue, against UVS.  Its 51 MB state stays in the 256 MB
    Infinity Cache: the step is bound by FP64 VALU issue, not HBM."""
    import torch
    import paper_2609_35258_amd as m
    from paper_2609_35258_amd import autotune
    p = W.cavity(64, Kn=0.075, nv=28)
    out = {"workload": "lid-driven cavity 64x64, Kn 0.075, lid Ma 0.16, Shakhov Pr 2/3, 28x28 Gauss-Hermite, fp64; "
                       "%d untimed then %d timed steps" % (warmup, steps),
           "bound": "cache-resident (51 MB state in the 256 MB Infinity Cache); FP64 VALU issue"}
    runs = {}
    for mode in ("mlvs", "fixed3", "uvs"):
        s = m.Solver.from_problem(p, precision=64, compat=4, adapt=ADAPT if mode == "mlvs" else None, graph=True)
        if mode == "fixed3":
            # three nested levels: 8x8 merges far out, 4x4 and 2x2 closer in
            nb = p.nv // 2
            bx, by = np.meshgrid(np.arange(nb), np.arange(nb))
            r = np.maximum(np.abs(bx - (nb - 1) / 2), np.abs(by - (nb - 1) / 2))
            kap = []
            for rmax in (6, 4, 2):
                k = np.zeros((nb, nb), np.uint8)
                k[r > rmax] = 1
                kap.append(k.ravel())
            cl = W.striped_levels(p.ni, p.nj, 3, 1)
            s.set_levels(np.stack(kap), cl)
        s.step(warmup)
        autotune.autotune(s, 64)
        torch.cuda.synchronize()
        c0 = s.counters()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        npts, ncells, _ = s.level_info()
        runs[mode] = (s.moments(), t)
        out[mode] = {"value": (s.counters()["cell_updates"] - c0["cell_updates"]) / t, "ms_per_step": 1e3 * t / steps,
                     "levels": [int(x) for x in npts], "nbar": float(np.sum(npts * ncells) / np.sum(ncells))}
        s.close()
    for mode in ("mlvs", "fixed3"):
        out[mode]["time_to_solution_ratio"] = runs["uvs"][1] / runs[mode][1]
        out[mode]["mlvs_vs_uvs_rel_l2"] = _fields_error(runs[mode][0], runs["uvs"][0])
        out[mode]["meets_1e-3_gate_rho_T"] = _gate(out[mode]["mlvs_vs_uvs_rel_l2"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed MLVS (and UVS) steps of the headline jet")
    ap.add_argument("--warmup", type=int, default=10, help="untimed MLVS steps after the base-grid steps")
    ap.add_argument("--interval", type=int, default=5, help="adaptation interval of the headline MLVS run")
    ap.add_argument("--no-uvs", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sections", action="store_true", help="only the headline (and the CPU baseline)")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--jet-only", action="store_true", help="only the headline jet (profiling runs)")
    ap.add_argument("--jet-mode", choices=("both", "mlvs", "uvs"), default="both")
    ap.add_argument("--tau-sweep", action="store_true", help="only the clustering-threshold sweep on the cylinder")
    ap.add_argument("--long-map", type=int, default=4, choices=[4, 9], help="mapping order of the --long runs")
    ap.add_argument("--long-scale", type=float, default=1.0,
                    help="factor on C_split, C_merge and eps_merge of the --long runs")
    ap.add_argument("--long", choices=("cylinder", "jet"), default=None,
                    help="only a whole run of that case, MLVS against UVS (10,000 cylinder or 2,000 jet steps)")
    ap.add_argument("--two-cavity-only", action="store_true", help="only the two-cavity comparison")
    ap.add_argument("--tc-mode", default="both", choices=["both", "uvs", "mlvs"])
    ap.add_argument("--tc-interval", type=int, default=5)
    ap.add_argument("--tc-map", type=int, default=4, choices=[4, 9])
    ap.add_argument("--tc-tau", type=float, default=0.05)
    ap.add_argument("--tc-scale", type=float, default=1.0, help="factor on C_split, C_merge and eps_merge")
    ap.add_argument("--tc-t-end", type=float, default=0.0,
                    help="with --two-cavity-only: run both forms to this time instead (the paper's t = 4)")
    ap.add_argument("--cylinder-only", action="store_true",
                    help="only the full-size cylinder comparison (profiling runs)")
    ap.add_argument("--cylinder-steps", type=int, default=200)
    ap.add_argument("--cylinder-kn", type=float, default=0.1)
    ap.add_argument("--cylinder-mode", choices=("both", "mlvs", "uvs"), default="both")
    ap.add_argument("--learned-only", action="store_true",
                    help="only the learned-vs-criterion comparison (selector training and adaptation)")
    ap.add_argument("--persistent-ab", action="store_true",
                    help="only the staged-against-persistent step comparison (cylinder, two-cavity)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; run it without --gpus or with "
              "--gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}))
        return
    if args.tau_sweep:
        print(json.dumps({"tau_sweep": tau_sweep()}), flush=True)
        return
    if args.long:
        print(json.dumps({"long_run": long_run(args.long, 10000 if args.long == "cylinder" else 2000,
                                               map_moments=args.long_map, scale=args.long_scale)}), flush=True)
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
    if args.persistent_ab:
        print(json.dumps({"persistent_ab": persistent_ab()}), flush=True)
        return
    if args.learned_only:
        print(json.dumps({"learned": learned_vs_criterion()}), flush=True)
        return
    if args.cylinder_only:
        print(json.dumps({"cylinder": cylinder_case(steps=args.cylinder_steps, mode=args.cylinder_mode,
                                                    Kn=args.cylinder_kn)}), flush=True)
        return
    if args.jet_only and args.jet_mode == "uvs":
        print(json.dumps({"jet": jet_headline(args.steps, args.warmup, with_mlvs=False, tune=not args.no_tune)}),
              flush=True)
        return
    head = jet_headline(args.steps, args.warmup, args.interval, with_uvs=not args.no_uvs
                                and args.jet_mode != "mlvs", tune=not args.no_tune)
    out = {"metric": "DUGKS cell·velocity updates/s, MLVS vs UVS time-to-solution at ≤1e-3 rel L2",
           "value": head["value"], "unit": "cell-velocity updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "slot jet 512x256 on [0,32]x[-8,8], sonic slot |y| <= 0.5, background rho 0.01 "
                                  "(pressure ratio 100), Kn_jet 1e-3, Shakhov Pr 2/3, 161x161 Newton-Cotes on "
                                  "[-7,7]^2, FP32 storage; MLVS C_split 0.01 C_merge 0.005 eps_merge 2e-5 tau_clust "
                                  "0.05, adaptation every %d steps inside the timed steps; %d untimed base-grid "
                                  "steps from the initial state, then %d untimed and %d timed MLVS steps"
                                  % (args.interval, JET_BASE_STEPS, max(args.warmup, 1), args.steps),
                      "n_cells": 131072, "base_points": 25921, "interval": args.interval,
                      "adaptations_timed": head["adaptations_timed"], "adapt_ms": head["adapt_ms"],
                      "adapt_split": head["adapt_split"],
                      "levels": head["levels"], "level_points": head["level_points"],
                      "level_cells": head["level_cells"], "nbar": head["nbar"], "n_cross": head["n_cross"],
                      "updates_per_step": head["updates_per_step"], "device_bytes": head["device_bytes"],
                      "graph": True, "variants": head["variants"], "tiles": head["tiles"]},
           "roofline": head["roofline"]}
    if "uvs" in head:
        out["uvs"] = head["uvs"]
    if not (args.no_sections or args.jet_only):
        for name, fn in (("sod", sod_case), ("cavity", cavity_case),
                         ("cylinder", lambda: cylinder_case(steps=args.cylinder_steps)),
                         ("cylinder_kn1", lambda: cylinder_case(steps=args.cylinder_steps, Kn=1.0)),
                         ("cylinder_on_gate", lambda: cylinder_case(steps=args.cylinder_steps, adapt=CYL_ADAPT_GATE)),
                         ("fp32_vs_fp64", fp32_vs_fp64), ("two_cavity", two_cavity_case)):
            t0 = time.perf_counter()
            out[name] = fn()
            print("section %s: %.1f s" % (name, time.perf_counter() - t0), file=sys.stderr, flush=True)
        if not args.no_learned:
            out["learned"] = learned_vs_criterion()
    if not (args.no_cpu_baseline or args.jet_only):
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(interval=args.interval)
        print("cpu baseline: %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
