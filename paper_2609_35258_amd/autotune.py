"""Autotuner for the launch variants of the step's kernels and the traversal
tiles of structured meshes.

For each tunable stage the library holds several instantiations of the kernel
(pairs of velocity points per lane per load batch and minimum waves per SIMD,
i.e. memory-level parallelism against a register budget per lane).  The tuner
times every variant on the solver's current
state with HIP events (``Solver.time_stage``), keeps the fastest, and caches
the choice in a JSON file keyed by GPU architecture, storage precision, the
stage's work shape (items, mean velocity points per item), the number of
variants the stage has and a hash of the built library, so later runs of the
same shape with the same kernels skip the sweep, and a rebuilt library or a
new variant sweeps again.  Variants only change scheduling, never the
results.

The traversal tiles (``Solver.set_tiling``: tw x th cells visited, and their
rows stored, together) set which stencil rows meet in one XCD's L2.  The tile
tuner times one whole step (the sum over the stages the step launches of
their mean launch time) for each candidate shape on the current state and
level set, keeps the fastest and caches it keyed by the mesh, the step's
stages and the mean level size.  Tiles do not change the results either.
"""
from __future__ import annotations

import functools
import hashlib
import json
import os
from typing import Dict, Iterable, Optional

TILES = ((16, 8), (32, 8), (8, 8), (32, 4), (64, 4), (16, 16), (8, 16), (0, 0))
TUNABLE = ("cell", "face_rec", "face_target", "xface", "update", "face", "update_cell", "persistent")


def default_cache() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "mlvs", "tuned.json")


def _arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


@functools.lru_cache(maxsize=1)
def _lib_tag() -> str:
    from . import LIB_PATH
    h = hashlib.sha256()
    with open(LIB_PATH, "rb") as f:
        for block in iter(lambda: f.read(1 << 20), b""):
            h.update(block)
    return h.hexdigest()[:12]


def shape_key(solver, stage: str, precision: int) -> Optional[str]:
    items, pts = solver.stage_size(stage)
    if items == 0:
        return None
    per = int(round(pts / items))
    # bucket the size so nearby shapes share an entry
    bucket = 1 << max(per - 1, 1).bit_length()
    return "%s|fp%d|%s|items~%d|pts<=%d|variants%d|lib%s" % (
        _arch(), precision, stage, 1 << max(items - 1, 1).bit_length(), bucket, solver.variants(stage), _lib_tag())


def autotune(solver, precision: int, stages: Optional[Iterable[str]] = None, reps: int = 5,
             cache: Optional[str] = None, force: bool = False) -> Dict[str, dict]:
    """Choose the fastest variant per stage; returns {stage: {variant, ms, key, from_cache}}.
    stages: default, the tunable stages the solver's step launches."""
    if stages is None:
        stages = [st for st in solver.step_stages() if st in TUNABLE]
    path = cache or default_cache()
    table = _load(path)
    out = {}
    for st in stages:
        key = shape_key(solver, st, precision)
        if key is None:
            continue
        if key in table and not force:
            solver.set_variant(st, table[key]["variant"])
            out[st] = dict(table[key], key=key, from_cache=True)
            continue
        times = []
        for v in range(solver.variants(st)):
            solver.set_variant(st, v)
            solver.time_stage(st, 1)                      # warm the variant
            times.append(solver.time_stage(st, reps))
        best = min(range(len(times)), key=lambda k: times[k])
        solver.set_variant(st, best)
        table[key] = {"variant": best, "ms": times[best], "all_ms": times}
        out[st] = dict(table[key], key=key, from_cache=False)
    _store(path, table)
    return out


def _load(path):
    if os.path.exists(path):
        try:
            with open(path) as f:
                return json.load(f)
        except (OSError, ValueError):
            pass
    return {}


def _store(path, table):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    except OSError:
        pass


def step_ms(solver, reps: int = 3) -> float:
    """Mean time of one step as the sum of its stages' mean launch times."""
    total = 0.0
    for st in solver.step_stages():
        if solver.stage_size(st)[0] == 0:
            continue
        solver.time_stage(st, 1)
        total += solver.time_stage(st, reps)
    return total


def autotune_tiles(solver, precision: int, candidates: Iterable = TILES, reps: int = 3,
                   cache: Optional[str] = None, force: bool = False) -> dict:
    """Choose the traversal tiles with the shortest step; returns {tiles, ms,
    all_ms, key, from_cache}, or {} where tiles do not apply (unstructured or
    1-D meshes)."""
    if not getattr(solver, "structured", False):
        return {}
    import numpy as np
    npts, ncells, _ = solver.level_info()
    nbar = int(round(float(np.sum(np.asarray(npts) * np.asarray(ncells)) / max(int(np.sum(ncells)), 1))))
    key = "%s|fp%d|tiles|cells%d|%s|pts<=%d|lib%s" % (
        _arch(), precision, solver.n_cells, "+".join(solver.step_stages()), 1 << max(nbar - 1, 1).bit_length(),
        _lib_tag())
    path = cache or default_cache()
    table = _load(path)
    if key in table and not force:
        solver.set_tiling(*table[key]["tiles"])
        return dict(table[key], key=key, from_cache=True)
    cands = [tuple(t) for t in candidates]
    times = []
    for t in cands:
        solver.set_tiling(*t)
        times.append(step_ms(solver, reps))
    best = min(range(len(cands)), key=lambda k: times[k])
    solver.set_tiling(*cands[best])
    table[key] = {"tiles": list(cands[best]), "ms": times[best], "all_ms": times,
                  "candidates": [list(t) for t in cands]}
    _store(path, table)
    return dict(table[key], key=key, from_cache=False)
