"""Tile-shape autotuner.

The sweep kernels are compiled in several tile shapes (items along a grid
line x lines per workgroup; see wiu_set_tuning).  The tuner times every pair
of shapes on the caller's actual problem and keeps the fastest; results are
cached as JSON keyed by device, scheme and problem size class, so later runs
reuse them without timing.
"""
import json
import os

import torch

from . import wenoiu

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "wenoiu", "tuning.json")


def _key(kind, scheme, cells, nblocks=1):
    dev = torch.cuda.get_device_name(0)
    # size class: powers of two of the cell count
    cls = max(0, int(cells).bit_length() - 1)
    return f"{dev}|{kind}|{scheme}|2^{cls}|{nblocks}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_batched(plan, reps=3, cache=DEFAULT_CACHE, force=False):
    """Pick the tile shapes of a BatchedPlan (graph-replayed steps).
    The state is saved and restored, so tuning does not advance it."""
    cells, _, _ = plan.info()
    key = _key("batched", plan.scheme, cells, len(plan.shapes))
    table = _load(cache) if cache else {}
    if not force and key in table:
        vx, ve = table[key]["variant"]
        plan.retune(vx, ve)
        return table[key]
    saved = plan.U_all.clone()
    times = {}
    for vx in range(wenoiu.tuning_variants(0)):
        for ve in range(wenoiu.tuning_variants(1)):
            plan.retune(vx, ve)
            times[(vx, ve)] = _time(lambda: plan.step(graph=True), reps)
            plan.U_all.copy_(saved)
    best = min(times, key=times.get)
    plan.retune(*best)
    res = {"variant": list(best), "ms": times[best], "all_ms": {f"{a},{b}": t for (a, b), t in times.items()}}
    if cache:
        table[key] = res
        _store(cache, table)
    return res


def tune_single(solver, U, reps=3, cache=DEFAULT_CACHE, force=False):
    """Pick the process-wide tile shapes for one grid (rhs timings)."""
    key = _key("single", solver.scheme, solver.grid.nx * solver.grid.ny)
    table = _load(cache) if cache else {}
    if not force and key in table:
        vx, ve = table[key]["variant"]
        wenoiu.set_tuning(0, vx)
        wenoiu.set_tuning(1, ve)
        return table[key]
    out = torch.empty_like(U)
    times = {}
    for vx in range(wenoiu.tuning_variants(0)):
        for ve in range(wenoiu.tuning_variants(1)):
            wenoiu.set_tuning(0, vx)
            wenoiu.set_tuning(1, ve)
            times[(vx, ve)] = _time(lambda: solver.rhs(U, out), reps)
    best = min(times, key=times.get)
    wenoiu.set_tuning(0, best[0])
    wenoiu.set_tuning(1, best[1])
    res = {"variant": list(best), "ms": times[best], "all_ms": {f"{a},{b}": t for (a, b), t in times.items()}}
    if cache:
        table[key] = res
        _store(cache, table)
    return res
