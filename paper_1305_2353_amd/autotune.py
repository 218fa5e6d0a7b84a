"""Autotuner for the Form launches.

The Form kernel has several tile schedules (ctp_opts.tile; for a batch 0 =
operands loaded straight into a ring of LDS buffers, product stored as whole
lines, 1-3 = operands staged through registers) and a batch runs its Form
as one persistent launch whose workgroup count is free.  Which combination
is fastest depends on the shapes (tile counts, K = nelim, ragged edges), so
the tuner times every candidate on the caller's own data and keeps the
fastest per problem signature (in memory, optionally mirrored to a JSON
file).

Timing only: the candidates compute the same result (each tile's
arithmetic is fixed), so choosing among them never changes the output.
"""

import json
import os

import torch

TILES = (0, 1, 2, 3)
SCHUR_TILES = (0, 5, 6)   # single-node Form: default, register-staged, LDS ring with the plain product
WORKGROUPS = (256, 512, 1024, 2048)

_cache = {}


def _load(path):
    if path and os.path.exists(path):
        with open(path) as fh:
            _cache.update(json.load(fh))


def _save(path):
    if path:
        with open(path, "w") as fh:
            json.dump(_cache, fh, indent=1, sort_keys=True)


def _time(fn, reps):
    best = None
    stream = torch.cuda.current_stream()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def batch_signature(batch):
    n = sum(s[0] for s in batch.shapes)
    p = sum(s[1] for s in batch.shapes)
    return f"batch:{batch.count}:{n}:{p}:{batch.opts.method}:{int(batch.tiled)}"


def tune_batch(batch, pristine, reps=2, cache_path=None):
    """Pick (tile, workgroups) for batch.run(); pristine: a copy of the
    panels, restored before every timed run.  Leaves the choice in
    batch.opts.tile / batch.info.form_workgroups and returns a report."""
    _load(cache_path)
    key = batch_signature(batch)
    if key in _cache:
        best = _cache[key]
        batch.opts.tile, batch.info.form_workgroups = best["tile"], best["workgroups"]
        return {"best": best, "cached": True}
    timings = []

    def run():
        batch.panels.copy_(pristine)
        batch.run()

    run()   # warm-up (kernel attributes, first-touch)
    for tile in TILES:
        for wg in WORKGROUPS:
            batch.opts.tile, batch.info.form_workgroups = tile, wg
            timings.append({"tile": tile, "workgroups": wg, "ms": round(_time(run, reps), 3)})
    best = min(timings, key=lambda t: t["ms"])
    batch.opts.tile, batch.info.form_workgroups = best["tile"], best["workgroups"]
    _cache[key] = best
    _save(cache_path)
    return {"best": best, "cached": False, "timings": timings}


def tune_schur(run_form, opts, key, reps=2, cache_path=None):
    """Pick opts.tile for a single supernode's Form; run_form() launches it
    (all row blocks) with the current opts."""
    _load(cache_path)
    if key in _cache:
        opts.tile = _cache[key]["tile"]
        return {"best": _cache[key], "cached": True}
    timings = []
    run_form()
    for tile in SCHUR_TILES:
        opts.tile = tile
        timings.append({"tile": tile, "ms": round(_time(run_form, reps), 3)})
    best = min(timings, key=lambda t: t["ms"])
    opts.tile = best["tile"]
    _cache[key] = best
    _save(cache_path)
    return {"best": best, "cached": False, "timings": timings}
