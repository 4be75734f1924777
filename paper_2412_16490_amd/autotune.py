"""Autotuner for the solver's launch knobs.

For a batch shape it times the full solve (ADMM + polish) over a small grid of
knobs and keeps the fastest configuration whose results are all converged:

* ``polish_chunk`` the iteration-chunk schedule of the FP64 polish: the
                   factorisations a QP takes in the one-lane polish (group
                   shape: one lane per QP, 64 QPs per wavefront) before it is
                   handed to the contact-parallel polish (group shape: one
                   lane per contact, 8 or 16 QPs per wavefront); 0 keeps every
                   QP in the one-lane polish, 1 hands nearly all on;
* ``admm_waves``   register budget of the ADMM kernel as resident waves per
                   SIMD (1 = no cap, 2, 3, 4): trades spills for occupancy;
* ``check_every``  iterations between residual checks / rho updates;
* ``batched``      persistent cost-sorted launch over a tile queue vs one
                   workgroup per tile in grasp order.

Results are cached in a JSON file keyed by (device name, m_max, histogram of
wrench counts, number of grasps rounded to a power of two), so a serving loop
or a benchmark tunes once per shape class.
"""
from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np

from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "bodex_qp_autotune.json")
DEFAULT_GRID = {"polish_chunk": [0, 1, 4, 8, 12, 16, 20, 24], "admm_waves": [1, 2, 3], "batched": [0, 1]}


def shape_key(device_name: str, batch: api.DeviceBatch) -> str:
    s = np.diff(batch.woff)
    hist = np.bincount(np.clip(s, 0, 64) // 8, minlength=9).tolist()
    g = 1 << int(np.ceil(np.log2(max(1, batch.n_grasps))))
    return "%s|m%d|s%s|g%d" % (device_name, batch.m_max, hist, g)


def _time_solve(params: api.Params, batch: api.DeviceBatch, reps: int, stream) -> tuple[float, bool]:
    import torch
    s = api.Solver(params, stream=stream.cuda_stream)
    st = api.new_state(batch.n_grasps, batch.n_qps, batch.m_max)
    res = api.new_result(batch.n_grasps, batch.n_qps, batch.m_max)
    with torch.cuda.stream(stream):
        s.solve(batch, state=st, result=res)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            s.solve(batch, state=st, result=res)
        stream.synchronize()
        dt = (time.perf_counter() - t0) / reps
    ok = bool(np.all((res["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
    s.close()
    return dt, ok


def tune(batch: api.DeviceBatch, base: api.Params | None = None, reps: int = 3,
         grid: dict | None = None, cache_path: str | None = DEFAULT_CACHE, force: bool = False):
    """Return (best knobs, table of (knobs, ms, converged))."""
    import torch
    dev = torch.cuda.get_device_name()
    key = shape_key(dev, batch)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if key in cache and not force:
        return cache[key]["best"], cache[key]["table"]
    grid = grid or DEFAULT_GRID
    s_max = int(np.max(np.diff(batch.woff)))
    stream = torch.cuda.Stream()
    table = []
    names = list(grid)
    for combo in itertools.product(*[grid[n] for n in names]):
        knobs = dict(zip(names, combo))
        p = api.Params.from_buffer_copy(bytes(base)) if base is not None else api.default_params()
        p.m_max = batch.m_max
        p.s_max = max(p.s_max, s_max)
        p = apply(p, knobs)
        ms, ok = _time_solve(p, batch, reps, stream)
        table.append({"knobs": knobs, "ms": round(ms * 1e3, 4), "converged": ok})
    good = [t for t in table if t["converged"]] or table
    best = min(good, key=lambda t: t["ms"])["knobs"]
    if cache_path:
        cache[key] = {"best": best, "table": table}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return best, table


def apply(params: api.Params, knobs: dict) -> api.Params:
    p = api.Params.from_buffer_copy(bytes(params))
    if "polish_chunk" in knobs:
        p.polish_chunk = int(knobs["polish_chunk"])
    if "admm_waves" in knobs:
        p.admm_waves = int(knobs["admm_waves"])
    if "check_every" in knobs:
        p.check_every = int(knobs["check_every"])
    if "batched" in knobs:
        if knobs["batched"]:
            p.flags |= api.F_BATCHED
        else:
            p.flags &= ~api.F_BATCHED
    return p
