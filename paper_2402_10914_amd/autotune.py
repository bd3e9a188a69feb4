"""Autotuner for the interface-kernel tile shape and the batch sweep order.

The library offers several interface tile shapes (TF interfaces x TR segments, ``api.tile_shapes()``)
and, for batches, three orders of the tile list (grid by grid, largest grid first, round-robin over
grids).  None of them changes a single bit of the results; they only change occupancy, halo
overhead, tail effects and cache locality.  The tuner times every candidate on the caller's actual
workload (HIP events around a captured-graph replay, or around ``dfw_run``), keeps the fastest and
caches the choice in a JSON file keyed by GPU architecture, HIP version, element type, flux and a
hash of the grid sizes.

Cache file: ``$DFW_TUNE_CACHE`` or ``~/.cache/dfweno/tuning.json``.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import torch

from . import api
from ._lib import DFW_ORDER_GRID, DFW_ORDER_INTERLEAVED, DFW_ORDER_LARGEST_FIRST

ORDERS = [DFW_ORDER_GRID, DFW_ORDER_LARGEST_FIRST, DFW_ORDER_INTERLEAVED]


def cache_path() -> str:
    return os.environ.get("DFW_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "dfweno", "tuning.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:  # pragma: no cover - depends on the runtime
        return "unknown"


def _key(kind, sizes, dtype, params: api.Params) -> str:
    """Problem sizes, every scheme option but the tile itself, and the library's tile shapes (a
    tile index means another shape in a library with another shape list)."""
    opts = {k: v for k, v in sorted(params.__dict__.items()) if k != "tile"}
    blob = json.dumps([sorted(sizes), opts, api.tile_shapes()])
    h = hashlib.sha1(blob.encode()).hexdigest()[:12]
    return f"{kind}|{_arch()}|hip{torch.version.hip}|{str(dtype).split('.')[-1]}|flux{params.flux}|{h}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    d = _load()
    d[key] = value
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1)
    os.replace(tmp, p)


def _time_batch(grids, Ws, alphas, params, dtype, order, steps, reps):
    b = api.Batch(grids, params, dtype, order)
    W0, A0 = b.pack(Ws, alphas)
    W, A = W0.clone(), A0.clone()
    b.run(W, A, steps, use_graph=True)  # capture
    best = float("inf")
    for _ in range(reps):
        W.copy_(W0)
        A.copy_(A0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(W, A, steps, use_graph=True)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_batch(grids, Ws, alphas, params: api.Params, dtype=torch.float64, steps=5, reps=2, use_cache=True):
    """Returns (tile, order, timings) for a batch; grids = [(nx, ny, dx, dy, bc_x, bc_y)]."""
    key = _key("batch", [(g[0], g[1], g[4], g[5]) for g in grids], dtype, params)
    if use_cache:
        hit = _load().get(key)
        if hit:
            return hit["tile"], hit["order"], hit["timings"]
    timings = {}
    for tile in range(len(api.tile_shapes())):
        p = api.Params(**{**params.__dict__, "tile": tile})
        for order in ORDERS:
            timings[f"{tile},{order}"] = _time_batch(grids, Ws, alphas, p, dtype, order, steps, reps)
    best = min(timings, key=timings.get)
    tile, order = (int(x) for x in best.split(","))
    _store(key, {"tile": tile, "order": order, "timings": timings})
    return tile, order, timings


def tune_grid(prob, params: api.Params, dtype=torch.float64, steps=5, reps=2, use_cache=True):
    """Returns (tile, timings) for one grid (a workloads.Problem)."""
    key = _key("grid", [(prob.nx, prob.ny, prob.bc_x, prob.bc_y)], dtype, params)
    if use_cache:
        hit = _load().get(key)
        if hit:
            return hit["tile"], hit["timings"]
    W0 = torch.tensor(prob.W, dtype=dtype, device="cuda")
    A0 = torch.tensor(prob.alpha, dtype=dtype, device="cuda")
    timings = {}
    for tile in range(len(api.tile_shapes())):
        p = api.Params(**{**params.__dict__, "tile": tile})
        st = api.Stepper.for_problem(prob, p, dtype)
        W, A = W0.clone(), A0.clone()
        st.run(W, A, 1)
        best = float("inf")
        for _ in range(reps):
            W.copy_(W0)
            A.copy_(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.run(W, A, steps)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        timings[str(tile)] = best
    tile = int(min(timings, key=timings.get))
    _store(key, {"tile": tile, "timings": timings})
    return tile, timings
