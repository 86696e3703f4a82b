"""Autotuner for the compositor's tile edge and LDS batch size.

For one workload shape (Gaussian count, SH degree, view sizes) it times a full forward + backward
step (HIP graph replays, HIP events) for every supported (tile, batch) pair and keeps the
fastest.  Results are cached in a JSON file keyed by device name, a resolution bucket, a
Gaussian-count bucket and the number of views, so later runs of similar workloads reuse them.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .rasterizer import Rasterizer, TrainStep

CANDIDATES = [(8, 64), (8, 128), (8, 256), (16, 64), (16, 128), (16, 256), (32, 128), (32, 256)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "odgs_autotune.json")


def bucket_key(n: int, wh, device=None) -> str:
    dev = torch.cuda.get_device_name(device) if torch.cuda.is_available() else "cpu"
    mpx = sum(w * h for w, h in wh) / 1e6
    res = "x".join(sorted({"%dx%d" % (w, h) for w, h in wh}))
    return "%s|%s|mp%d|n2^%d|v%d" % (dev, res, round(math.log2(max(mpx, 1e-3))), round(math.log2(max(n, 1))), len(wh))


def _time_step(step: TrainStep, reps: int) -> float:
    step.capture()
    for _ in range(2):
        step.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(params, cams: torch.Tensor, dL: torch.Tensor, sh_degree: int, wh, settings: dict | None = None,
         candidates=CANDIDATES, reps: int = 5, cache: str | None = DEFAULT_CACHE, log=None) -> dict:
    """Return {"tile", "batch", "ms", "table"} for the fastest supported pair.

    params: (means, scales, quats, opacities, sh) device tensors; cams: [V, 12]; dL: upstream
    image gradient.  Candidates whose tile does not divide every view size are skipped."""
    n = int(params[0].shape[1])
    key = bucket_key(n, wh)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
        if key in db:
            return db[key]
    table = []
    for tile, batch in candidates:
        if any(w % tile or h % tile for w, h in wh):
            continue
        st = dict(settings or {}, tile=tile, batch=batch)
        rast = Rasterizer(n, sh_degree, wh, st)
        s0 = rast.bin_checked(*params, cams)
        rast._alloc(int(s0["n_pairs"] * 1.05) + 4096)
        step = TrainStep(rast, params, cams, dL)
        ms = _time_step(step, reps)
        if rast.status()["flags"]:
            raise RuntimeError("pair overflow while tuning")
        table.append(dict(tile=tile, batch=batch, ms=ms, pairs=s0["n_pairs"]))
        if log:
            log("tile %2d batch %3d: %.3f ms/step, %d pairs" % (tile, batch, ms, s0["n_pairs"]))
        del step, rast
        torch.cuda.empty_cache()
    best = min(table, key=lambda r: r["ms"])
    res = dict(tile=best["tile"], batch=best["batch"], ms=best["ms"], table=table)
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db = {}
        if os.path.exists(cache):
            with open(cache) as f:
                db = json.load(f)
        db[key] = res
        tmp = cache + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, cache)
    return res
