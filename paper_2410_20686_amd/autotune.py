"""Autotuner for the compositors' tile edge and LDS batch sizes.

For one workload shape (Gaussian count, SH degree, view sizes) and every tile edge that divides
all views, it bins once, then times each stage of a forward + backward step with HIP events:
binning and the reverse projection once, the forward compositor at every forward batch size and
the reverse compositor at every backward batch size (the batch sizes only change how many
Gaussians a workgroup stages in LDS per round, not the workspace, so the stages are timed
separately and the best of each kept).  The fastest tile's choice is confirmed by timing whole
steps as HIP graph replays.  Results are cached in a JSON file keyed by device name, a
resolution bucket, a Gaussian-count bucket and the number of views.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .rasterizer import Rasterizer, TrainStep

TILES = (8, 16, 32)
BATCHES = {8: (32, 64, 128, 256), 16: (32, 64, 128, 256), 32: (64, 128, 256)}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "odgs_autotune.json")


def bucket_key(n: int, wh, device=None) -> str:
    dev = torch.cuda.get_device_name(device) if torch.cuda.is_available() else "cpu"
    mpx = sum(w * h for w, h in wh) / 1e6
    res = "x".join(sorted({"%dx%d" % (w, h) for w, h in wh}))
    return "%s|%s|mp%d|n2^%d|v%d" % (dev, res, round(math.log2(max(mpx, 1e-3))), round(math.log2(max(n, 1))), len(wh))


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _time_graph(step: TrainStep, reps: int) -> float:
    step.capture()
    return _time(step.replay, reps)


def tune(params, cams: torch.Tensor, dL: torch.Tensor, sh_degree: int, wh, settings: dict | None = None,
         tiles=TILES, batches=None, reps: int = 5, cache: str | None = DEFAULT_CACHE, log=None) -> dict:
    """Return {"tile", "batch", "batch_bwd", "ms", "table"}: the fastest configuration and, per
    tile, the stage timings it was chosen from (ms per step).

    params: (means, scales, quats, opacities, sh) device tensors; cams: [V, 12]; dL: upstream
    image gradient."""
    batches = batches or BATCHES
    n = int(params[0].shape[1])
    key = bucket_key(n, wh)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
        if key in db:
            return db[key]
    table = []
    for tile in tiles:
        if any(w % tile or h % tile for w, h in wh):
            continue
        st = dict(settings or {}, tile=tile, batch=0, batch_bwd=0)
        rast = Rasterizer(n, sh_degree, wh, st)
        s0 = rast.bin_checked(*params, cams)
        rast._alloc(int(s0["n_pairs"] * 1.05) + 4096)
        step = TrainStep(rast, params, cams, dL)
        step.run()
        row = dict(tile=tile, pairs=int(s0["n_pairs"]), bin=_time(step.bin, reps), fwd={}, bwd={})
        for b in batches[tile]:
            rast.set_batches(b, rast.plan.s.batch_bwd)
            row["fwd"][b] = _time(step.fwd, reps)
        for b in batches[tile]:
            rast.set_batches(rast.plan.s.batch, b)
            # (the accumulators keep adding up across repetitions without a preprocess: timing only)
            row["bwd"][b] = _time(lambda: (step.composite_bwd(), step.project_bwd()), reps)
        row["batch"] = min(row["fwd"], key=row["fwd"].get)
        row["batch_bwd"] = min(row["bwd"], key=row["bwd"].get)
        row["ms"] = row["bin"] + row["fwd"][row["batch"]] + row["bwd"][row["batch_bwd"]]
        if rast.status()["flags"]:
            raise RuntimeError("pair overflow while tuning")
        table.append(row)
        if log:
            log("tile %2d: bin %.3f, fwd %s, bwd+proj %s -> %.3f ms" % (
                tile, row["bin"], {k: round(v, 3) for k, v in row["fwd"].items()},
                {k: round(v, 3) for k, v in row["bwd"].items()}, row["ms"]))
        del step, rast
        torch.cuda.empty_cache()
    best = min(table, key=lambda r: r["ms"])
    # confirm with whole-step graph replays
    rast = Rasterizer(n, sh_degree, wh, dict(settings or {}, tile=best["tile"], batch=best["batch"],
                                             batch_bwd=best["batch_bwd"]))
    s0 = rast.bin_checked(*params, cams)
    rast._alloc(int(s0["n_pairs"] * 1.05) + 4096)
    ms = _time_graph(TrainStep(rast, params, cams, dL), reps)
    res = dict(tile=best["tile"], batch=best["batch"], batch_bwd=best["batch_bwd"], ms=ms,
               table=[{k: (({str(b): t for b, t in v.items()}) if isinstance(v, dict) else v) for k, v in r.items()}
                      for r in table])
    if log:
        log("chosen tile %d batch %d batch_bwd %d: %.3f ms/step (graph)" % (res["tile"], res["batch"],
                                                                          res["batch_bwd"], ms))
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
