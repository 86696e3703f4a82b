#!/usr/bin/env python
"""Benchmark of the gfx950 omnidirectional Gaussian rasterizer.

Metric: forward+backward megapixels per second at 2048x1024 with 500k Gaussians, all views of
one step batched into one launch per stage (one HIP graph per step), next to the same work done
as one pipeline per view.

Workload "M": 500,000 Gaussians of the roaming distribution (70% in 50 blobs, 30% uniform in the
shell r in [2, 20], SH degree 3), 8 views of 2048x1024 ERP with camera centres uniform in a 1 m
cube and random yaw; upstream image gradient N(0, 1).  A step = preprocess, bin + sort, forward
compositing, reverse compositing and projection adjoint over all 8 views, gradients summed over
views.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd megapixels/s at 2048×1024, 500k Gaussians; batched vs per-view"
HBM_PEAK_GBS = 8000.0
# FP32 vector issue rate without packed instructions: 256 CUs x 64 lanes x 2.4 GHz (lane-ops/s)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic FP32 lane-operations per (pixel, list entry) evaluation of the compositors: about 9
# when the entry is rejected (offset, exponent, footprint test) and about 23 (forward) or 50
# (reverse) when it is accepted, exp included (the per-unit figures of the measurement plan).
OPS_REJECT = 9
OPS_FWD_ACCEPT, OPS_BWD_ACCEPT = 23, 50

# Algorithmic HBM bytes of one fwd+bwd step (SH degree 3): per Gaussian, the parameters read
# (236 B) in the forward, read again and their gradients written (236 + 236 B) in the backward,
# once per step for all views; per (Gaussian, view) item a 48 B record and 16 B of scan state in
# the forward and 40 B of 2D gradients in the backward; per Gaussian-tile pair 12 B emitted, >= 24 B
# sorted and a 44 B record gathered by each compositor; per pixel 20 B written by the forward
# (RGB, T, last index) and 20 B read by the backward (dL/dRGB, T, last index).
def step_bytes(n, views, pairs, pixels):
    return 3 * 236 * n + (48 + 16 + 40) * n * views + (12 + 24 + 44 + 44) * pairs + 40 * pixels


PROFILE = os.path.join(ROOT, "profiles", "render_kernels_M_500k_8x2048x1024.txt")


def profiled(kernel: str):
    """The committed rocprofv3 summary's figures for one kernel (average duration, calibrated HBM
    bytes per launch, ...), or None when the summary is missing, lacks the kernel, or was taken
    from other compositor sources."""
    from paper_2410_20686_amd import profiling
    rows, src = profiling.read_summary(PROFILE)
    if not rows or src != profiling.source_hash(ROOT):
        return None
    return rows.get(kernel)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--batch", type=int, default=0, help="forward LDS batch (0: library default)")
    ap.add_argument("--batch-bwd", type=int, default=0, help="reverse LDS batch (0: library default)")
    ap.add_argument("--n", type=int, default=0, help="Gaussian count (0: the workload's own)")
    ap.add_argument("--workload", default="M", choices=("M", "cfg0", "cfg1", "cfg2", "cfg3", "cfg4"),
                    help="M is the metric's workload; the others are context runs (same JSON fields)")
    ap.add_argument("--schedule", default="queue", choices=("queue", "persistent", "tile_id"),
                    help="compositor tile scheduling: one workgroup per tile, longest list first (default), "
                         "persistent workgroups claiming tiles from that queue, or one workgroup per tile in "
                         "tile id order")
    ap.add_argument("--autotune", action="store_true", help="pick the tile and batch sizes with the autotuner first")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of this many MiB (a known-size reference "
                         "dispatch for hardware byte counters)")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-train", action="store_true", help="skip timing the loss + Adam training iteration")
    ap.add_argument("--no-spherical", action="store_true",
                    help="skip timing the same step with the spherical (exact per-ray) footprint")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels-per-view", type=int, default=4096)
    return ap.parse_args()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def time_graph(fn, steps, warmup):
    """Capture fn() into one HIP graph and time `steps` replays (after `warmup` replays)."""
    import torch
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # eager warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, g


def time_stages(step, steps):
    """Eager steps with HIP events around every entry point (all on torch's current stream, the
    stream the kernels are launched on).  Returns mean ms per stage."""
    import torch
    names = ("bin", "fwd", "composite_bwd", "project_bwd")
    fns = (step.bin, step.fwd, step.composite_bwd, step.project_bwd)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record()
        for j, f in enumerate(fns):
            f()
            ev[k][j + 1].record()
    torch.cuda.synchronize()
    return {n: sum(ev[k][j].elapsed_time(ev[k][j + 1]) for k in range(steps)) / steps for j, n in enumerate(names)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % args.gpus)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2410_20686_amd import scenes
    from paper_2410_20686_amd import _odgs as B
    from paper_2410_20686_amd.rasterizer import Rasterizer, TrainStep

    t0 = time.time()
    sc, cams, st = scenes.config(args.workload, n=args.n or None)
    st = dict(st, tile=args.tile, batch=args.batch, batch_bwd=args.batch_bwd, schedule=args.schedule)
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    V = len(wh)
    mp_per_step = sum(w * h for w, h in wh) / 1e6
    dL_np = scenes.upstream_gradient(cams, 1005)
    log("scene ready %.1fs" % (time.time() - t0))

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    tensors = [dev(a) for a in (sc.means, sc.scales, sc.quats, sc.opacities, sc.sh, cams.cams)]
    dL = dev(dL_np)

    tuned = None
    if args.autotune:
        from paper_2410_20686_amd import autotune
        tuned = autotune.tune(tensors[:5], tensors[5], dL, sc.sh_degree, wh, st, cache=None, log=log)
        st = dict(st, tile=tuned["tile"], batch=tuned["batch"], batch_bwd=tuned["batch_bwd"])
        log("autotuned:", tuned["tile"], tuned["batch"], tuned["batch_bwd"])

    # size the pair list from one binning pass, then keep it fixed (no host sync inside steps)
    rast = Rasterizer(sc.n, sc.sh_degree, wh, st)
    status0 = rast.bin_checked(*tensors)
    rast._alloc(int(status0["n_pairs"] * 1.05) + 4096)
    step = TrainStep(rast, tensors[:5], tensors[5], dL)
    ms_batched, _graph = time_graph(step.run, args.steps, args.warmup)
    status = rast.status()
    if status["flags"] & B.STATUS_OVERFLOW:
        raise RuntimeError("pair list overflowed during timing")
    log("batched %.3f ms/step, P=%d" % (ms_batched, status["n_pairs"]))

    stages = time_stages(step, max(3, min(args.steps, 10)))
    # work counters for the algorithmic op count: one extra forward in the counting variant
    rast.set_batches(rast.plan.s.batch, rast.plan.s.batch_bwd, count_work=True)
    step.fwd()
    pc = rast.pixel_counts().to(torch.int64)
    cnt = pc.sum(dim=0).cpu().numpy()
    rast.set_batches(rast.plan.s.batch, rast.plan.s.batch_bwd, count_work=False)
    # wavefront iterations: every 8x8 quadrant is one wavefront, which steps through its list
    # until its slowest pixel is done
    wave_iters = [0, 0]
    off = 0
    for (w, h) in wh:
        q = pc[off:off + w * h].reshape(h // 8, 8, w // 8, 8, 4).amax(dim=(1, 3))
        wave_iters[0] += int(q[..., 2].sum())
        wave_iters[1] += int(q[..., 3].sum())
        off += w * h
    contrib_total, evals_fwd, evals_bwd = int(cnt[1]), int(cnt[2]), int(cnt[3])
    log("stages ms", stages)

    # a whole training iteration (L1 loss against a fixed target + backward + Adam update) as
    # context for the metric; targets are the step's own first image dimmed by 10%
    train = None
    if not args.no_train:
        from paper_2410_20686_amd.optim import GaussianParams, LossTrainStep
        target = (step.rgb * 0.9).contiguous()
        o = tensors[3].clamp(1e-4, 1 - 1e-4)
        gp = GaussianParams(tensors[0], torch.log(tensors[1]), tensors[2], torch.log(o / (1 - o)), tensors[4],
                            sh_degree=sc.sh_degree)
        tstep = LossTrainStep(rast, gp, tensors[5], target)
        ms_train, _g3 = time_graph(tstep.run, args.steps, args.warmup)
        train = dict(ms_per_step=round(ms_train, 4), loss_last=round(float(tstep.loss.cpu()), 6))
        if rast.status()["flags"] & B.STATUS_OVERFLOW:
            train = dict(note="pair list overflowed while the parameters moved; not timed")
        log("train iteration %.3f ms" % ms_train)
        del tstep, gp

    # the same step with the spherical footprint (exact per-ray evaluation instead of the local
    # affine approximation): its own pair list (cone rectangles) and compositors
    sph = None
    if not args.no_spherical:
        st_s = dict(st, footprint="spherical")
        rs = Rasterizer(sc.n, sc.sh_degree, wh, st_s)
        s0 = rs.bin_checked(*tensors)
        rs._alloc(int(s0["n_pairs"] * 1.05) + 4096)
        sstep = TrainStep(rs, tensors[:5], tensors[5], dL)
        ms_sph, _g4 = time_graph(sstep.run, args.steps, args.warmup)
        if rs.status()["flags"] & B.STATUS_OVERFLOW:
            raise RuntimeError("pair list overflowed during timing (spherical footprint)")
        sst = time_stages(sstep, max(3, min(args.steps, 10)))
        sph = dict(ms_per_step=round(ms_sph, 4), value=round(mp_per_step / (ms_sph / 1e3), 2), unit="MP/s",
                   pairs=int(rs.status()["n_pairs"]), stages_ms={k: round(v, 4) for k, v in sst.items()})
        log("spherical footprint %.3f ms/step, P=%d, stages %s" % (ms_sph, sph["pairs"], sst))
        del sstep, rs

    per_view = None
    if not args.no_per_view:
        pv_steps = []
        for v in range(V):
            cv = cams.view(v)
            rv = Rasterizer(sc.n, sc.sh_degree, [wh[v]], st)
            tv = tensors[:5] + [dev(cv.cams)]
            off = 3 * sum(w * h for w, h in wh[:v])
            dv = dL[off:off + 3 * wh[v][0] * wh[v][1]]
            s0 = rv.bin_checked(*tv)
            rv._alloc(int(s0["n_pairs"] * 1.05) + 4096)
            pv_steps.append(TrainStep(rv, tv[:5], tv[5], dv))
        acc = tuple(torch.empty_like(x) for x in tensors[:5])

        def run_per_view():
            for k, s in enumerate(pv_steps):
                s.run()
                for a, g in zip(acc, s.grads):
                    if k == 0:
                        a.copy_(g)
                    else:
                        a.add_(g)

        ms_pv, _g2 = time_graph(run_per_view, args.steps, args.warmup)
        per_view = dict(ms_per_step=ms_pv, value=mp_per_step / (ms_pv / 1e3), speedup_batched=ms_pv / ms_batched)
        log("per-view %.3f ms/step" % ms_pv)
        del pv_steps

    # roofline of the dominant kernel (reverse compositing: one kernel per odgs_composite_bwd call)
    dom = max(stages, key=stages.get)
    alg_ops = {
        "fwd": OPS_REJECT * (evals_fwd - contrib_total) + OPS_FWD_ACCEPT * contrib_total,
        "composite_bwd": OPS_REJECT * (evals_bwd - contrib_total) + OPS_BWD_ACCEPT * contrib_total,
    }
    roof = None
    if dom in alg_ops:
        achieved = alg_ops[dom] / (stages[dom] / 1e3) / 1e12
        # one wavefront per 16x16 block at tiles of 16 and 32, one workgroup per tile at 8
        if dom == "composite_bwd":
            kname = ("odgs::render_bwd4_kernel<%d, %d>" if st["tile"] >= 16 else "odgs::render_bwd_kernel<%d, %d>") % (
                st["tile"], rast.plan.s.batch_bwd)
        elif st["tile"] >= 16:
            kname = "odgs::render_fwd4_kernel<%d, %d>" % (st["tile"], rast.plan.s.batch)
        else:
            kname = "odgs::render_fwd_kernel<%d, %d, false, false>" % (st["tile"], rast.plan.s.batch)
        prof = profiled(kname)
        # the same algorithmic work over the committed profile's average duration of this kernel
        ach_prof = alg_ops[dom] / (prof["avg_us"] * 1e-6) / 1e12 if prof else None
        roof = dict(bound="alu", kernel=dom, achieved=round(achieved, 3), peak=round(ALU_PEAK_TOPS, 2), unit="Top/s",
                    frac=round(achieved / ALU_PEAK_TOPS, 4),
                    traffic=int(prof["traffic_bytes"]) if prof else None,
                    ops_per_launch=alg_ops[dom], duration_us=round(stages[dom] * 1e3, 1),
                    duration_us_profile=prof["avg_us"] if prof else None,
                    achieved_profile=round(ach_prof, 3) if prof else None,
                    frac_profile=round(ach_prof / ALU_PEAK_TOPS, 4) if prof else None,
                    hbm_frac_profile=prof["hbm_frac"] if prof else None,
                    lds_busy_profile=prof.get("lds_busy") if prof else None,
                    lds_bw_frac_profile=prof.get("lds_bw_frac") if prof else None,
                    lane_util_profile=prof.get("lanes") if prof else None,
                    valu_issue_profile=prof["valu_issue"] if prof else None,
                    work=dict(tests=evals_bwd if dom == "composite_bwd" else evals_fwd, accepts=contrib_total,
                              wave_iters=wave_iters[1] if dom == "composite_bwd" else wave_iters[0]))
    # the whole step against the HBM roofline, with the algorithmic bytes of one step
    sb = step_bytes(sc.n, V, int(status["n_pairs"]), sum(w * h for w, h in wh))
    hbm_step = dict(bytes=sb, GBs=round(sb / (ms_batched / 1e3) / 1e9, 1),
                    frac=round(sb / (ms_batched / 1e3) / (HBM_PEAK_GBS * 1e9), 4))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        _, pix = scenes.sparse_upstream_gradient(cams, 2005, args.cpu_pixels_per_view)
        gpix = np.random.default_rng(3005).standard_normal((len(pix), 3))
        tc = time.time()
        O.render(sc, cams, st, mode=32, pix=pix, band=True)
        O.backward(sc, cams, st, gpix, mode=32, pix=pix, band=True)
        dt = time.time() - tc
        cpu = dict(value=round(len(pix) / 1e6 / dt, 6), unit="MP/s", cores=O.num_threads(), kind="oracle",
                   sample="%d random pixels (%d per view) of workload %s, band-mode (tile-list candidates) forward "
                          "+ backward in FP32 decision mode, each call including its own projection of all items and "
                          "tile-list construction; %.1f s" % (len(pix), args.cpu_pixels_per_view, args.workload, dt))
        log("cpu baseline", cpu)

    value = mp_per_step / (ms_batched / 1e3)
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "MP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_batched, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("M: 500k Gaussians (roaming: 70%% in 50 blobs, 30%% shell r 2-20, SH degree 3), "
                                "%d views 2048x1024, fwd+bwd, all views batched in one HIP graph per step" % V)
                   if args.workload == "M" else "%s (context run, not the metric's workload): %d Gaussians, "
                   "views %s" % (args.workload, sc.n, sorted(set(wh))),
                   "gaussians": sc.n, "views": V, "width": wh[0][0], "height": wh[0][1], "sh_degree": sc.sh_degree,
                   "tile": st["tile"], "batch": rast.plan.s.batch, "batch_bwd": rast.plan.s.batch_bwd,
                   "pairs": status["n_pairs"], "schedule": args.schedule,
                   "autotuned": tuned is not None},
        "per_view": per_view,
        "train_iteration": train,
        "spherical_footprint": sph,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "roofline": roof,
        "hbm_step": hbm_step,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
