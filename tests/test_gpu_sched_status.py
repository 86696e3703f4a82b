"""Compositor scheduling and the device status record, through the C ABI.

* The three tile schedules (one workgroup per task in longest-first queue order, persistent
  workgroups claiming tasks from that queue, one workgroup per tile in tile id order) composite the
  same pixels in the same order, so images are bit-identical; gradients agree to the order in which
  per-tile partial sums reach the FP64 accumulators, and where the queue splits tiles into quadrant
  tasks, to the parity tolerance.
* The work queue is a permutation of the global tile ids in non-increasing list length.
* The longest lists (every list, in a launch of few tiles) are split into quadrant tasks by the
  queue schedules, with the same images and (up to summation order) gradients.
* The reverse compositor refuses a pair list the forward has not composited (a bin_sort between
  them), reporting it in the status record instead of reading stale culling masks.
* Culled and non-finite items are counted.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests import _gpu as G
from tests._util import settings
from tests.test_gpu_parity import CASES, _masked_upstream, _views

pytestmark = pytest.mark.gpu


def _uneven_case():
    sc = scenes.roaming_scene(6007, 3, seed=81)
    cams = scenes.uneven_cameras(4, seed=81, sizes=((128, 64), (256, 128), (512, 256)))
    return sc, cams


@pytest.mark.parametrize("footprint", ["affine", "spherical"])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_schedules_agree(tile, footprint):
    sc, cams = _uneven_case()
    st = settings(tile=tile, footprint=footprint)
    fwd = O.render(sc, cams, st, mode=32)
    dL = _masked_upstream(cams, fwd["margin"], seed=1081)
    runs = {s: G.run_gpu(sc, cams, dict(st, schedule=s), dL=dL) for s in ("queue", "persistent", "tile_id")}
    for s in ("persistent", "tile_id"):
        np.testing.assert_array_equal(runs[s]["rgb"], runs["queue"]["rgb"])
        np.testing.assert_array_equal(runs[s]["T"], runs["queue"]["T"])
    # the two queue schedules take the same tasks: only the order of the FP64 totals differs
    G.assert_grads_close(runs["persistent"]["grads"], runs["queue"]["grads"], rtol=1e-6, floor=1e-9)
    if tile == 16:
        # at 16x16 the queue splits this small launch's lists into quadrant tasks, whose float
        # partial sums per entry round differently from whole tiles': the parity tolerance
        G.assert_grads_close(runs["tile_id"]["grads"], runs["queue"]["grads"])
    else:
        G.assert_grads_close(runs["tile_id"]["grads"], runs["queue"]["grads"], rtol=1e-6, floor=1e-9)
    # and the default schedule against the oracle
    ok = G.strict_pixels(fwd["margin"])
    assert np.abs(runs["queue"]["T"] - fwd["T"])[ok].max() <= G.RGB_ATOL
    ref = O.backward(sc, cams, st, dL, mode=32)
    G.assert_grads_close(runs["queue"]["grads"], ref)


def test_queue_is_longest_first_permutation():
    import torch
    sc, cams = _uneven_case()
    res = G.run_gpu(sc, cams, settings(schedule="persistent"), return_rast=True)
    rast = res["rast"]
    p = rast.plan
    tiles = int(p.tile_base[cams.n_views])
    q = rast.ws[p.off_queue + 64:p.off_queue + 64 + 4 * tiles].view(torch.int32).cpu().numpy()
    r = rast.ws[p.off_ranges:p.off_ranges + 8 * tiles].view(torch.int32).cpu().numpy().reshape(tiles, 2)
    np.testing.assert_array_equal(np.sort(q), np.arange(tiles))
    length = (r[:, 1] - r[:, 0])[q].astype(np.float64)
    # longest first, up to cost buckets 1/32 of an octave wide: no later entry is longer than
    # 33/32 of an earlier one (empty tiles last)
    later_max = np.maximum.accumulate(length[::-1])[::-1]
    assert (later_max[1:] <= length[:-1] * (33.0 / 32.0)).all()
    ctr = rast.ws[p.off_queue:p.off_queue + 16].view(torch.int32).cpu().numpy()
    np.testing.assert_array_equal(ctr, 0)  # left cleared by the persistent forward


def _long_list_case(opacity_scale):
    """Two 128x64 views inside a shell of 16k Gaussians: lists of about a thousand pairs per 16x16
    tile.  Scaling the opacities down (and so the footprints) keeps most pixels compositing to the
    end of their lists; at full opacity they stop early."""
    sc = scenes.sphere_scene(16000, 3, seed=87, r_range=(0.5, 1.5))
    sc.opacities[:] = sc.opacities * opacity_scale
    return sc, scenes.identity_cameras(128, 64, 2)


def expected_split_tiles(lengths):
    """Tiles the queue splits into quadrant tasks: lists in the cost bucket of the split length or
    above (buckets of 1/32 octave: exponent and top five mantissa bits of the float length), the
    split length being 1/4096 of all pairs, and at least 1024 pairs once there are 4096 tiles or
    more; at most max(1024, tiles / 8) tiles (all of them below 1024)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    tiles = len(lengths)

    def bucket(x):
        x = np.asarray(x, dtype=np.int64)
        b = 1 + ((x.astype(np.float32).view(np.uint32).astype(np.int64) - 0x3F800000) >> 18)
        return np.where(x == 0, 0, b)

    thr = max(1024 if tiles >= 4096 else 1, int(lengths.sum()) // 4096)
    cap = tiles if tiles < 1024 else max(1024, tiles // 8)
    return min(int((bucket(lengths) >= bucket(thr)).sum()), cap)


@pytest.mark.parametrize("footprint,opacity_scale", [("affine", 0.03), ("affine", 1.0), ("spherical", 0.03)])
def test_split_tiles(footprint, opacity_scale):
    """Under the queue schedules a launch of few tiles composites every non-empty 16x16 list as four
    single-quadrant tasks (forward and reverse): images bit-identical to whole-tile compositing in
    tile id order, 2D gradients and parameter gradients against the oracle."""
    import torch
    sc, cams = _long_list_case(opacity_scale)
    st = settings(tile=16, footprint=footprint)
    fwd = O.render(sc, cams, st, mode=32)
    dL = _masked_upstream(cams, fwd["margin"], seed=1083)
    runs = {s: G.run_gpu(sc, cams, dict(st, schedule=s), dL=dL, return_rast=True, split_bwd=True)
            for s in ("queue", "persistent", "tile_id")}
    for s, res in runs.items():
        rast = res["rast"]
        p = rast.plan
        tiles = int(p.tile_base[cams.n_views])
        r = rast.ws[p.off_ranges:p.off_ranges + 8 * tiles].view(torch.int32).cpu().numpy().reshape(tiles, 2)
        hdr = rast.ws[p.off_queue:p.off_queue + 64].view(torch.int32).cpu().numpy()
        split = expected_split_tiles(r[:, 1] - r[:, 0])
        assert split > 0
        assert hdr[4] == split  # counted by binning
        assert hdr[5] == (0 if s == "tile_id" else split)  # split by the forward
    base = runs["tile_id"]
    for s in ("queue", "persistent"):
        np.testing.assert_array_equal(runs[s]["rgb"], base["rgb"])
        np.testing.assert_array_equal(runs[s]["T"], base["T"])
        # a quadrant task sums its entries' float contributions over 64 pixels, a whole tile over
        # 256: the per-(entry, tile) partial sums round differently, so only the parity tolerance
        # holds between the two
        G.assert_grads_close(runs[s]["grads"], base["grads"])
    res = runs["queue"]
    ok = G.strict_pixels(fwd["margin"])
    assert np.abs(res["T"] - fwd["T"])[ok].max() <= G.RGB_ATOL
    okc = np.concatenate([np.tile(ok[o:o + w * h], 3) for o, w, h in _views(cams)])
    assert np.abs(res["rgb"] - fwd["rgb"])[okc].max() <= G.RGB_ATOL
    ref = O.backward(sc, cams, st, dL, mode=32, want_g2d=True)
    if footprint == "affine":
        ref2d = O.g2d_to_sigma(O.project(sc, cams, st), ref["g2d"])
        labels = ("u", "v", "S_uu", "S_uv", "S_vv", "opacity", "r", "g", "b")
        G.assert_grads_close({k: res["g2d"][..., j] for j, k in enumerate(labels)},
                             {k: ref2d[..., j] for j, k in enumerate(labels)}, names=labels)
        G.assert_grads_close(res["grads"], ref)
    else:
        # the spherical footprint's parity bar: the gradient tolerance plus the distance the float
        # evaluation of the exponent alone puts between a float renderer and the reference
        labels = ("mx", "my", "mz", "Sxx", "Sxy", "Sxz", "Syy", "Syz", "Szz", "opacity", "r", "g", "b")
        sl = G.float_exponent_slack(sc, cams, st, dL, ref)
        G.assert_grads_close({k: res["g2d"][..., j] for j, k in enumerate(labels)},
                             {k: ref["g2d_kernel"][..., j] for j, k in enumerate(labels)}, names=labels,
                             slack={k: sl["g2d"][..., j] for j, k in enumerate(labels)})
        G.assert_grads_close(res["grads"], ref, slack=sl)


def test_backward_refuses_a_stale_pair_list():
    """bin_sort between forward and backward: the reverse compositor accumulates nothing and sets
    the stale-forward flag; a forward on the new list clears the condition."""
    import torch
    from paper_2410_20686_amd import _odgs as B
    from paper_2410_20686_amd.rasterizer import Rasterizer
    name, sc, cams, st = CASES[1]
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    rast = Rasterizer(sc.n, sc.sh_degree, wh, st)
    t = G.to_gpu(sc, cams)
    rast.bin_checked(*t)
    rast.render_fwd()
    dL = torch.from_numpy(scenes.upstream_gradient(cams, 1090).astype(np.float32)).cuda()
    rast.bin(*t)  # new pair list, no forward
    rast.composite_bwd(dL)
    s = rast.status()
    assert s["flags"] & B.STATUS_STALE_FORWARD and s["fwd_gen"] != s["bin_gen"]
    assert not rast.g2d().abs().max().item()
    # preprocess resets the flags; the forward marks the list, and the backward runs
    rast.bin(*t)
    rast.render_fwd()
    rast.composite_bwd(dL)
    s = rast.status()
    assert not s["flags"] & B.STATUS_STALE_FORWARD and s["fwd_gen"] == s["bin_gen"]
    assert rast.g2d().abs().max().item() > 0


def test_status_counters_many_workgroups():
    """Past 512 preprocess workgroups the kept and culled counts are summed per workgroup and
    folded by a separate kernel (below, one atomic per workgroup): the totals are the oracle's."""
    sc = scenes.sphere_scene(140_001, 0, seed=93)  # 69 chunks of 2048 -> 552 workgroups
    cams = scenes.yaw_cameras(1, 256, 128, seed=93)
    st = settings()
    bad = np.array([3, 70_000, 140_000])
    sc.means[0, bad] = np.nan
    res = G.run_gpu(sc, cams, st)
    s = res["status"]
    rows = O.project(sc.subset(np.setdiff1d(np.arange(sc.n), bad)), cams, st)
    kept = int((rows[..., O.F_KEPT] > 0).sum())
    assert s["n_nonfinite"] == len(bad)
    assert s["n_visible"] == kept and s["n_culled"] == sc.n - kept
    assert s["n_pairs"] > 0


def test_culled_and_nonfinite_counters():
    """Gaussians with a NaN / infinite parameter or a zero quaternion are culled in every view
    and counted; the others render as the oracle renders the scene without them."""
    sc0 = scenes.sphere_scene(2003, 3, seed=91)
    cams = scenes.yaw_cameras(2, 256, 128, seed=91)
    st = settings()
    bad = np.array([5, 77, 400, 1001, 1500, 2002])
    sc = sc0.copy()
    sc.means[1, bad[0]] = np.nan
    sc.scales[2, bad[1]] = np.inf
    sc.quats[:, bad[2]] = 0.0
    sc.opacities[bad[3]] = np.nan
    sc.sh[17, bad[4]] = -np.inf
    sc.quats[3, bad[5]] = np.nan
    keep = np.setdiff1d(np.arange(sc.n), bad)
    good = sc0.subset(keep)
    res = G.run_gpu(sc, cams, st, return_rast=True)
    s = res["status"]
    rows = O.project(good, cams, st)
    kept = int((rows[..., O.F_KEPT] > 0).sum())
    assert s["n_nonfinite"] == len(bad)
    assert s["n_visible"] == kept and s["n_culled"] == cams.n_views * sc.n - kept
    okeys, ovals = O.keys(good, cams, st)
    keys, gauss = res["rast"].keys()
    np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint64), okeys)
    np.testing.assert_array_equal(gauss.cpu().numpy(), keep[ovals])
    ref = O.render(good, cams, st, mode=32)
    ok = G.strict_pixels(ref["margin"])
    assert np.abs(res["T"] - ref["T"])[ok].max() <= G.RGB_ATOL
