"""Parity at the workloads' full sizes, in the launch configuration the benchmark times (all
views batched, tile 16, default LDS batches): bit-exact key lists, colours at sampled pixels against the
brute-force oracle, and every parameter gradient under an upstream gradient that is non-zero
only on the sampled pixels (so the oracle evaluates those pixels only, while the GPU runs the
whole image)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _view_offsets(cams):
    off = [0]
    for w, h in cams.wh:
        off.append(off[-1] + int(w) * int(h))
    return off


def _sampled(res, cams, pix):
    off = _view_offsets(cams)
    rgb = np.zeros((len(pix), 3))
    T = np.zeros(len(pix))
    for k, (v, x, y) in enumerate(pix):
        w, h = int(cams.wh[v, 0]), int(cams.wh[v, 1])
        p = int(y) * w + int(x)
        for c in range(3):
            rgb[k, c] = res["rgb"][3 * off[v] + c * w * h + p]
        T[k] = res["T"][off[v] + p]
    return rgb, T


def _check(sc, cams, st, n_pix, seed, key_views=None):
    """slack: for the spherical footprint, the gradient bound adds the per-element effect of the
    float exponent (tests/_gpu.float_exponent_slack)."""
    dL, pix = scenes.sparse_upstream_gradient(cams, seed, n_pix)
    ref = O.render(sc, cams, st, mode=32, pix=pix)
    ok = G.strict_pixels(ref["margin"])
    # upstream gradient only on strictly comparable sampled pixels
    off = _view_offsets(cams)
    gpix = np.zeros((len(pix), 3))
    for k, (v, x, y) in enumerate(pix):
        w, h = int(cams.wh[v, 0]), int(cams.wh[v, 1])
        p = int(y) * w + int(x)
        for c in range(3):
            i = 3 * off[v] + c * w * h + p
            if not ok[k]:
                dL[i] = 0.0
            gpix[k, c] = dL[i]
    res = G.run_gpu(sc, cams, st, dL=dL, return_rast=key_views is not None)
    rgb, T = _sampled(res, cams, pix)
    assert np.abs(rgb - ref["rgb"])[ok].max() <= G.RGB_ATOL
    assert np.abs(T - ref["T"])[ok].max() <= G.RGB_ATOL
    assert (~ok).sum() <= max(2, 0.01 * len(pix))
    gref = O.backward(sc, cams, st, gpix, mode=32, pix=pix)
    slack = G.float_exponent_slack(sc, cams, st, gpix, gref, pix=pix) if O.spherical(st) else None
    G.assert_grads_close(res["grads"], gref, slack=slack)
    if key_views is not None:
        sub = scenes.Cameras(np.ascontiguousarray(cams.cams[:key_views]), np.ascontiguousarray(cams.wh[:key_views]))
        okeys, ovals = O.keys(sc, sub, st)
        keys, gauss = res["rast"].keys()
        keys = keys.cpu().numpy().view(np.uint64)
        gauss = gauss.cpu().numpy().astype(np.uint32)
        plan = res["rast"].plan
        sel = (keys >> np.uint64(32)) < np.uint64(plan.tile_base[key_views])
        np.testing.assert_array_equal(keys[sel], okeys)
        np.testing.assert_array_equal(gauss[sel], ovals)
        if key_views == cams.n_views:
            assert res["status"]["n_pairs"] == len(okeys)
    return res


def test_cfg2_roaming_500k_4096x2048():
    sc, cams, st = scenes.config("cfg2")
    _check(sc, cams, st, n_pix=768, seed=1002, key_views=1)


def test_M_500k_8x2048x1024_batched():
    sc, cams, st = scenes.config("M")
    _check(sc, cams, st, n_pix=96, seed=1005, key_views=cams.n_views)


def test_M_single_view_split_tiles():
    """One view of M alone (the per-view launch): its longest lists are split into quadrant tasks
    while the rest stay whole tiles, in one forward and one reverse launch."""
    import torch
    from tests.test_gpu_sched_status import expected_split_tiles
    sc, cams, st = scenes.config("M")
    cams = cams.view(0)
    res = _check(sc, cams, st, n_pix=256, seed=1025, key_views=1)
    rast = res["rast"]
    p = rast.plan
    tiles = int(p.tile_base[1])
    r = rast.ws[p.off_ranges:p.off_ranges + 8 * tiles].view(torch.int32).cpu().numpy().reshape(tiles, 2)
    hdr = rast.ws[p.off_queue:p.off_queue + 64].view(torch.int32).cpu().numpy()
    split = expected_split_tiles(r[:, 1] - r[:, 0])
    assert 0 < split < tiles and hdr[4] == split and hdr[5] == split


def test_M_spherical_footprint_batched():
    """The spherical footprint at the benchmark's workload M: every view's key list bit-exact,
    sampled colours, and every parameter gradient."""
    sc, cams, st = scenes.config("M")
    _check(sc, cams, dict(st, footprint="spherical"), n_pix=48, seed=1015, key_views=cams.n_views)


def test_cfg3_1M_8x2048x1024_batched():
    sc, cams, st = scenes.config("cfg3")
    _check(sc, cams, st, n_pix=64, seed=1003, key_views=cams.n_views)


def test_cfg1_100k_2048x1024():
    sc, cams, st = scenes.config("cfg1")
    _check(sc, cams, st, n_pix=512, seed=1001, key_views=1)


def test_cfg4_16_uneven_views_autotuned():
    """16 views of three resolutions with Haar-random rotations: tile edge and batch chosen by the
    autotuner on this device, then parity in that configuration."""
    import torch
    from paper_2410_20686_amd import autotune
    sc, cams, st = scenes.config("cfg4")
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    t = G.to_gpu(sc, cams)
    dL = torch.from_numpy(scenes.upstream_gradient(cams, 1004)).cuda()
    best = autotune.tune(t[:5], t[5], dL, sc.sh_degree, wh, st, reps=3, cache=None, log=print)
    assert best["tile"] in autotune.TILES
    assert best["batch"] in autotune.BATCHES[best["tile"]] and best["batch_bwd"] in autotune.BATCHES[best["tile"]]
    assert len(best["table"]) == len(autotune.TILES)
    del t, dL
    torch.cuda.empty_cache()
    _check(sc, cams, dict(st, tile=best["tile"], batch=best["batch"], batch_bwd=best["batch_bwd"]), n_pix=48,
           seed=1004, key_views=cams.n_views)
