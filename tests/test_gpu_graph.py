"""HIP-graph capture of the whole fwd+bwd step: every replay matches an eager step, with eager
work and synchronisation between replays, and replays pick up new camera poses written in
place into the device pose tensor."""
import numpy as np
import pytest

from paper_2410_20686_amd import scenes
from tests import _gpu as G
from tests._util import settings

pytestmark = pytest.mark.gpu


def _setup(**kw):
    import torch
    from paper_2410_20686_amd.rasterizer import Rasterizer, TrainStep
    sc = scenes.roaming_scene(6007, 3, seed=51)
    cams = scenes.uneven_cameras(3, seed=51, sizes=((128, 64), (256, 128), (512, 256)))
    t = G.to_gpu(sc, cams)
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    rast = Rasterizer(sc.n, 3, wh, settings(**kw), pair_capacity=8 * sc.n * len(wh))
    dL = torch.from_numpy(scenes.upstream_gradient(cams, 1051)).cuda()
    return sc, cams, t, rast, TrainStep(rast, t[:5], t[5], dL)


def _snapshot(step):
    import torch
    torch.cuda.synchronize()
    return step.rgb.clone(), tuple(g.clone() for g in step.grads)


def _compare(a, b):
    """Images bit-identical; gradients equal up to the order in which per-tile sums reach the
    FP64 accumulators, which differs from run to run (relative 1e-4 plus 1e-5 of the tensor's
    largest magnitude: a loose bound for a difference at double rounding)."""
    import torch
    assert torch.equal(a[0], b[0])
    names = ("means", "scales", "quats", "opacities", "sh")
    G.assert_grads_close({k: g.cpu().numpy() for k, g in zip(names, a[1])},
                         {k: g.cpu().numpy() for k, g in zip(names, b[1])}, rtol=1e-4, floor=1e-5)


@pytest.mark.parametrize("footprint", ["affine", "spherical"])
def test_graph_replays_match_eager(footprint):
    import torch
    sc, cams, t, rast, step = _setup(footprint=footprint)
    step.run()
    ref = _snapshot(step)
    step.capture()
    other = step.rgb.new_zeros(1000)
    for k in range(3):
        step.rgb.zero_()
        step.replay()
        _compare(_snapshot(step), ref)
        other += torch.randn_like(other)  # unrelated eager work between replays
        torch.cuda.synchronize()
    st = rast.status()
    assert st["flags"] == 0 and st["n_pairs"] > 0


def test_graph_replay_uses_new_poses():
    import torch
    sc, cams, t, rast, step = _setup()
    step.capture()
    # new poses, same view sizes (the plan fixes the sizes; only poses live in device memory)
    new = scenes.Cameras(scenes.uneven_cameras(3, seed=99).cams, cams.wh.copy())
    step.cams.copy_(torch.from_numpy(new.cams).cuda())
    step.replay()
    got = _snapshot(step)
    assert not (rast.status()["flags"] & 1)
    step.run()  # eager with the same (new) poses
    _compare(got, _snapshot(step))
    ref = G.run_gpu(sc, new, settings())
    assert np.array_equal(got[0].cpu().numpy(), ref["rgb"])


def test_graph_accumulates_densification_statistics():
    """The statistics accumulate once per replay (counts exactly, sums up to atomics order)."""
    import torch
    from paper_2410_20686_amd.densify import DensifyStats
    from paper_2410_20686_amd.rasterizer import TrainStep
    sc, cams, t, rast, step0 = _setup()
    stats = DensifyStats(sc.n)
    step = TrainStep(rast, t[:5], t[5], step0.dL, stats=stats)
    step.run()
    torch.cuda.synchronize()
    one = (stats.grad_sum.clone(), stats.tau_sum.clone(), stats.count.clone())
    assert int(one[2].sum()) > 0
    stats.reset()
    step.capture()     # one eager run on the capture stream, then the recording
    stats.reset()
    for k in range(1, 4):
        step.replay()
        torch.cuda.synchronize()
        assert torch.equal(stats.count, k * one[2])
        torch.testing.assert_close(stats.tau_sum, k * one[1], rtol=1e-6, atol=0)
        torch.testing.assert_close(stats.grad_sum, k * one[0], rtol=1e-4, atol=1e-5 * float(one[0].max()))


@pytest.mark.parametrize("footprint", ["affine", "spherical"])
def test_graph_replay_matches_oracle(footprint):
    """A replayed graph step (third replay, eager work in between) against the oracle: images on
    every strictly comparable pixel and all five parameter gradients."""
    import torch
    from oracle import oracle as O
    from paper_2410_20686_amd.rasterizer import Rasterizer, TrainStep
    from tests.test_gpu_parity import _masked_upstream
    sc = scenes.roaming_scene(4001, 3, seed=52)
    cams = scenes.uneven_cameras(3, seed=52, sizes=((128, 64), (256, 128), (512, 256)))
    st = settings(footprint=footprint)
    fwd = O.render(sc, cams, st, mode=32)
    dL = _masked_upstream(cams, fwd["margin"], seed=1052)
    t = G.to_gpu(sc, cams)
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    rast = Rasterizer(sc.n, 3, wh, st, pair_capacity=8 * sc.n * len(wh))
    step = TrainStep(rast, t[:5], t[5], torch.from_numpy(dL.astype(np.float32)).cuda())
    step.capture()
    other = step.rgb.new_zeros(1000)
    for _ in range(3):
        step.rgb.zero_()
        for g in step.grads:
            g.zero_()
        step.replay()
        other += torch.randn_like(other)
        torch.cuda.synchronize()
    assert rast.status()["flags"] == 0
    ok = G.strict_pixels(fwd["margin"])
    off, okc = 0, []
    for w, h in wh:
        okc.append(np.tile(ok[off:off + w * h], 3))
        off += w * h
    okc = np.concatenate(okc)
    assert np.abs(step.rgb.cpu().numpy() - fwd["rgb"])[okc].max() <= G.RGB_ATOL
    ref = O.backward(sc, cams, st, dL, mode=32)
    names = ("means", "scales", "quats", "opacities", "sh")
    G.assert_grads_close({k: g.cpu().numpy() for k, g in zip(names, step.grads)}, ref)
