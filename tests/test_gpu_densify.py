"""Parity of the densification kernels (statistics gathered by the reverse projection stage, and
the clone / split / prune step) with the oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import densify as OD
from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests import _gpu as G
from tests._util import settings

pytestmark = pytest.mark.gpu


def _stats_case(name):
    if name == "uneven3":
        sc = scenes.sphere_scene(3001, 3, seed=51)
        cams = scenes.uneven_cameras(3, seed=51, sizes=((128, 64), (256, 128), (512, 256)))
        return sc, cams, settings()
    sc = scenes.roaming_scene(4099, 3, seed=52)
    return sc, scenes.yaw_cameras(2, 512, 256, seed=52), settings(bg=(0.2, 0.1, 0.05))


def _masked_upstream(cams, margin, seed):
    dL = scenes.upstream_gradient(cams, seed).astype(np.float64)
    ok = G.strict_pixels(margin)
    parts, base, off = [], 0, 0
    for w, h in cams.wh:
        w, h = int(w), int(h)
        m = np.tile(ok[off:off + w * h], 3)
        parts.append(np.where(m, dL[base:base + 3 * w * h], 0.0))
        base += 3 * w * h
        off += w * h
    return np.concatenate(parts)


@pytest.mark.parametrize("name", ["uneven3", "roam_yaw2"])
def test_statistics_match_oracle(name):
    import torch
    from paper_2410_20686_amd.densify import DensifyStats
    from paper_2410_20686_amd.rasterizer import Rasterizer
    sc, cams, st = _stats_case(name)
    fwd = O.render(sc, cams, st, mode=32)
    dL = _masked_upstream(cams, fwd["margin"], seed=1050)
    gs, ts, cnt = OD.stats(sc, cams, st, dL, mode=32)
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    rast = Rasterizer(sc.n, sc.sh_degree, wh, st)
    t = G.to_gpu(sc, cams)
    stats = DensifyStats(sc.n)
    dLg = torch.from_numpy(dL.astype(np.float32)).cuda()
    for rep in (1, 2):  # accumulates over steps
        rast.bin_checked(*t)
        rast.render_fwd()
        rast.render_bwd(*t, dLg, stats=stats)
        torch.cuda.synchronize()
        c = stats.count.cpu().numpy()
        np.testing.assert_array_equal(c, rep * cnt)
        np.testing.assert_allclose(stats.tau_sum.cpu().numpy(), rep * ts, rtol=2e-6, atol=1e-12)
        g = stats.grad_sum.cpu().numpy().astype(np.float64)
        lim = 1e-3 * rep * gs + 1e-6 * rep * gs.max()
        bad = np.abs(g - rep * gs) > lim
        assert not bad.any(), (name, rep, bad.sum(), g[bad][:3], rep * gs[bad][:3])
    stats.reset()
    torch.cuda.synchronize()
    assert int(stats.count.abs().sum()) == 0


def _random_densify_inputs(n, seed, extent):
    rng = np.random.default_rng(seed)
    f = np.float32
    means = rng.uniform(-10, 10, (3, n)).astype(f)
    big = f(1e-3) * f(extent)
    scales = (big * rng.uniform(0.3, 3.0, (3, n))).astype(f)
    scales[rng.integers(0, 3, n // 50), rng.integers(0, n, n // 50)] = big   # exactly on the boundary
    quats = rng.standard_normal((4, n)).astype(f)
    opac = rng.uniform(0.0, 0.05, n).astype(f)
    opac[: n // 100] = f(0.005)                                              # exactly at min_opacity
    sh = rng.standard_normal((48, n)).astype(f)
    count = rng.integers(0, 4, n).astype(np.int32)
    tau = (count * rng.uniform(2e-5, 1e-4, n)).astype(f)
    grad = (tau * rng.uniform(0.5, 1.5, n)).astype(f)
    eq = rng.choice(n, n // 40, replace=False)
    grad[eq] = tau[eq]                                                       # exactly at the threshold
    noise = rng.standard_normal((2, 3, n)).astype(f)
    return means, scales, quats, opac, sh, grad, tau, count, noise


def _gpu_densify(arrs, extent, max_scale_frac=0.0):
    import torch
    from paper_2410_20686_amd.densify import DensifyStats, densify
    means, scales, quats, opac, sh, grad, tau, count, noise = arrs
    n = means.shape[1]
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    stats = DensifyStats(n)
    stats.grad_sum.copy_(T(grad))
    stats.tau_sum.copy_(T(tau))
    stats.count.copy_(T(count))
    params = tuple(T(a) for a in (means, scales, quats, opac, sh))
    new, src, counts = densify(params, stats, T(noise), extent, 3, max_scale_frac=max_scale_frac)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in new], src.cpu().numpy(), counts


@pytest.mark.parametrize("n,frac", [(100_003, 0.0), (100_003, 0.002), (257, 0.0), (1, 0.0)])
def test_densify_matches_oracle(n, frac):
    extent = 37.5
    arrs = _random_densify_inputs(n, 60 + n % 7, extent)
    ref = OD.densify(*arrs, extent=extent, max_scale_frac=frac)
    (m, s, q, o, sh), src, counts = _gpu_densify(arrs, extent, frac)
    assert counts == ref["counts"]
    np.testing.assert_array_equal(src, ref["src"])
    np.testing.assert_array_equal(q, ref["quats"])
    np.testing.assert_array_equal(o, ref["opacities"])
    np.testing.assert_array_equal(sh, ref["sh"])
    np.testing.assert_array_equal(s, ref["scales"])          # copies and s / 1.6 (correctly rounded)
    k = counts[0] + counts[1]
    np.testing.assert_array_equal(m[:, :k], ref["means"][:, :k])
    # children: m + R (s * xi), FP32 on the device vs FP64 rounded once
    mag = np.abs(arrs[0]).max() + 4 * np.abs(arrs[1]).max() * 5
    np.testing.assert_allclose(m[:, k:], ref["means"][:, k:], rtol=0, atol=4e-7 * mag)


def test_densify_empty():
    arrs = _random_densify_inputs(0, 1, 1.0)
    (m, s, q, o, sh), src, counts = _gpu_densify(arrs, 1.0)
    assert counts == (0, 0, 0, 0) and src.size == 0


def test_statistics_then_densify_end_to_end():
    """Statistics from a GPU backward, then the step on the GPU vs the oracle's step on the same
    statistics (the decisions are FP32 comparisons of those inputs, so identical)."""
    import torch
    from paper_2410_20686_amd.densify import DensifyStats, densify
    from paper_2410_20686_amd.rasterizer import Rasterizer
    sc, cams, st = scenes.config("cfg0")
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    rast = Rasterizer(sc.n, sc.sh_degree, wh, st)
    t = G.to_gpu(sc, cams)
    stats = DensifyStats(sc.n)
    dL = torch.from_numpy(scenes.upstream_gradient(cams, 1000) * np.float32(1e-3)).cuda()
    rast.bin_checked(*t)
    rast.render_fwd()
    rast.render_bwd(*t, dL, stats=stats)
    noise = torch.from_numpy(np.random.default_rng(9).standard_normal((2, 3, sc.n)).astype(np.float32)).cuda()
    new, src, counts = densify(tuple(t[:5]), stats, noise, 100.0, sc.sh_degree)
    torch.cuda.synchronize()
    host = lambda x: x.cpu().numpy()
    ref = OD.densify(*(host(x) for x in t[:5]), host(stats.grad_sum), host(stats.tau_sum), host(stats.count),
                     host(noise), extent=100.0)
    assert counts == ref["counts"]
    assert counts[1] + counts[2] > 0, counts   # the case exercises clones and splits
    np.testing.assert_array_equal(host(src), ref["src"])
    np.testing.assert_array_equal(host(new[1]), ref["scales"])
