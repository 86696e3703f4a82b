"""The differentiable front end: ``rasterizer.render`` as a ``torch.autograd.Function``, with
``.backward()`` through PyTorch's autograd, against the oracle; and its refusal to run a
backward on a workspace that another forward or binning has since overwritten."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import _gpu as G
from tests.test_gpu_parity import CASES, _masked_upstream

pytestmark = pytest.mark.gpu


def _setup(case):
    import torch
    from paper_2410_20686_amd.rasterizer import Rasterizer
    name, sc, cams, st = case
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    rast = Rasterizer(sc.n, sc.sh_degree, wh, st)
    t = G.to_gpu(sc, cams)
    params = [x.clone().requires_grad_(True) for x in t[:5]]
    return sc, cams, st, rast, params, t[5], torch


@pytest.mark.parametrize("case", CASES[1:3], ids=[c[0] for c in CASES[1:3]])
def test_autograd_backward_matches_oracle(case):
    from paper_2410_20686_amd.rasterizer import render
    sc, cams, st, rast, params, cams_t, torch = _setup(case)
    fwd = O.render(sc, cams, st, mode=32)
    dL = _masked_upstream(cams, fwd["margin"], seed=1210)
    rgb, T = render(*params, cams_t, rast)
    assert rgb.requires_grad and not T.requires_grad
    loss = (rgb * torch.from_numpy(dL.astype(np.float32)).cuda()).sum()
    loss.backward()
    ok = G.strict_pixels(fwd["margin"])
    assert np.abs(T.detach().cpu().numpy() - fwd["T"])[ok].max() <= G.RGB_ATOL
    ref = O.backward(sc, cams, st, dL, mode=32)
    names = ("means", "scales", "quats", "opacities", "sh")
    G.assert_grads_close({k: p.grad.cpu().numpy() for k, p in zip(names, params)}, ref)


def test_autograd_refuses_overwritten_workspace():
    from paper_2410_20686_amd.rasterizer import render
    sc, cams, st, rast, params, cams_t, torch = _setup(CASES[1])
    rgb1, _ = render(*params, cams_t, rast)
    rgb2, _ = render(*params, cams_t, rast)  # a second forward on the same workspace
    with pytest.raises(RuntimeError, match="another forward"):
        rgb1.sum().backward()
    rgb2.sum().backward()  # the latest forward still differentiates
    assert all(p.grad is not None for p in params)
    rgb3, _ = render(*params, cams_t, rast)
    rast.bin(*[p.detach() for p in params], cams_t)  # binning alone also replaces the lists
    with pytest.raises(RuntimeError, match="another forward"):
        rgb3.sum().backward()
