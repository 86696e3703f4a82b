"""Spherical footprint on the GPU (ODGS_FLAG_SPHERICAL) against the oracle: bit-exact key lists
from the cone rectangles, forward colours / transmittance / depth, and both backward stages (the
reverse compositor's 13 per-item values, the projection adjoint applied to them, end to end)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests import _gpu as G
from tests import test_gpu_parity as P
from tests._util import settings

pytestmark = pytest.mark.gpu

SPH = dict(footprint="spherical")


def _f32(sc):
    return scenes.Scene(*(np.ascontiguousarray(getattr(sc, f), dtype=np.float32)
                          for f in ("means", "scales", "quats", "opacities", "sh")), sc.sh_degree)


def _cases():
    from tests.test_oracle_spherical import _hard_scene
    cases = []
    sc = scenes.sphere_scene(3001, 3, seed=51)
    cams = scenes.uneven_cameras(3, seed=51, sizes=((128, 64), (256, 128), (512, 256)))
    cases.append(("sph_uneven3", sc, cams, settings(**SPH)))
    cases.append(("sph_hard", _f32(_hard_scene()), scenes.uneven_cameras(2, seed=52, sizes=((128, 64), (256, 128))),
                  settings(bg=(0.1, 0.2, 0.3), **SPH)))
    cases.append(("sph_needles", P._needle_scene(n=2001, seed=53), scenes.identity_cameras(512, 256),
                  settings(dilation=0.1, **SPH)))
    return cases


CASES = _cases()


@pytest.mark.parametrize("tile,binning", [(8, "auto"), (16, "direct"), (16, "coarse"), (32, "auto")])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_key_list_bit_exact(case, tile, binning):
    P.check_key_list(case, tile, binning)


@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_forward_matches_oracle(case, tile):
    name, sc, cams, st = case
    P.test_forward_matches_oracle((name, sc, cams, dict(st, tile=tile)))


def test_depth_output_matches_oracle():
    import torch
    name, sc, cams, st = CASES[0]
    res = G.run_gpu(sc, cams, st, return_rast=True)
    depth = torch.empty_like(torch.from_numpy(res["T"])).cuda()
    res["rast"].render_fwd(out_depth=depth)
    torch.cuda.synchronize()
    ref = O.render(sc, cams, st, mode=32)
    ok = G.strict_pixels(ref["margin"])
    got = depth.cpu().numpy()
    np.testing.assert_allclose(got[ok], ref["depth"][ok], rtol=1e-5, atol=1e-4)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_backward_matches_oracle(case):
    name, sc, cams, st = case
    fwd = O.render(sc, cams, st, mode=32)
    dL = P._masked_upstream(cams, fwd["margin"], seed=1050)
    res = G.run_gpu(sc, cams, st, dL=dL, split_bwd=True)
    ref = O.backward(sc, cams, st, dL, mode=32, want_g2d=True)
    labels = ("mx", "my", "mz", "Sxx", "Sxy", "Sxz", "Syy", "Syz", "Szz", "opacity", "r", "g", "b")
    g, r = res["g2d"], ref["g2d_kernel"]
    assert g.shape[-1] == 13
    # every tensor, needles included, at the gradient tolerance plus the per-element distance the
    # float evaluation of the exponent alone puts between a float renderer and the reference
    sl = G.float_exponent_slack(sc, cams, st, dL, ref)
    G.assert_grads_close({k: g[..., j] for j, k in enumerate(labels)},
                         {k: r[..., j] for j, k in enumerate(labels)}, names=labels,
                         slack={k: sl["g2d"][..., j] for j, k in enumerate(labels)})
    adj = O.project_adjoint(sc, cams, st, res["g2d"].astype(np.float64))
    G.assert_grads_close(res["grads"], adj, rtol=1e-5, floor=1e-7)
    rep = G.assert_grads_close(res["grads"], ref, slack=sl)
    print(name, rep)


@pytest.mark.parametrize("tile", [16, 32])
def test_backward_after_depth_forward(tile):
    """The depth forward variant also hands its quadrant masks to the backward."""
    name, sc, cams, st = CASES[0]
    got, ref = P.backward_after_forward_variant(sc, cams, dict(st, tile=tile), "depth", seed=1051)
    G.assert_grads_close(got, ref)


@pytest.mark.parametrize("tile", [8, 32])
def test_backward_other_tiles(tile):
    """Tile 8: one wavefront per tile; tile 32: sixteen wavefronts sharing one set of LDS
    accumulators (atomics) instead of a slot set per wavefront."""
    name, sc, cams, st = CASES[0]
    test_backward_matches_oracle((name, sc, cams, dict(st, tile=tile)))
