"""Perspective (pinhole) views on the GPU, alone and mixed with ERP views in one batch: records,
bit-exact key lists, forward and backward against the oracle (the same checks as the ERP cases)."""
import numpy as np
import pytest

from paper_2410_20686_amd import scenes
from tests import test_gpu_parity as P
from tests._util import settings

pytestmark = pytest.mark.gpu


def _cubemap_case():
    sc = scenes.sphere_scene(3001, 3, seed=61)
    faces = scenes.cubemap_cameras(64, centre=(0.2, -0.1, 0.3))
    erp = scenes.yaw_cameras(1, 256, 128, seed=61)
    cams = scenes.Cameras(np.concatenate([faces.cams, erp.cams]), np.concatenate([faces.wh, erp.wh]))
    st = settings(pinhole={v: (32.0, 32.0, 32.0, 32.0) for v in range(6)})
    return ("cubemap_plus_erp", sc, cams, st)


def _wide_case():
    """One off-centre pinhole view with unequal focal lengths, many Gaussians crossing its edges."""
    sc = scenes.roaming_scene(4001, 3, seed=62, r_range=(2.0, 8.0))
    cams = scenes.yaw_cameras(1, 192, 128, seed=62)
    st = settings(pinhole={0: (90.0, 70.0, 100.0, 60.0)}, bg=(0.1, 0.2, 0.3))
    return ("pinhole_wide", sc, cams, st)


CASES = [_cubemap_case(), _wide_case()]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pinhole_records(case):
    P.test_records_match_oracle(case)


@pytest.mark.parametrize("tile,binning", [(8, "auto"), (16, "direct"), (16, "coarse"), (32, "auto")])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pinhole_key_list_bit_exact(case, tile, binning):
    P.check_key_list(case, tile, binning)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pinhole_forward(case):
    P.test_forward_matches_oracle(case)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pinhole_backward(case):
    P.test_backward_matches_oracle(case)
