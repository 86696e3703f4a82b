"""Pins of the CPU oracle's compositing, binning and gradient.

Closed forms of Eq. alphablending, depth ordering, transmittance monotonicity, the yaw/seam
symmetry of Eq. equirec_proj, brute force vs tile lists, culling, and the analytic gradient
against FP64 central finite differences.  CPU only.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests._util import cams_from, image, make_scene, plane, rot_y, settings

SQ = 2 * np.sqrt(np.pi)  # DC coefficient per unit of colour (degree-0 basis constant 1/(2 sqrt(pi)))


def _alpha_at(row, o, px, py):
    a, b, c = row[O.F_CONIC:O.F_CONIC + 3]
    du, dv = px - row[O.F_U], py - row[O.F_V]
    return o * np.exp(-0.5 * (a * du * du + 2 * b * du * dv + c * dv * dv))


@pytest.mark.parametrize("k", [10, 40])
def test_stacked_identical_gaussians(k):
    """K identical co-located Gaussians: C = c (1 - (1-a)^n), T = (1-a)^n, where n stops before
    the transmittance would fall below 1e-4."""
    rgb = np.array([0.8, 0.4, 0.2])
    sc = make_scene([[0.0, 0.0, 5.0]] * k, [0.5, 0.5, 0.5], opac=0.3, sh=np.repeat(((rgb - 0.5) * SQ)[:, None], k, 1))
    cams = scenes.identity_cameras(256, 128)
    row = O.project(sc, cams, settings())[0, 0]
    x, y = 127, 63
    a = _alpha_at(row, 0.3, x + 0.5, y + 0.5)
    n = 0
    while n < k and (1 - a) ** (n + 1) >= 1e-4:
        n += 1
    pix = np.array([[0, x, y]], dtype=np.int32)
    r = O.render(sc, cams, settings(), mode=64, pix=pix)
    assert r["ncontrib"][0] == n
    np.testing.assert_allclose(r["T"][0], (1 - a) ** n, rtol=1e-12)
    np.testing.assert_allclose(r["rgb"][0], rgb * (1 - (1 - a) ** n), rtol=1e-12)
    # alpha-weighted depth: every contributor sits at radial depth 5
    np.testing.assert_allclose(r["depth"][0], 5.0 * (1 - (1 - a) ** n), rtol=1e-12)


def test_alpha_weighted_depth_of_two_layers():
    """Two Gaussians on one ray at radial depths 3 and 6: D = a1 3 + a2 (1 - a1) 6."""
    sc = make_scene([[0.0, 0.0, 6.0], [0.0, 0.0, 3.0]], [[0.4, 0.4, 0.4], [0.2, 0.2, 0.2]], opac=[0.7, 0.5])
    cams = scenes.identity_cameras(256, 128)
    rows = O.project(sc, cams, settings())[0]
    x, y = 127, 63
    a_far = _alpha_at(rows[0], 0.7, x + 0.5, y + 0.5)
    a_near = _alpha_at(rows[1], 0.5, x + 0.5, y + 0.5)
    r = O.render(sc, cams, settings(), mode=64, pix=np.array([[0, x, y]], dtype=np.int32))
    np.testing.assert_allclose(r["depth"][0], a_near * 3.0 + a_far * (1 - a_near) * 6.0, rtol=1e-12)
    np.testing.assert_allclose(r["T"][0], (1 - a_near) * (1 - a_far), rtol=1e-12)


def test_front_to_back_order_by_radial_depth():
    """Eq. alphablending is accumulated in depth order, whatever the storage order."""
    red = (np.array([1.0, 0.0, 0.0]) - 0.5) * SQ
    blue = (np.array([0.0, 0.0, 1.0]) - 0.5) * SQ
    means = [[0.0, 0.0, 6.0], [0.0, 0.0, 3.0]]      # far blue first, near red second
    sh = np.stack([blue, red], axis=1)
    sc = make_scene(means, [0.3, 0.3, 0.3], opac=[0.9, 0.7], sh=sh)
    cams = scenes.identity_cameras(256, 128)
    rows = O.project(sc, cams, settings(dilation=0.0))[0]
    pix = np.array([[0, 128, 64]], dtype=np.int32)
    r = O.render(sc, cams, settings(dilation=0.0), mode=64, pix=pix)
    a_far = _alpha_at(rows[0], 0.9, 128.5, 64.5)
    a_near = _alpha_at(rows[1], 0.7, 128.5, 64.5)
    expect = np.array([a_near, 0.0, a_far * (1 - a_near)])
    np.testing.assert_allclose(r["rgb"][0], expect, rtol=1e-12, atol=1e-15)
    sc_swapped = sc.subset([1, 0])
    r2 = O.render(sc_swapped, cams, settings(dilation=0.0), mode=64, pix=pix)
    np.testing.assert_array_equal(r2["rgb"], r["rgb"])


def test_transmittance_monotone_and_alpha_bounded():
    """Rendering growing depth-ordered prefixes never raises a pixel's transmittance; the
    accumulated alpha 1 - T stays in [0, 1] and the colour within [0, (1 - T) max rgb]."""
    sc, cams, st = scenes.config("cfg0", n=600)
    sc = sc.as_f64()
    depth = O.project(sc, cams, st)[0, :, O.F_DEPTH]
    order = np.argsort(depth, kind="stable")
    prev = None
    rgbmax = O.project(sc, cams, st)[0, :, O.F_RGB:O.F_RGB + 3].max()
    for k in (0, 50, 150, 300, 600):
        r = O.render(sc.subset(order[:k]), cams, st, mode=64)
        T = r["T"]
        assert np.all(T <= 1.0) and np.all(T >= 1e-4)
        assert np.all(r["rgb"] >= 0.0)
        img = r["rgb"].reshape(3, -1)
        assert np.all(img <= (1.0 - T)[None, :] * rgbmax + 1e-12)
        if prev is not None:
            assert np.all(T <= prev + 1e-15)
        prev = T


@pytest.mark.parametrize("k", [1, 7, 64, 128])
def test_yaw_rotation_is_circular_shift(k):
    """Yawing the camera by 2 pi k / W about its own y axis shifts the ERP image circularly by
    k pixels (Eq. equirec_proj is linear in the azimuth; the covariance is yaw invariant)."""
    W, H = 256, 128
    sc = scenes.sphere_scene(800, 3, seed=11).as_f64()
    c = np.array([0.1, -0.05, 0.2])
    R0 = rot_y(0.37)
    beta = 2 * np.pi * k / W
    R1 = rot_y(beta) @ R0
    cams = cams_from([R0, R1], [-R0 @ c, -R1 @ c], [[W, H], [W, H]])
    st = settings()
    r = O.render(sc, cams, st, mode=64)
    a, b = image(r["rgb"], cams, 0), image(r["rgb"], cams, 1)
    np.testing.assert_allclose(b, np.roll(a, -k, axis=2), atol=1e-9)
    np.testing.assert_allclose(plane(r["T"], cams, 1), np.roll(plane(r["T"], cams, 0), -k, axis=1), atol=1e-9)


def test_seam_straddlers_render_continuously():
    """Gaussians straddling the +-pi seam render exactly as the same Gaussians seen at the image
    centre after a half-turn yaw: both border columns carry them and nothing is cut."""
    W, H = 256, 128
    rng = np.random.default_rng(3)
    n = 60
    az = np.pi + rng.uniform(-0.05, 0.05, n)
    el = rng.uniform(-0.6, 0.6, n)
    r = rng.uniform(2, 4, n)
    means = np.stack([r * np.cos(el) * np.sin(az), -r * np.sin(el), r * np.cos(el) * np.cos(az)], axis=1)
    sc = make_scene(means, rng.uniform(0.02, 0.1, (n, 3)), opac=rng.uniform(0.3, 0.9, n),
                    sh=rng.uniform(-1.5, 1.5, (3, n)))
    cams = cams_from([np.eye(3), rot_y(np.pi)], [np.zeros(3), np.zeros(3)], [[W, H], [W, H]])
    res = O.render(sc, cams, settings(), mode=64)
    seam, centre = image(res["rgb"], cams, 0), image(res["rgb"], cams, 1)
    np.testing.assert_allclose(seam, np.roll(centre, W // 2, axis=2), atol=1e-9)
    assert seam[:, :, 0].sum() > 1.0 and seam[:, :, W - 1].sum() > 1.0


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tile_lists_render_identically_to_brute_force(tile):
    sc, _, st = scenes.config("cfg0", n=1500)
    cams = scenes.uneven_cameras(3, seed=2, sizes=((128, 64), (256, 128), (64, 32)))
    st = settings(tile=tile)
    a = O.render(sc, cams, st, mode=32, band=False)
    b = O.render(sc, cams, st, mode=32, band=True)
    for key in ("rgb", "T", "ncontrib", "sig"):
        np.testing.assert_array_equal(a[key], b[key])


def test_key_list_structure_and_coverage():
    """Keys are sorted (tile, depth) with ascending index on ties, carry each Gaussian's depth
    bits, list each footprint rectangle once, and every pixel where a Gaussian reaches
    alpha >= 1/255 lies in one of its tiles."""
    sc, cams, st = scenes.config("cfg0")
    rows = O.project(sc, cams, st)[0]
    keys, vals = O.keys(sc, cams, st)
    order = np.lexsort((vals, keys))
    np.testing.assert_array_equal(order, np.arange(len(keys)))
    np.testing.assert_array_equal(keys & 0xFFFFFFFF, rows[vals, O.F_DEPTH_BITS].astype(np.uint64))
    W, H, B = 256, 128, st["tile"]
    ntx = W // B
    counts = np.bincount(vals, minlength=sc.n)
    kept = rows[:, O.F_KEPT] > 0
    np.testing.assert_array_equal(counts[kept], (rows[kept, O.F_RECT + 1] * rows[kept, O.F_RECT + 3]).astype(int))
    assert np.all(counts[~kept] == 0)
    tiles_of = {}
    for k, v in zip((keys >> 32).astype(np.int64), vals):
        tiles_of.setdefault(int(v), set()).add(int(k))
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    tile_id = (py // B).astype(int) * ntx + (px // B).astype(int)
    for i in np.nonzero(kept)[0]:
        a, b, c = rows[i, O.F_CONIC:O.F_CONIC + 3]
        du = px - rows[i, O.F_U]
        du = np.where(du >= W / 2, du - W, np.where(du < -W / 2, du + W, du))
        dv = py - rows[i, O.F_V]
        power = -0.5 * (a * du * du + 2 * b * du * dv + c * dv * dv)
        hit = power >= rows[i, O.F_PMIN] - 1e-6
        need = set(np.unique(tile_id[hit]).tolist())
        assert need <= tiles_of.get(int(i), set()), i


def test_culling_rules():
    """Spherical-shell culling (Sec. 3.2), pole, opacity below 1/255 and non-finite inputs."""
    means = [[0, 0, 0.1], [0, 0, 2e4], [0, -3.0, 0], [0, 0, 3.0], [np.nan, 0, 3.0], [0, 0, 3.0], [0, 0, 3.0], [1, 0, 3]]
    quats = [[1, 0, 0, 0]] * 5 + [[0, 0, 0, 0]] + [[1, 0, 0, 0]] * 2
    opac = [0.5, 0.5, 0.5, 0.003, 0.5, 0.5, 0.5, 0.5]
    sh = np.zeros((3, 8))
    sh[0, 6] = np.nan
    sc = make_scene(means, [0.1, 0.1, 0.1], quats=quats, opac=opac, sh=sh)
    cams = scenes.identity_cameras(128, 64)
    rows = O.project(sc, cams, settings())[0]
    np.testing.assert_array_equal(rows[:, O.F_CULL].astype(int), [1, 1, 2, 3, 1, 4, 6, 0])
    keys, vals = O.keys(sc, cams, settings())
    assert set(vals.tolist()) == {7}
    r = O.render(sc.subset([0, 1, 2, 3, 4, 5, 6]), cams, settings(bg=(0.25, 0.5, 0.75)), mode=32)
    np.testing.assert_array_equal(r["T"], 1.0)
    np.testing.assert_array_equal(image(r["rgb"], cams, 0)[:, 10, 10], [0.25, 0.5, 0.75])


def test_empty_scene():
    sc = make_scene(np.zeros((0, 3)), np.zeros((0, 3)))
    cams = scenes.identity_cameras(64, 32)
    r = O.render(sc, cams, settings(bg=(0.1, 0.2, 0.3)), mode=32)
    np.testing.assert_array_equal(r["T"], 1.0)
    assert O.keys(sc, cams, settings())[0].size == 0


def _fd_scene():
    sc = scenes.sphere_scene(300, 3, seed=21).as_f64()
    cams = scenes.uneven_cameras(3, seed=5, sizes=((64, 32), (128, 64), (256, 128)))
    st = settings(bg=(0.1, 0.2, 0.3))
    return sc, cams, st


def test_backward_matches_central_finite_differences():
    """The analytic FP64 gradient equals FP64 central differences of the FP64 render over 64
    random parameters; parameters whose +-h renders take a different discrete decision (a
    contributor, the opacity clamp or the termination step) are redrawn."""
    sc, cams, st = _fd_scene()
    dL = scenes.upstream_gradient(cams, 77).astype(np.float64)
    g = O.backward(sc, cams, st, dL, mode=64)
    rng = np.random.default_rng(12)
    groups = [("means", 3), ("scales", 3), ("quats", 4), ("opacities", 1), ("sh", 48)]
    visible = np.nonzero(np.abs(g["opacities"]) > 0)[0]
    checked = 0
    tries = 0
    while checked < 64:
        tries += 1
        assert tries < 400
        name, rows = groups[checked % len(groups)]
        i = int(rng.choice(visible))
        c = int(rng.integers(0, rows))
        base = getattr(sc, name)
        x0 = base[i] if name == "opacities" else base[c, i]
        h = 1e-6 * max(1.0, abs(x0))

        def loss(delta):
            s = sc.copy()
            arr = getattr(s, name)
            if name == "opacities":
                arr[i] += delta
            else:
                arr[c, i] += delta
            r = O.render(s, cams, st, mode=64)
            return float(np.dot(r["rgb"], dL)), r["sig"]

        lp, sp = loss(h)
        lm, sm = loss(-h)
        if not np.array_equal(sp, sm):
            continue
        fd = (lp - lm) / (2 * h)
        an = g[name][i] if name == "opacities" else g[name][c, i]
        gmax = np.abs(g[name]).max()
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-7 * gmax, (name, i, c, fd, an)
        checked += 1


def test_fp32_and_fp64_modes_agree():
    """The float-decision compositor stays within 1e-5 of the double one on cfg0."""
    sc, cams, st = scenes.config("cfg0")
    a = O.render(sc, cams, st, mode=32)
    b = O.render(sc, cams, st, mode=64)
    ok = (a["margin"] > 1e-3) & (b["margin"] > 1e-3)
    okc = np.tile(ok, 3)
    assert np.abs(a["rgb"] - b["rgb"])[okc].max() < 1e-5


def test_backward_fd_uneven_16_views():
    """cfg4 shape (16 views of three sizes, Haar-random rotations, roaming scene): the analytic
    FP64 gradient equals FP64 central differences over 64 random parameters."""
    sc = scenes.roaming_scene(400, 3, seed=4, r_range=(2.0, 6.0)).as_f64()
    cams = scenes.uneven_cameras(16, seed=4, sizes=((64, 32), (128, 64), (256, 128)))
    st = settings(bg=(0.05, 0.1, 0.15))
    dL = scenes.upstream_gradient(cams, 1004).astype(np.float64)
    g = O.backward(sc, cams, st, dL, mode=64)
    rng = np.random.default_rng(44)
    groups = [("means", 3), ("scales", 3), ("quats", 4), ("opacities", 1), ("sh", 48)]
    visible = np.nonzero(np.abs(g["opacities"]) > 0)[0]
    checked = tries = 0
    while checked < 64:
        tries += 1
        assert tries < 400
        name, rows = groups[int(rng.integers(0, len(groups)))]
        i = int(rng.choice(visible))
        c = int(rng.integers(0, rows))
        base = getattr(sc, name)
        x0 = base[i] if name == "opacities" else base[c, i]
        h = 1e-6 * max(1.0, abs(x0))

        def loss(delta):
            s = sc.copy()
            arr = getattr(s, name)
            if name == "opacities":
                arr[i] += delta
            else:
                arr[c, i] += delta
            r = O.render(s, cams, st, mode=64)
            return float(np.dot(r["rgb"], dL)), r["sig"]

        lp, sp = loss(h)
        lm, sm = loss(-h)
        if not np.array_equal(sp, sm):
            continue
        fd = (lp - lm) / (2 * h)
        an = g[name][i] if name == "opacities" else g[name][c, i]
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-7 * np.abs(g[name]).max(), (name, i, c, fd, an)
        checked += 1


def test_projection_adjoint_in_covariance_terms():
    """The projection adjoint applied to the 2D gradients re-expressed w.r.t. the 2D covariance
    (-M G M with M the inverse covariance) reproduces the full backward: pins the conversion and
    the covariance-form outputs of the dual-number projection."""
    sc = scenes.roaming_scene(700, 3, seed=81, r_range=(2.0, 6.0)).as_f64()
    cams = scenes.uneven_cameras(2, seed=81, sizes=((128, 64), (256, 128)))
    st = settings(bg=(0.1, 0.0, 0.2))
    dL = scenes.upstream_gradient(cams, 1081).astype(np.float64)
    g = O.backward(sc, cams, st, dL, mode=64, want_g2d=True)
    rows = O.project(sc, cams, st)
    h = O.project_adjoint(sc, cams, st, O.g2d_to_sigma(rows, g["g2d"]))
    for k in ("means", "scales", "quats", "opacities", "sh"):
        np.testing.assert_allclose(h[k], g[k], rtol=1e-9, atol=1e-12 * np.abs(g[k]).max())


def test_band_backward_equals_brute_force():
    """The backward with tile-list candidates (band mode) reproduces the brute-force backward: the
    contributor lists are the same by construction (only summation order across threads differs)."""
    sc = scenes.sphere_scene(1500, 3, seed=61)
    cams = scenes.uneven_cameras(2, seed=61, sizes=((128, 64), (256, 128)))
    st = settings()
    dL = scenes.upstream_gradient(cams, 1061).astype(np.float64)
    a = O.backward(sc, cams, st, dL, mode=32, want_g2d=True)
    b = O.backward(sc, cams, st, dL, mode=32, want_g2d=True, band=True)
    for k in ("means", "scales", "quats", "opacities", "sh", "g2d"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-10, atol=1e-12 * np.abs(a[k]).max())


@pytest.mark.parametrize("footprint", ["affine", "spherical"])
def test_fp32_and_fp64_modes_agree_on_needles(footprint):
    """The float decision form (records rounded to float, exponent in the kernel's float form)
    renders the needle scene (axis ratios up to 800:1, poles, seam) within 5e-5 of the double
    definition wherever neither pass stops within 1e-3 of the termination threshold (measured:
    8e-6 affine, 3e-6 spherical)."""
    from tests.test_gpu_parity import _needle_scene
    sc = _needle_scene(n=1201, seed=62)
    cams = scenes.identity_cameras(256, 128)
    st = settings(dilation=0.1, footprint=footprint)
    a = O.render(sc, cams, st, mode=32)
    b = O.render(sc, cams, st, mode=64)
    ok = (a["margin"] > 1e-3) & (b["margin"] > 1e-3)
    okc = np.tile(ok, 3)
    assert ok.mean() > 0.9
    assert np.abs(a["rgb"] - b["rgb"])[okc].max() < 5e-5
