"""Pins of the densification oracle (Sec. 3.3 threshold, 3DGS clone / split / prune) against
closed forms, finite differences of the rendered loss under rigid motions of one Gaussian, the
key list, and a worked example whose expected output is written out by hand."""
import numpy as np

from oracle import densify as D
from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests._util import cams_from, make_scene, settings

TMIN, TMAX = D.TAU_MIN, D.TAU_MAX


def test_threshold_closed_forms():
    """Equator: tau_min; elevation +-60 deg: the midpoint; camera raised so the elevation is
    -45 deg: tau_min + (1 - 1/sqrt 2)(tau_max - tau_min).  Two views add up."""
    r = 3.0
    s60, c60 = np.sin(np.pi / 3), np.cos(np.pi / 3)
    means = [[0, 0, r], [0, -r * s60, r * c60], [r * c60, r * s60, 0.0]]
    sc = make_scene(means, [0.05, 0.05, 0.05], opac=0.9)
    cams = cams_from([np.eye(3)], [np.zeros(3)], [(256, 128)])
    dL = scenes.upstream_gradient(cams, 5)
    g, t, c = D.stats(sc, cams, settings(), dL, mode=64)
    np.testing.assert_array_equal(c, [1, 1, 1])
    np.testing.assert_allclose(t, [TMIN, 0.5 * (TMIN + TMAX), 0.5 * (TMIN + TMAX)], rtol=1e-12)
    # second view: camera shifted so that mu = m + (0, r, 0) -> first Gaussian at elevation -45 deg
    cams2 = cams_from([np.eye(3), np.eye(3)], [np.zeros(3), np.array([0.0, r, 0.0])], [(256, 128), (256, 128)])
    dL2 = scenes.upstream_gradient(cams2, 6)
    g2, t2, c2 = D.stats(sc, cams2, settings(), dL2, mode=64)
    assert c2[0] == 2
    np.testing.assert_allclose(t2[0], TMIN + TMIN + (1 - np.sqrt(0.5)) * (TMAX - TMIN), rtol=1e-12)


def _rotate_about_camera(m, axis, angle):
    """Rotate point m about the camera's y axis (yaw) or about the horizontal axis through the
    camera perpendicular to m's azimuth (elevation), by ``angle`` (identity camera)."""
    if axis == "yaw":
        c, s = np.cos(angle), np.sin(angle)
        return np.array([m[0] * c + m[2] * s, m[1], -m[0] * s + m[2] * c])
    r = np.linalg.norm(m)
    rho = np.hypot(m[0], m[2])
    th = np.arctan2(-m[1], rho) + angle
    phi = np.arctan2(m[0], m[2])
    return r * np.array([np.cos(th) * np.sin(phi), -np.sin(th), np.cos(th) * np.cos(phi)])


def test_position_gradient_statistic_by_finite_differences():
    """For isotropic SH0 Gaussians on the equator, a yaw of the mean by d moves u by W d / 2pi
    and leaves everything else unchanged; an elevation change moves v by -H d / pi and changes
    the 2D covariance only at second order (which central differences cancel).  So central
    differences of the loss give dL/du and dL/dv, and from them the statistic's value."""
    rng = np.random.default_rng(70)
    W, H = 256, 128
    n_t = 6
    az = rng.uniform(-3.0, 3.0, n_t)
    r = rng.uniform(2.0, 4.0, n_t)
    tm = np.stack([r * np.sin(az), np.zeros(n_t), r * np.cos(az)], axis=1)
    # occluders and background Gaussians (anisotropic, anywhere)
    n_o = 60
    d = rng.standard_normal((n_o, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    om = d * rng.uniform(1.5, 5.0, (n_o, 1))
    om[:20, 1] *= 0.1
    means = np.concatenate([tm, om])
    scales = np.concatenate([np.repeat(rng.uniform(0.05, 0.15, (n_t, 1)), 3, axis=1),
                             np.exp(rng.uniform(np.log(0.02), np.log(0.2), (n_o, 3)))])
    q = rng.standard_normal((n_t + n_o, 4))
    opac = rng.uniform(0.3, 0.9, n_t + n_o)
    sh = rng.uniform(-1.5, 1.5, (3, n_t + n_o))
    sc = make_scene(means, scales, quats=q, opac=opac, sh=sh)
    cams = cams_from([np.eye(3)], [np.zeros(3)], [(W, H)])
    st = settings(bg=(0.1, 0.2, 0.3))
    dL = scenes.upstream_gradient(cams, 71).astype(np.float64)
    gs, ts, cnt = D.stats(sc, cams, st, dL, mode=64)
    checked = 0
    for i in range(n_t):
        fd = {}
        for axis in ("yaw", "elev"):
            h = 1e-6

            def loss(a):
                s = sc.copy()
                s.means[:, i] = _rotate_about_camera(sc.means[:, i], axis, a)
                res = O.render(s, cams, st, mode=64)
                return float(np.dot(res["rgb"], dL)), res["sig"]

            lp, sp = loss(h)
            lm, sm = loss(-h)
            fd[axis] = (lp - lm) / (2 * h) if np.array_equal(sp, sm) else None
        if fd["yaw"] is None or fd["elev"] is None or cnt[i] == 0:
            continue
        du = fd["yaw"] * 2 * np.pi / W     # dL/du
        dv = -fd["elev"] * np.pi / H       # dL/dv
        expect = np.hypot(du * W / 2, dv * H / 2)
        assert abs(gs[i] - expect) <= 1e-5 * expect + 1e-9, (i, gs[i], expect)
        checked += 1
    assert checked >= 4


def test_visibility_count_matches_key_list():
    sc = scenes.roaming_scene(3000, 1, seed=72)
    cams = scenes.uneven_cameras(3, seed=72, sizes=((128, 64), (256, 128)))
    st = settings()
    keys, vals = O.keys(sc, cams, st)
    dL = scenes.upstream_gradient(cams, 73)
    g, t, c = D.stats(sc, cams, st, dL)
    tile_base = np.cumsum([0] + [int(w) // 16 * (int(h) // 16) for w, h in cams.wh])
    view = np.searchsorted(tile_base, (keys >> np.uint64(32)).astype(np.int64), side="right") - 1
    pairs = np.unique(np.stack([view, vals.astype(np.int64)], axis=1), axis=0)
    expect = np.bincount(pairs[:, 1], minlength=sc.n)
    np.testing.assert_array_equal(c, expect)
    assert (g[c == 0] == 0).all() and (t[c == 0] == 0).all()
    assert (t[c > 0] >= c[c > 0] * TMIN * (1 - 1e-12)).all() and (t <= c * TMAX * (1 + 1e-12)).all()


def test_densify_worked_example():
    """Seven Gaussians, expected result written out by hand (extent 100, so the clone / split
    boundary is a largest scale of 0.1):
      0 never visible -> kept;            1 selected, small  -> kept + clone;
      2 selected, large, rotated 90 deg about z -> two children, parent removed;
      3 selected, small, opacity 0.001 -> original and clone pruned;
      4 not selected, opacity 0.001 -> pruned;
      5 selected, large, opacity 0.001 -> children pruned, parent removed;
      6 grad_sum == tau_sum (selected), small -> kept + clone."""
    n = 7
    means = np.array([[1, 2, 3], [4, 5, 6], [7, 8, 9], [1, 1, 1], [2, 2, 2], [3, 3, 3], [5, 4, 3]], np.float32).T.copy()
    scales = np.array([[.01, .02, .03], [.05, .05, .05], [.4, .2, .1], [.01, .01, .01], [.3, .3, .3],
                       [.5, .1, .1], [.1, .05, .02]], np.float32).T.copy()
    c45 = np.float32(np.cos(np.pi / 4))
    quats = np.array([[1, 0, 0, 0]] * 2 + [[c45, 0, 0, c45]] + [[1, 0, 0, 0]] * 4, np.float32).T.copy()
    opac = np.array([.5, .6, .7, .001, .001, .001, .9], np.float32)
    sh = np.arange(3 * n, dtype=np.float32).reshape(3, n)
    grad_sum = np.array([0, 3e-4, 2e-4, 9e-4, 0, 5e-4, 1e-4], np.float32)
    tau_sum = np.array([0, 1e-4, 1e-4, 2e-4, 1e-4, 1e-4, 1e-4], np.float32)
    count = np.array([0, 2, 1, 3, 1, 1, 1], np.int32)
    noise = np.zeros((2, 3, n), np.float32)
    noise[0, :, 2] = (1.0, 0.0, 0.0)
    noise[1, :, 2] = (0.0, 0.0, -2.0)
    out = D.densify(means, scales, quats, opac, sh, grad_sum, tau_sum, count, noise, extent=100.0)
    assert out["counts"] == (3, 2, 1, 1)
    np.testing.assert_array_equal(out["src"], [0, 1, 6, 1, 6, 2, 2])
    # child 0: m + R (s * xi) = (7,8,9) + Rz(90)(0.4, 0, 0) = (7, 8.4, 9); child 1: (7, 8, 9 - 0.2)
    np.testing.assert_allclose(out["means"][:, 5], [7.0, 8.4, 9.0], atol=1e-6)
    np.testing.assert_allclose(out["means"][:, 6], [7.0, 8.0, 8.8], atol=1e-6)
    np.testing.assert_allclose(out["scales"][:, 5], [.25, .125, .0625], rtol=1e-6)
    np.testing.assert_array_equal(out["scales"][:, 6], out["scales"][:, 5])
    np.testing.assert_array_equal(out["means"][:, :5], means[:, [0, 1, 6, 1, 6]])
    np.testing.assert_array_equal(out["opacities"], opac[[0, 1, 6, 1, 6, 2, 2]])
    np.testing.assert_array_equal(out["sh"], sh[:, [0, 1, 6, 1, 6, 2, 2]])
    np.testing.assert_array_equal(out["quats"], quats[:, [0, 1, 6, 1, 6, 2, 2]])
    # with the world-size rule at 0.002 * extent = 0.2, the children (largest scale 0.25) are
    # pruned as well; every other survivor has a largest scale of at most 0.1
    out2 = D.densify(means, scales, quats, opac, sh, grad_sum, tau_sum, count, noise, extent=100.0,
                     max_scale_frac=0.002)
    assert out2["counts"] == (3, 2, 0, 0)
    np.testing.assert_array_equal(out2["src"], [0, 1, 6, 1, 6])


def test_densify_nothing_selected_is_identity():
    rng = np.random.default_rng(74)
    n = 500
    m = rng.standard_normal((3, n)).astype(np.float32)
    s = rng.uniform(0.01, 0.2, (3, n)).astype(np.float32)
    q = rng.standard_normal((4, n)).astype(np.float32)
    o = rng.uniform(0.01, 1, n).astype(np.float32)
    sh = rng.standard_normal((48, n)).astype(np.float32)
    out = D.densify(m, s, q, o, sh, np.zeros(n, np.float32), np.ones(n, np.float32), np.ones(n, np.int32),
                    rng.standard_normal((2, 3, n)).astype(np.float32), extent=10.0)
    assert out["counts"] == (n, 0, 0, 0)
    for k, a in (("means", m), ("scales", s), ("quats", q), ("opacities", o), ("sh", sh)):
        np.testing.assert_array_equal(out[k], a)
