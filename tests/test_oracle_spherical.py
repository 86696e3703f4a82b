"""Pins of the oracle's spherical footprint: the exact per-ray evaluation of a 3D Gaussian in
equirectangular views that replaces the local affine approximation (the limitation named in
Sec. 5).  Each pixel ray t d (t > 0) gets exp(-m/2) with m the minimum of the Gaussian's
Mahalanobis distance along the ray.

Pinned by: numerical line minimisation of the covariance built here from the raw parameters,
the isotropic closed form, the tangent-frame form against the definition, convergence to the
affine model as the Gaussian shrinks, yaw = circular shift, band = brute force (the cone
rectangle covers every accepted pixel), FP64 central differences of the gradient, and the
kernel-layout adjoint against the definition-layout adjoint."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests._util import cams_from, image, make_scene, plane, rot_y, settings

SPH = dict(footprint="spherical")


def _quat_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _pixel_dir(x, y, W, H):
    phi = (x + 0.5) / W * 2 * np.pi - np.pi
    th = np.pi / 2 - (y + 0.5) / H * np.pi
    return np.array([np.cos(th) * np.sin(phi), -np.sin(th), np.cos(th) * np.cos(phi)])


def _queries(sc, cams, st, rng, n, near_only=True):
    """(view, x, y, gaussian) rows, mostly pixels near kept Gaussians' centres."""
    rows = O.project(sc, cams, st)
    out = []
    while len(out) < n:
        v = int(rng.integers(0, cams.wh.shape[0]))
        i = int(rng.integers(0, sc.n))
        if rows[v, i, O.F_KEPT] != 1:
            continue
        W, H = (int(x) for x in cams.wh[v])
        if near_only:
            x = int(np.floor(rows[v, i, O.F_U] + rng.normal(0, 4))) % W
            y = int(np.clip(np.floor(rows[v, i, O.F_V] + rng.normal(0, 4)), 0, H - 1))
        else:
            x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        out.append((v, x, y, i))
    return np.array(out, dtype=np.int32)


def test_definition_equals_numerical_line_minimum():
    """m by the oracle's closed form equals a numerical minimisation over t of the quadratic
    built here from the raw parameters: Sigma = R(q) diag(s^2) R(q)^T in world space, moved to
    the camera, plus the angular low-pass delta (pi/H)^2 at the mean's distance."""
    sc = scenes.sphere_scene(200, 0, seed=31, r_range=(1.5, 4.0)).as_f64()
    cams = scenes.yaw_cameras(2, 128, 64, seed=31)
    st = settings(dilation=0.3, **SPH)
    rng = np.random.default_rng(31)
    q = _queries(sc, cams, st, rng, 120)
    ev = O.sph_eval(sc, cams, st, q)
    checked = 0
    for (v, x, y, i), e in zip(q, ev):
        R = cams.cams[v, :9].reshape(3, 3)
        t = cams.cams[v, 9:]
        W, H = (int(a) for a in cams.wh[v])
        Rq = _quat_rot(sc.quats[:, i])
        Sig = Rq @ np.diag(sc.scales[:, i] ** 2) @ Rq.T
        mu = R @ sc.means[:, i] + t
        r = np.linalg.norm(mu)
        Sc = R @ Sig @ R.T + float(np.float32(0.3)) * (np.pi / H) ** 2 * r * r * np.eye(3)
        Ai = np.linalg.inv(Sc)
        d = _pixel_dir(x, y, W, H)
        f = lambda tt: (tt * d - mu) @ Ai @ (tt * d - mu)
        res = minimize_scalar(f, bounds=(0.0, 4.0 * r), method="bounded", options=dict(xatol=1e-12 * r))
        if e[1] <= 0:  # minimiser behind the camera: no contribution
            continue
        assert abs(e[0] - res.fun) <= 1e-7 * max(1.0, res.fun), (v, x, y, i, e[0], res.fun)
        checked += 1
    assert checked > 100


@pytest.mark.parametrize("dil", [0.0, 0.3])
def test_isotropic_closed_form(dil):
    """Isotropic Gaussian, radius s at distance r: m = r^2 sin^2(gamma) / (s^2 + delta r^2), with
    gamma the angle between the pixel ray and the mean and delta = dilation (pi / H)^2; the
    rendered colour of a lone Gaussian is o exp(-m/2) rgb where that is >= 1/255."""
    W, H = 256, 128
    s, o = 0.15, 0.8
    mu = np.array([0.7, -1.1, 2.3])
    sc = make_scene([mu], [[s, s, s]], opac=o, sh=[[1.0], [0.4], [-0.3]])
    cams = cams_from([np.eye(3)], [np.zeros(3)], [(W, H)])
    st = settings(dilation=dil, **SPH)
    img = image(O.render(sc, cams, st, mode=64)["rgb"], cams, 0)
    r = np.linalg.norm(mu)
    dlt = float(np.float32(dil)) * (np.pi / H) ** 2
    ys, xs = np.mgrid[0:H, 0:W]
    phi = (xs + 0.5) / W * 2 * np.pi - np.pi
    th = np.pi / 2 - (ys + 0.5) / H * np.pi
    d = np.stack([np.cos(th) * np.sin(phi), -np.sin(th), np.cos(th) * np.cos(phi)])
    cosg = np.tensordot(mu / r, d, axes=1)
    m = r * r * (1 - cosg ** 2) / (s * s + dlt * r * r)
    a = o * np.exp(-0.5 * m)
    a = np.where((cosg > 0) & (a >= 1 / 255), np.minimum(a, 0.99), 0.0)
    C0 = 0.28209479177387814
    rgb = np.maximum(np.array([1.0, 0.4, -0.3]) * C0 + 0.5, 0)
    np.testing.assert_allclose(img, a[None] * rgb[:, None, None], atol=1e-12)
    assert (a > 0).sum() > 50


def test_tangent_frame_form_equals_definition():
    """The kernel's sum-of-squares form (tangent frame, factor of P^-1 / 2, w, k2) evaluated in
    double equals the definition c - b^2 / a; the float exponent is within float rounding of
    -m/2, and accepted exactly where the definition accepts away from the threshold."""
    sc = scenes.roaming_scene(400, 0, seed=32, r_range=(1.2, 6.0)).as_f64()
    cams = scenes.uneven_cameras(3, seed=32, sizes=((128, 64), (256, 128), (512, 256)))
    st = settings(**SPH)
    rng = np.random.default_rng(32)
    q = _queries(sc, cams, st, rng, 400)
    ev = O.sph_eval(sc, cams, st, q)
    rows = O.project(sc, cams, st)
    front = ev[:, 1] > 0
    assert front.sum() > 350
    np.testing.assert_allclose(ev[front, 2], ev[front, 0], rtol=1e-8, atol=1e-10)
    pmin = rows[q[:, 0], q[:, 3], O.F_PMIN]
    power = -0.5 * ev[:, 0]
    acc = front & (power >= pmin)
    clear = np.abs(power - pmin) > 1e-4 * (1 + np.abs(pmin))
    np.testing.assert_array_equal(ev[clear, 4].astype(bool), acc[clear])
    both = acc & (ev[:, 4] == 1)
    np.testing.assert_allclose(ev[both, 3], power[both], rtol=1e-4, atol=1e-5)
    assert both.sum() > 100


def test_small_gaussians_converge_to_the_affine_model():
    """Without the low-pass term, the affine (tangent-plane) exponent and the exact per-ray one
    differ at first order in the Gaussian's angular size: halving every scale roughly halves the
    largest relative difference of m inside the footprint, at latitudes up to about 60 degrees."""
    rng = np.random.default_rng(33)
    n = 40
    az = rng.uniform(-np.pi, np.pi, n)
    el = rng.uniform(-1.05, 1.05, n)
    r = rng.uniform(4, 6, n)
    means = np.stack([r * np.cos(el) * np.sin(az), -r * np.sin(el), r * np.cos(el) * np.cos(az)], axis=1)
    quats = rng.standard_normal((n, 4))
    base = rng.uniform(0.5, 1.0, (n, 3))
    W, H = 2048, 1024
    cams = cams_from([np.eye(3)], [np.zeros(3)], [(W, H)])
    errs = []
    for scale in (0.04, 0.02, 0.01):
        sc = make_scene(means, base * scale, quats=quats, opac=0.9)
        st_a = settings(dilation=0.0)
        st_s = settings(dilation=0.0, **SPH)
        rows = O.project(sc, cams, st_a)[0]
        qs, maff = [], []
        for i in range(n):
            a, b, c = rows[i, O.F_CONIC:O.F_CONIC + 3]
            u, v = rows[i, O.F_U], rows[i, O.F_V]
            for _ in range(30):
                x = int(np.floor(u + rng.normal(0, 1.5 * np.sqrt(rows[i, O.F_COV2])))) % W
                y = int(np.clip(np.floor(v + rng.normal(0, 1.5 * np.sqrt(rows[i, O.F_COV2 + 2]))), 0, H - 1))
                du = (x + 0.5 - u + W / 2) % W - W / 2
                dv = y + 0.5 - v
                m = a * du * du + 2 * b * du * dv + c * dv * dv
                if m < 9.0:
                    qs.append((0, x, y, i))
                    maff.append(m)
        ev = O.sph_eval(sc, cams, st_s, np.array(qs))
        maff = np.array(maff)
        errs.append(np.max(np.abs(ev[:, 0] - maff) / (1.0 + maff)))
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert errs[-1] < 0.05, errs
    assert all(1.5 < q < 2.7 for q in ratios), (errs, ratios)


@pytest.mark.parametrize("k", [3, 128])
def test_yaw_rotation_is_circular_shift(k):
    W, H = 256, 128
    sc = scenes.sphere_scene(600, 3, seed=34).as_f64()
    c = np.array([0.1, -0.05, 0.2])
    R0 = rot_y(0.37)
    R1 = rot_y(2 * np.pi * k / W) @ R0
    cams = cams_from([R0, R1], [-R0 @ c, -R1 @ c], [[W, H], [W, H]])
    r = O.render(sc, cams, settings(**SPH), mode=64)
    a, b = image(r["rgb"], cams, 0), image(r["rgb"], cams, 1)
    np.testing.assert_allclose(b, np.roll(a, -k, axis=2), atol=1e-9)
    np.testing.assert_allclose(plane(r["T"], cams, 1), np.roll(plane(r["T"], cams, 0), -k, axis=1), atol=1e-9)


def _hard_scene():
    """Small and large Gaussians, some near the poles, some across the seam, some so large and
    close that their cone holds the whole sphere."""
    rng = np.random.default_rng(35)
    sc = scenes.roaming_scene(1500, 3, seed=35, r_range=(1.0, 6.0))
    n = 40
    az = np.concatenate([rng.uniform(-np.pi, np.pi, n - 10), np.pi + rng.uniform(-0.1, 0.1, 10)])
    el = np.concatenate([rng.choice([-1, 1], 20) * rng.uniform(1.2, 1.55, 20), rng.uniform(-1, 1, n - 20)])
    r = rng.uniform(0.6, 3.0, n)
    means = np.stack([r * np.cos(el) * np.sin(az), -r * np.sin(el), r * np.cos(el) * np.cos(az)], axis=1)
    big = make_scene(means, rng.uniform(0.05, 0.5, (n, 3)), quats=rng.standard_normal((n, 4)),
                     opac=rng.uniform(0.05, 0.9, n), sh=rng.uniform(-1, 1, (48, n)), sh_degree=3)
    return scenes.Scene(*(np.concatenate([getattr(sc, f).astype(np.float64), getattr(big, f)], axis=-1)
                          for f in ("means", "scales", "quats", "opacities", "sh")), 3)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_cone_rectangles_render_identically_to_brute_force(tile):
    sc = _hard_scene()
    cams = scenes.uneven_cameras(2, seed=36, sizes=((128, 64), (256, 128)))
    st = settings(tile=tile, **SPH)
    a = O.render(sc, cams, st, mode=32, band=False)
    b = O.render(sc, cams, st, mode=32, band=True)
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    np.testing.assert_array_equal(a["sig"], b["sig"])
    rows = O.project(sc, cams, st)
    full = (rows[..., O.F_KEPT] == 1) & (rows[..., O.F_BETA] >= np.pi)
    assert full.sum() >= 1 and (a["T"] < 0.5).mean() > 0.2


def test_spherical_and_affine_agree_at_the_equator_for_small_gaussians():
    """At the equator of a 2:1 image the angular low-pass delta (pi/H)^2 equals the affine one in
    pixels, so small distant Gaussians render nearly alike in both models."""
    rng = np.random.default_rng(37)
    n = 30
    az = rng.uniform(-np.pi, np.pi, n)
    el = rng.uniform(-0.02, 0.02, n)
    r = rng.uniform(8, 10, n)
    means = np.stack([r * np.cos(el) * np.sin(az), -r * np.sin(el), r * np.cos(el) * np.cos(az)], axis=1)
    sc = make_scene(means, rng.uniform(0.005, 0.01, (n, 3)), quats=rng.standard_normal((n, 4)), opac=0.7,
                    sh=rng.uniform(-1, 1, (3, n)))
    cams = cams_from([np.eye(3)], [np.zeros(3)], [(1024, 512)])
    a = O.render(sc, cams, settings(), mode=64)["rgb"]
    b = O.render(sc, cams, settings(**SPH), mode=64)["rgb"]
    assert np.abs(a - b).max() < 0.01 and np.abs(a).max() > 0.2


def test_gradient_by_finite_differences():
    sc = scenes.sphere_scene(250, 3, seed=38, r_range=(1.5, 4.0)).as_f64()
    cams = scenes.uneven_cameras(2, seed=38, sizes=((64, 32), (128, 64)))
    st = settings(bg=(0.1, 0.2, 0.0), **SPH)
    dL = scenes.upstream_gradient(cams, 1038).astype(np.float64)
    g = O.backward(sc, cams, st, dL, mode=64)
    rng = np.random.default_rng(39)
    groups = [("means", 3), ("scales", 3), ("quats", 4), ("opacities", 1), ("sh", 48)]
    visible = np.nonzero(np.abs(g["opacities"]) > 0)[0]
    checked = tries = 0
    while checked < 50:
        tries += 1
        assert tries < 400
        name, nrows = groups[checked % len(groups)]
        i = int(rng.choice(visible))
        c = int(rng.integers(0, nrows))
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


def test_kernel_layout_adjoint_reproduces_the_backward():
    """Gradients taken w.r.t. the kernel's variables (mu^, Sigma~) and pushed through the
    projection equal those taken w.r.t. (mu^, A = Sigma~^-1): two derivations of the chain rule."""
    sc = scenes.roaming_scene(600, 3, seed=40, r_range=(1.5, 6.0)).as_f64()
    cams = scenes.uneven_cameras(2, seed=40, sizes=((128, 64), (256, 128)))
    st = settings(bg=(0.1, 0.0, 0.2), **SPH)
    dL = scenes.upstream_gradient(cams, 1040).astype(np.float64)
    g = O.backward(sc, cams, st, dL, mode=64, want_g2d=True)
    h = O.project_adjoint(sc, cams, st, g["g2d_kernel"])
    for k in ("means", "scales", "quats", "opacities", "sh"):
        np.testing.assert_allclose(h[k], g[k], rtol=1e-7, atol=1e-10 * np.abs(g[k]).max())
    assert np.abs(g["means"]).max() > 0


@pytest.mark.parametrize("footprint", ["affine", "spherical"])
def test_float_exponent_mode_moves_gradients_only_slightly(footprint):
    """Mode 33 (the derivative taken at the float pass's own exponents) differs from the reference
    (mode 32) only through the exponents' float rounding: on ordinary Gaussians by less than 5e-5
    (affine) or 5e-4 (spherical: three-term dot products of the ray with whitening vectors of
    length ~1/angular size) relative per element, plus a 1e-7 floor of the tensor's scale."""
    sc = scenes.roaming_scene(700, 3, seed=44, r_range=(1.5, 6.0))
    cams = scenes.uneven_cameras(2, seed=44, sizes=((128, 64), (256, 128)))
    st = settings(footprint=footprint)
    dL = scenes.upstream_gradient(cams, 1044).astype(np.float64)
    a = O.backward(sc, cams, st, dL, mode=32)
    b = O.backward(sc, cams, st, dL, mode=33)
    moved = 0.0
    for k in ("means", "scales", "quats", "opacities", "sh"):
        lim = (5e-5 if footprint == "affine" else 5e-4) * np.abs(a[k]) + 1e-7 * np.abs(a[k]).max()
        assert (np.abs(a[k] - b[k]) <= lim).all(), k
        moved = max(moved, np.abs(a[k] - b[k]).max())
    assert moved > 0.0  # the float exponents do differ from the double ones somewhere
