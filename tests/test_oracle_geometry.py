"""Pins of the CPU oracle's projection against facts the paper and textbook mathematics fix.

Every test here runs on the CPU and never touches the GPU path.  The oracle computes J_omni as
the product S_o Q_o J_o T_mu of Sec. 3.2; the tests check it against independent routes to the
same matrices: Appendix B's Cartesian derivative, numerical differentiation of the projection,
closed forms for isotropic and equatorial Gaussians, a perspective camera (Eq. jacob_pers), a
Monte-Carlo projection of samples, and library rotations.
"""
import os

import numpy as np
import pytest
from numpy.polynomial import legendre
from scipy.spatial.transform import Rotation

from oracle import oracle as O
from paper_2410_20686_amd import scenes
from tests._util import cams_from, make_scene, rot_y, settings

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _proj(sc, cams, st=None):
    return O.project(sc, cams, st or settings())


def _cov2(row, dil):
    dil = float(np.float32(dil))  # settings reach the rasterizer (and the oracle) as float32
    uu, uv, vv = row[O.F_COV2:O.F_COV2 + 3]
    return np.array([[uu - dil, uv], [uv, vv - dil]])


def test_erp_closed_form_positions():
    """Eq. equirec_proj (Sec. 3.2) at hand-worked points, including the +-pi seam (u = W)."""
    data = np.loadtxt(os.path.join(GOLDEN, "erp_points.txt"))
    sc = make_scene(data[:, :3] * 3.0, [0.01, 0.01, 0.01])
    pr = _proj(sc, scenes.identity_cameras(256, 128))[0]
    np.testing.assert_allclose(pr[:, O.F_U], data[:, 3], atol=1e-10)
    np.testing.assert_allclose(pr[:, O.F_V], data[:, 4], atol=1e-10)


def _random_camera_space_points(rng, n, max_elev=1.3, max_az=3.0):
    az = rng.uniform(-max_az, max_az, n)
    el = rng.uniform(-max_elev, max_elev, n)
    r = rng.uniform(1.0, 10.0, n)
    # OpenCV axes: elevation measured upwards, y points down
    return np.stack([r * np.cos(el) * np.sin(az), -r * np.sin(el), r * np.cos(el) * np.cos(az)], axis=1)


def _appendix_b_jacobian(mu, W, H):
    """Appendix B's Cartesian derivative of pi_o, written from its first matrix line."""
    x, y, z = mu
    p = x * x + z * z
    r2 = p + y * y
    return np.array([[W / (2 * np.pi) * z / p, 0.0, -W / (2 * np.pi) * x / p],
                     [-H / (np.pi * r2) * x * y / np.sqrt(p), H / (np.pi * r2) * np.sqrt(p),
                      -H / (np.pi * r2) * y * z / np.sqrt(p)]])


def test_jacobian_matches_appendix_b_and_finite_differences():
    rng = np.random.default_rng(1)
    W, H = 512, 256
    mus = _random_camera_space_points(rng, 40)
    sc = make_scene(mus, [0.05, 0.05, 0.05])
    cams = scenes.identity_cameras(W, H)
    pr = _proj(sc, cams)[0]
    h = 1e-6
    for i, mu in enumerate(mus):
        J = pr[i, O.F_J:O.F_J + 6].reshape(2, 3)
        np.testing.assert_allclose(J, _appendix_b_jacobian(mu, W, H), rtol=1e-11, atol=1e-11 * np.abs(J).max())
        fd = np.zeros((2, 3))
        for k in range(3):
            mp, mm = mu.copy(), mu.copy()
            mp[k] += h
            mm[k] -= h
            a = _proj(make_scene([mp, mm], [0.05, 0.05, 0.05]), cams)[0]
            fd[0, k] = (a[0, O.F_U] - a[1, O.F_U]) / (2 * h)
            fd[1, k] = (a[0, O.F_V] - a[1, O.F_V]) / (2 * h)
        np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-6 * np.abs(J).max())


def test_isotropic_gaussian_closed_form():
    """Eq. omni_J + Eq. omni_QS: an isotropic Gaussian (Sigma = s^2 I) at elevation theta and
    distance r has Sigma_2D = diag((W s sec(theta) / (2 pi r))^2, (H s / (pi r))^2), for any
    camera rotation."""
    rng = np.random.default_rng(2)
    W, H, dil = 1024, 512, 0.3
    for trial in range(20):
        Rc = Rotation.random(random_state=trial).as_matrix()
        t = rng.uniform(-1, 1, 3)
        mu = _random_camera_space_points(rng, 1)[0]
        m = Rc.T @ (mu - t)
        s = rng.uniform(0.01, 0.3)
        sc = make_scene([m], [s, s, s], quats=Rotation.random(random_state=100 + trial).as_quat()[[3, 0, 1, 2]])
        row = _proj(sc, cams_from([Rc], [t], [[W, H]]), settings(dilation=dil))[0, 0]
        r = np.linalg.norm(mu)
        theta = np.arctan2(-mu[1], np.hypot(mu[0], mu[2]))
        expect = np.diag([(W * s / (2 * np.pi * r * np.cos(theta))) ** 2, (H * s / (np.pi * r)) ** 2])
        np.testing.assert_allclose(_cov2(row, dil), expect, rtol=1e-10, atol=1e-12 * expect.max())


def test_equator_matches_perspective_projection():
    """At zero elevation, J_omni equals the perspective Jacobian of Eq. jacob_pers (focal
    lengths W/2pi, H/pi) of a camera yawed to look at the Gaussian: a small Gaussian on the
    equator is projected like a perspective camera would project it."""
    rng = np.random.default_rng(3)
    W, H = 2048, 1024
    fx, fy = W / (2 * np.pi), H / np.pi
    for trial in range(20):
        az, r = rng.uniform(-3.0, 3.0), rng.uniform(1.5, 8.0)
        mu = np.array([r * np.sin(az), 0.0, r * np.cos(az)])
        q = Rotation.random(random_state=trial).as_quat()[[3, 0, 1, 2]]
        sc = make_scene([mu], rng.uniform(0.01, 0.2, 3), quats=q)
        row = _proj(sc, scenes.identity_cameras(W, H))[0, 0]
        cov3 = row[O.F_COV3:O.F_COV3 + 6]
        Sig = np.array([[cov3[0], cov3[1], cov3[2]], [cov3[1], cov3[3], cov3[4]], [cov3[2], cov3[4], cov3[5]]])
        Ry = rot_y(az)                      # turns the Gaussian onto the new camera's +z axis
        mu_p = Ry @ mu
        assert abs(mu_p[0]) < 1e-12 and abs(mu_p[1]) < 1e-12
        Jp = np.array([[fx / mu_p[2], 0.0, -fx * mu_p[0] / mu_p[2] ** 2],
                       [0.0, fy / mu_p[2], -fy * mu_p[1] / mu_p[2] ** 2]])
        expect = Jp @ Ry @ Sig @ Ry.T @ Jp.T
        np.testing.assert_allclose(_cov2(row, 0.3), expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())


def test_monte_carlo_projection_of_samples():
    """The local-affine 2D covariance equals the covariance of 3D samples pushed through the
    exact ERP map (Sec. 3.2), up to sampling noise, for a small Gaussian."""
    rng = np.random.default_rng(4)
    W, H = 2048, 1024
    for trial, (el, az) in enumerate([(0.4, 1.0), (-0.9, -2.5), (1.1, 0.3)]):
        r = 5.0
        mu = np.array([r * np.cos(el) * np.sin(az), -r * np.sin(el), r * np.cos(el) * np.cos(az)])
        q = Rotation.random(random_state=7 + trial).as_quat()[[3, 0, 1, 2]]
        sc = make_scene([mu], [0.004, 0.002, 0.003], quats=q)
        row = _proj(sc, scenes.identity_cameras(W, H))[0, 0]
        c3 = row[O.F_COV3:O.F_COV3 + 6]
        Sig = np.array([[c3[0], c3[1], c3[2]], [c3[1], c3[3], c3[4]], [c3[2], c3[4], c3[5]]])
        pts = rng.multivariate_normal(mu, Sig, size=400_000)
        u = W / (2 * np.pi) * np.arctan2(pts[:, 0], pts[:, 2]) + W / 2
        v = -H / np.pi * np.arctan2(-pts[:, 1], np.hypot(pts[:, 0], pts[:, 2])) + H / 2
        emp = np.cov(np.stack([u, v]))
        model = _cov2(row, 0.3)
        scale = np.sqrt(model[0, 0] * model[1, 1])
        assert abs(emp[0, 0] / model[0, 0] - 1) < 0.015
        assert abs(emp[1, 1] / model[1, 1] - 1) < 0.015
        assert abs(emp[0, 1] - model[0, 1]) < 0.015 * scale


def test_quaternion_to_covariance():
    """Sigma = R S S^T R^T (Sec. 3.1): a quaternion for a rotation by a about z (any length)
    gives Rz(a) diag(s^2) Rz(a)^T; random quaternions match scipy's rotation matrices."""
    s = np.array([0.1, 0.2, 0.3])
    for a in (0.0, 0.3, 1.2, -2.0):
        q = 3.0 * np.array([np.cos(a / 2), 0.0, 0.0, np.sin(a / 2)])
        Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
        expect = Rz @ np.diag(s ** 2) @ Rz.T
        row = _proj(make_scene([[0.3, 0.1, 4.0]], s, quats=q), scenes.identity_cameras(64, 32))[0, 0]
        c3 = row[O.F_COV3:O.F_COV3 + 6]
        got = np.array([[c3[0], c3[1], c3[2]], [c3[1], c3[3], c3[4]], [c3[2], c3[4], c3[5]]])
        np.testing.assert_allclose(got, expect, atol=1e-14)
    rng = np.random.default_rng(5)
    for trial in range(10):
        rot = Rotation.random(random_state=trial)
        xyzw = rot.as_quat() * rng.uniform(0.3, 3.0)
        s = rng.uniform(0.01, 0.5, 3)
        R = rot.as_matrix()
        expect = R @ np.diag(s ** 2) @ R.T
        row = _proj(make_scene([[0.3, 0.1, 4.0]], s, quats=xyzw[[3, 0, 1, 2]]), scenes.identity_cameras(64, 32))[0, 0]
        c3 = row[O.F_COV3:O.F_COV3 + 6]
        got = np.array([[c3[0], c3[1], c3[2]], [c3[1], c3[3], c3[4]], [c3[2], c3[4], c3[5]]])
        np.testing.assert_allclose(got, expect, atol=1e-13)


def test_rigid_motion_of_world_and_camera_is_invisible():
    """Moving the world and the camera by the same rigid motion leaves every projected quantity
    unchanged (checks where W = world-to-camera rotation enters Sigma_2D = J W Sigma W^T J^T)."""
    sc = scenes.sphere_scene(60, 0, seed=9).as_f64()
    Rc = Rotation.random(random_state=1).as_matrix()
    tc = np.array([0.2, -0.1, 0.3])
    Q = Rotation.random(random_state=2)
    d = np.array([1.0, -2.0, 0.5])
    sc2 = sc.copy()
    sc2.means = np.ascontiguousarray((Q.as_matrix() @ sc.means) + d[:, None])
    qr = Rotation.from_quat(sc.quats[[1, 2, 3, 0]].T)
    sc2.quats = np.ascontiguousarray((Q * qr).as_quat().T[[3, 0, 1, 2]])
    Rc2 = Rc @ Q.as_matrix().T
    tc2 = tc - Rc2 @ d
    a = _proj(sc, cams_from([Rc], [tc], [[512, 256]]))[0]
    b = _proj(sc2, cams_from([Rc2], [tc2], [[512, 256]]))[0]
    for f, w in ((O.F_U, 1), (O.F_V, 1), (O.F_COV2, 3), (O.F_CONIC, 3), (O.F_RGB, 3)):
        np.testing.assert_allclose(b[:, f:f + w], a[:, f:f + w], rtol=1e-9, atol=1e-9)


def test_sh_basis_orthonormal():
    """The real SH basis is orthonormal on the unit sphere (Gauss-Legendre x uniform azimuth
    quadrature, exact for these polynomial degrees)."""
    z, wz = legendre.leggauss(24)
    phi = np.linspace(0, 2 * np.pi, 48, endpoint=False)
    Z, P = np.meshgrid(z, phi, indexing="ij")
    Wq = np.repeat(wz, len(phi)) * (2 * np.pi / len(phi))
    s = np.sqrt(1 - Z ** 2)
    dirs = np.stack([s * np.cos(P), s * np.sin(P), Z], axis=-1).reshape(-1, 3)
    Y = O.sh_basis(dirs, 16)
    gram = (Y * Wq[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_addition_theorem():
    """sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a . b) for each band l (basis-independent)."""
    rng = np.random.default_rng(6)
    a = rng.standard_normal((50, 3))
    b = rng.standard_normal((50, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, Yb = O.sh_basis(a, 16), O.sh_basis(b, 16)
    cosg = np.sum(a * b, axis=1)
    for l in range(4):
        sl = slice(l * l, (l + 1) * (l + 1))
        lhs = np.sum(Ya[:, sl] * Yb[:, sl], axis=1)
        rhs = (2 * l + 1) / (4 * np.pi) * legendre.legval(cosg, [0] * l + [1])
        np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_degree0_colour_is_view_independent():
    rng = np.random.default_rng(7)
    dc = rng.uniform(-1.5, 1.5, (3, 5))
    sc = make_scene(rng.uniform(-3, 3, (5, 3)) + np.array([0, 0, 6.0]), [0.1, 0.1, 0.1], sh=dc)
    cams = scenes.yaw_cameras(3, 128, 64, seed=1)
    pr = _proj(sc, cams)
    expect = dc.T / (2 * np.sqrt(np.pi)) + 0.5
    for v in range(3):
        np.testing.assert_allclose(pr[v, :, O.F_RGB:O.F_RGB + 3], np.maximum(expect, 0), atol=1e-14)


# Appendix C, gradient of the loss w.r.t. the camera-space mean t through J: coefficient of each
# dL/dJ(i,j) in dL/dt_x, dL/dt_y, dL/dt_z, transcribed as printed (rows 1 and 2).
def _appendix_c(t, W, H):
    tx, ty, tz = t
    p = tx * tx + tz * tz
    r2 = p + ty * ty
    r4 = r2 * r2
    sp = np.sqrt(p)
    c = np.zeros((3, 2, 3))  # [d/dt_k][J row][J col]
    c[0, 0, 0] = -W / np.pi * tx * tz / p ** 2
    c[0, 0, 2] = W / (2 * np.pi) * (tx ** 2 - tz ** 2) / p ** 2
    c[0, 1, 0] = H / np.pi * ty * (tz ** 2 * r2 - 2 * tx ** 2 * p) / (r4 * p ** 1.5)
    c[0, 1, 1] = H / np.pi * tx * (r2 - 2 * ty ** 2) / (r4 * sp)
    c[0, 1, 2] = -H / np.pi * tx * ty * tz * (2 * p + r2) / (r4 * p ** 1.5)
    c[1, 1, 0] = H / np.pi * tx * (r2 - 2 * ty ** 2) / (r4 * sp)
    c[1, 1, 1] = 2 * H / np.pi * ty * sp / r4
    c[1, 1, 2] = H / np.pi * tz * (r2 - 2 * ty ** 2) / (r4 * sp)
    c[2, 0, 0] = W / (2 * np.pi) * (tx ** 2 - tz ** 2) / p ** 2
    c[2, 0, 2] = W / np.pi * tx * tz / p ** 2
    c[2, 1, 0] = -H / np.pi * tx * ty * tz * (2 * p + r2) / (r4 * p ** 1.5)
    c[2, 1, 1] = H / np.pi * tz * (r2 - 2 * ty ** 2) / (r4 * sp)
    c[2, 1, 2] = H / np.pi * ty * (tx ** 2 * r2 - 2 * tz ** 2 * p) / (r4 * p ** 1.5)
    return c


def test_appendix_c_position_terms():
    """Appendix C's first-row terms equal dJ_omni/dt of the oracle's J (finite differences);
    its second-row terms hold with the opposite sign (the reading recorded for that appendix),
    i.e. they are derivatives of -J row 2, not of the J of Eq. omni_Jacobian."""
    rng = np.random.default_rng(8)
    W, H = 1024, 512
    cams = scenes.identity_cameras(W, H)
    h = 1e-6
    for mu in _random_camera_space_points(rng, 10):
        ac = _appendix_c(mu, W, H)
        for k in range(3):
            mp, mm = mu.copy(), mu.copy()
            mp[k] += h
            mm[k] -= h
            a = _proj(make_scene([mp, mm], [0.05, 0.05, 0.05]), cams)[0]
            dJ = (a[0, O.F_J:O.F_J + 6] - a[1, O.F_J:O.F_J + 6]).reshape(2, 3) / (2 * h)
            tol = 1e-6 * np.abs(dJ).max() + 1e-9
            np.testing.assert_allclose(dJ[0], ac[k, 0], atol=tol)
            np.testing.assert_allclose(dJ[1], -ac[k, 1], atol=tol)
