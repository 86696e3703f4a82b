"""Seeded synthetic scenes, camera poses and upstream image gradients.

This module only draws inputs. It holds none of the rasterizer's arithmetic, so the CPU
reference and the GPU path can both consume it without sharing any of the method.

Conventions of the arrays it returns (the C ABI's input layout):

* ``means``      float32 [3][N]   world-space Gaussian centres (structure of arrays)
* ``scales``     float32 [3][N]   linear, strictly positive axis scales
* ``quats``      float32 [4][N]   (w, x, y, z), not necessarily unit length
* ``opacities``  float32 [N]      in (0, 1)
* ``sh``         float32 [K*3][N] spherical-harmonic colour coefficients, plane k*3+channel,
                                  K = (degree+1)^2
* ``cams``       float32 [V][12]  world-to-camera rotation R (row-major 3x3) then t (3):
                                  x_cam = R x_world + t, OpenCV axes (z forward, x right, y down)
* ``wh``         int32   [V][2]   (width, height) of each equirectangular view

Workload recipes (the paper's datasets are not available; these stand in for them,
with resolutions in the range the paper uses, 1920x960 to 4096x2048):

* ``cfg0`` 2,000 Gaussians, directions uniform on the sphere, radius U[1,5], log-scales
  U[ln 0.01, ln 0.2], random unit quaternions, opacity sigmoid(N(0,1)), SH degree 0 with
  RGB uniform in [0,1]; one identity camera, 256x128.
* ``cfg1`` 100,000 Gaussians drawn as cfg0 but SH degree 3 (coefficients beyond DC
  N(0, 0.2^2)); identity camera, 2048x1024.
* ``cfg2`` 500,000 Gaussians: 70% in 50 blobs (blob centre direction uniform, radius
  U[2,20], member offsets N(0, 0.5^2 I)), 30% uniform in volume in the shell r in [2,20],
  SH degree 3, 5% of them moved onto the +-pi seam of the identity camera; 4096x2048.
* ``cfg3`` 1,000,000 Gaussians with the cfg2 distribution; 8 views 2048x1024, camera
  centres uniform in a 1 m cube, random yaw about the camera's y axis.
* ``cfg4`` 300,000 Gaussians with the cfg2 distribution; 16 views with sizes drawn from
  {1024x512, 2048x1024, 4096x2048}, uniformly random rotations, centres as cfg3.
* ``M``    500,000 Gaussians with the cfg2 distribution; 8 views 2048x1024 as cfg3.

Every draw uses numpy's PCG64 generator seeded with the config index (M uses 5); the
upstream image gradient of a config uses seed 1000 + index.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# RGB uniform in [0, 1] under a degree-0 colour basis constant of 1/(2*sqrt(pi)) and an
# offset of 0.5 corresponds to a DC coefficient uniform in [-sqrt(pi), sqrt(pi)].
_DC_HALF_RANGE = float(np.sqrt(np.pi))


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def as_f64(self) -> "Scene":
        return Scene(*(np.ascontiguousarray(a, dtype=np.float64) for a in
                       (self.means, self.scales, self.quats, self.opacities, self.sh)),
                     self.sh_degree)

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.scales.copy(), self.quats.copy(),
                     self.opacities.copy(), self.sh.copy(), self.sh_degree)

    def subset(self, idx) -> "Scene":
        return Scene(np.ascontiguousarray(self.means[:, idx]), np.ascontiguousarray(self.scales[:, idx]),
                     np.ascontiguousarray(self.quats[:, idx]), np.ascontiguousarray(self.opacities[idx]),
                     np.ascontiguousarray(self.sh[:, idx]), self.sh_degree)


@dataclasses.dataclass
class Cameras:
    cams: np.ndarray  # float32 [V][12]
    wh: np.ndarray    # int32 [V][2]

    @property
    def n_views(self) -> int:
        return int(self.cams.shape[0])

    @property
    def pixels(self) -> int:
        return int(np.sum(self.wh[:, 0].astype(np.int64) * self.wh[:, 1]))

    def view(self, v: int) -> "Cameras":
        return Cameras(np.ascontiguousarray(self.cams[v:v + 1]), np.ascontiguousarray(self.wh[v:v + 1]))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_rows(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _appearance(rng, n, sh_degree, log_scale_range=(np.log(0.01), np.log(0.2))):
    scales = np.exp(rng.uniform(log_scale_range[0], log_scale_range[1], size=(3, n)))
    quats = _unit_rows(rng.standard_normal((n, 4))).T
    opac = _sigmoid(rng.standard_normal(n))
    k = (sh_degree + 1) ** 2
    sh = np.zeros((k * 3, n))
    sh[0:3] = rng.uniform(-_DC_HALF_RANGE, _DC_HALF_RANGE, size=(3, n))
    if k > 1:
        sh[3:] = rng.normal(0.0, 0.2, size=((k - 1) * 3, n))
    return scales, quats, opac, sh


def _finish(means, scales, quats, opac, sh, deg) -> Scene:
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means), f(scales), f(quats), f(opac), f(sh), deg)


def sphere_scene(n: int, sh_degree: int, seed: int, r_range=(1.0, 5.0)) -> Scene:
    """cfg0/cfg1 distribution: direction uniform on the sphere, radius uniform in r_range."""
    rng = np.random.default_rng(seed)
    dirs = _unit_rows(rng.standard_normal((n, 3)))
    rad = rng.uniform(r_range[0], r_range[1], size=n)
    means = (dirs * rad[:, None]).T
    return _finish(means, *_appearance(rng, n, sh_degree), sh_degree)


def roaming_scene(n: int, sh_degree: int, seed: int, n_blobs: int = 50, blob_frac: float = 0.7,
                  r_range=(2.0, 20.0), blob_sigma: float = 0.5, seam_frac: float = 0.05) -> Scene:
    """cfg2 distribution: clustered blobs plus a uniform shell, with seam straddlers injected.

    Seam straddlers: a random ``seam_frac`` of the Gaussians is rotated about the world y axis
    so that its azimuth (seen from the origin, forward = +z) lies within two largest scales of
    the +-pi direction, i.e. its footprint crosses the left/right image border of an identity
    camera at the origin.
    """
    rng = np.random.default_rng(seed)
    n_blob = int(round(n * blob_frac))
    n_shell = n - n_blob
    centres = _unit_rows(rng.standard_normal((n_blobs, 3))) * rng.uniform(*r_range, size=n_blobs)[:, None]
    member = rng.integers(0, n_blobs, size=n_blob)
    blob_pts = centres[member] + rng.normal(0.0, blob_sigma, size=(n_blob, 3))
    # uniform in volume: r^3 uniform between r0^3 and r1^3
    r3 = rng.uniform(r_range[0] ** 3, r_range[1] ** 3, size=n_shell)
    shell_pts = _unit_rows(rng.standard_normal((n_shell, 3))) * np.cbrt(r3)[:, None]
    pts = np.concatenate([blob_pts, shell_pts], axis=0)
    pts = pts[rng.permutation(n)]
    scales, quats, opac, sh = _appearance(rng, n, sh_degree)
    n_seam = int(round(n * seam_frac))
    if n_seam:
        sel = rng.choice(n, size=n_seam, replace=False)
        p = pts[sel]
        horiz = np.sqrt(p[:, 0] ** 2 + p[:, 2] ** 2)
        rad = np.linalg.norm(p, axis=1)
        ang = 2.0 * scales[:, sel].max(axis=0) / np.maximum(rad, 1e-6)
        az = np.pi + rng.uniform(-1.0, 1.0, size=n_seam) * ang
        pts[sel, 0] = horiz * np.sin(az)
        pts[sel, 2] = horiz * np.cos(az)
    return _finish(pts.T, scales, quats, opac, sh, sh_degree)


def _pack_cams(rots, centres, wh) -> Cameras:
    cams = np.zeros((len(rots), 12))
    for v, (r, c) in enumerate(zip(rots, centres)):
        cams[v, :9] = r.reshape(-1)
        cams[v, 9:] = -r @ c
    return Cameras(np.ascontiguousarray(cams, dtype=np.float32), np.ascontiguousarray(wh, dtype=np.int32))


def identity_cameras(width: int, height: int, n_views: int = 1) -> Cameras:
    return _pack_cams([np.eye(3)] * n_views, [np.zeros(3)] * n_views, [[width, height]] * n_views)


def yaw_matrix(angle: float) -> np.ndarray:
    """Rotation by ``angle`` about the camera's y axis (an input-side pose, not the method)."""
    c, s = np.cos(angle), np.sin(angle)
    return np.array([[c, 0.0, -s], [0.0, 1.0, 0.0], [s, 0.0, c]])


def cube_rotations():
    """World-to-camera rotations of the six cube faces (camera axes x right, y down, z forward as
    rows): looking along +z, -z, +x, -x, +y, -y."""
    faces = []
    for z, y in (((0, 0, 1), (0, 1, 0)), ((0, 0, -1), (0, 1, 0)), ((1, 0, 0), (0, 1, 0)),
                 ((-1, 0, 0), (0, 1, 0)), ((0, 1, 0), (0, 0, -1)), ((0, -1, 0), (0, 0, 1))):
        z, y = np.array(z, float), np.array(y, float)
        faces.append(np.stack([np.cross(y, z), y, z]))
    return faces


def cubemap_cameras(face: int, centre=(0.0, 0.0, 0.0)) -> Cameras:
    """Six square pinhole views (90 degree field of view, face x face pixels) around one centre;
    use with settings pinhole={v: (face / 2, face / 2, face / 2, face / 2)}."""
    c = np.asarray(centre, dtype=np.float64)
    Rs = cube_rotations()
    return _pack_cams(Rs, [c] * 6, [[face, face]] * 6)


def yaw_cameras(n_views: int, width: int, height: int, seed: int) -> Cameras:
    """cfg3/M cameras: centres uniform in [-0.5, 0.5]^3, yaw uniform in [0, 2pi)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.5, 0.5, size=(n_views, 3))
    yaws = rng.uniform(0.0, 2.0 * np.pi, size=n_views)
    return _pack_cams([yaw_matrix(a) for a in yaws], centres, [[width, height]] * n_views)


def random_rotation(rng) -> np.ndarray:
    """Haar-uniform rotation from the QR factorisation of a Gaussian matrix."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def uneven_cameras(n_views: int, seed: int,
                   sizes=((1024, 512), (2048, 1024), (4096, 2048))) -> Cameras:
    """cfg4 cameras: sizes drawn from ``sizes``, uniformly random rotations, centres in the cube."""
    rng = np.random.default_rng(seed)
    wh = [sizes[i] for i in rng.integers(0, len(sizes), size=n_views)]
    rots = [random_rotation(rng) for _ in range(n_views)]
    centres = rng.uniform(-0.5, 0.5, size=(n_views, 3))
    return _pack_cams(rots, centres, wh)


def upstream_gradient(cams: Cameras, seed: int) -> np.ndarray:
    """N(0,1) gradient of the loss w.r.t. every output pixel, layout [V][3][H][W] concatenated."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(3 * cams.pixels).astype(np.float32)


def sparse_upstream_gradient(cams: Cameras, seed: int, n_pixels: int):
    """N(0,1) gradient on ``n_pixels`` random pixels per view, zero elsewhere.

    Returns (grad [V][3][H][W] concatenated, pixel list int32 [n][3] of (view, x, y)).
    Used at full resolution so the CPU reference only has to evaluate the sampled pixels.
    """
    rng = np.random.default_rng(seed)
    grad = np.zeros(3 * cams.pixels, dtype=np.float32)
    pix = []
    base = 0
    for v in range(cams.n_views):
        w, h = int(cams.wh[v, 0]), int(cams.wh[v, 1])
        flat = rng.choice(w * h, size=min(n_pixels, w * h), replace=False)
        flat.sort()
        for c in range(3):
            grad[base + c * w * h + flat] = rng.standard_normal(len(flat))
        pix.append(np.stack([np.full(len(flat), v), flat % w, flat // w], axis=1))
        base += 3 * w * h
    return grad, np.ascontiguousarray(np.concatenate(pix, axis=0), dtype=np.int32)


DEFAULT_SETTINGS = dict(tile=16, batch=0, batch_bwd=0, near=0.2, far=1.0e4, dilation=0.3, pole_eps=1.0e-4,
                        bg=(0.0, 0.0, 0.0))


def config(name: str, n: int | None = None, scale: int = 1):
    """Scene + cameras of a named workload. ``n`` overrides the Gaussian count and ``scale``
    divides every view's resolution (for reduced-size parity cases)."""
    def sz(w, h):
        return w // scale, h // scale
    if name == "cfg0":
        sc = sphere_scene(n or 2000, 0, seed=0)
        cams = identity_cameras(*sz(256, 128))
    elif name == "cfg1":
        sc = sphere_scene(n or 100_000, 3, seed=1)
        cams = identity_cameras(*sz(2048, 1024))
    elif name == "cfg2":
        sc = roaming_scene(n or 500_000, 3, seed=2)
        cams = identity_cameras(*sz(4096, 2048))
    elif name == "cfg3":
        sc = roaming_scene(n or 1_000_000, 3, seed=3)
        cams = yaw_cameras(8, *sz(2048, 1024), seed=3)
    elif name == "cfg4":
        sc = roaming_scene(n or 300_000, 3, seed=4)
        cams = uneven_cameras(16, seed=4, sizes=tuple(sz(w, h) for w, h in
                                                      ((1024, 512), (2048, 1024), (4096, 2048))))
    elif name == "M":
        sc = roaming_scene(n or 500_000, 3, seed=5)
        cams = yaw_cameras(8, *sz(2048, 1024), seed=5)
    else:
        raise KeyError(name)
    return sc, cams, dict(DEFAULT_SETTINGS)


CONFIG_SEEDS = {"cfg0": 0, "cfg1": 1, "cfg2": 2, "cfg3": 3, "cfg4": 4, "M": 5}
