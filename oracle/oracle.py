"""Python access to the CPU oracle (``oracle/odgs_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``.  The GPU product path never imports this module.

All parameters are passed to the C code as float64 copies of the scene arrays (the float32
inputs of the GPU path convert exactly), so finite differences can perturb them in double.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "odgs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

NF = 41  # doubles per projection row, see oracle_project in the C source
F_KEPT, F_CULL, F_DEPTH, F_DEPTH_BITS, F_U, F_V = 0, 1, 2, 3, 4, 5
F_CONIC, F_OPAC, F_PMIN, F_RGB, F_RECT, F_COV2, F_J, F_COV3, F_MU, F_R, F_RGB_RAW = 6, 9, 10, 11, 14, 18, 21, 27, 33, 36, 37
F_BETA = 40


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain C++17 + OpenMP, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ODGS_ORACLE_LIB")  # another build of the same source (sanitizer test)
        if not path:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        scene_args = [P, P, P, P, P, i64, i32, P, P, i32, P]
        L.oracle_num_threads.restype = i32
        L.oracle_sh_basis.argtypes = [P, i64, i32, P]
        L.oracle_project.argtypes = scene_args + [P]
        L.oracle_project.restype = i32
        L.oracle_keys.argtypes = scene_args + [P, P, i64]
        L.oracle_keys.restype = i64
        L.oracle_render.argtypes = scene_args + [i32, i32, P, i64, P, P, P, P, P, P]
        L.oracle_render.restype = i32
        L.oracle_backward.argtypes = scene_args + [i32, P, i64, P, P, P, P, P, P, P, P, i32]
        L.oracle_backward.restype = i32
        L.oracle_project_adjoint.argtypes = scene_args + [P, P, P, P, P, P]
        L.oracle_project_adjoint.restype = i32
        L.oracle_sph_eval.argtypes = scene_args + [P, i64, P]
        L.oracle_sph_eval.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def settings_array(settings: dict) -> np.ndarray:
    """Settings as doubles.  The real-valued ones are first rounded to float32, the precision in
    which the rasterizer's C interface receives them, so both sides use identical constants."""
    bg = settings.get("bg", (0.0, 0.0, 0.0))
    vals = [settings["near"], settings["far"], settings["dilation"], settings["pole_eps"], bg[0], bg[1], bg[2]]
    vals = [float(np.float32(x)) for x in vals]
    # pinhole views: {view: (fx, fy, cx, cy)}, appended as (view, fx, fy, cx, cy) records
    pin = settings.get("pinhole") or {}
    tail = [float(len(pin))]
    for v in sorted(pin):
        tail += [float(v)] + [float(np.float32(x)) for x in pin[v]]
    # footprint model: "affine" (the paper's local affine approximation) or "spherical" (exact
    # per-ray maximum of the 3D Gaussian in equirectangular views)
    fp = settings.get("footprint", "affine")
    if fp not in ("affine", "spherical"):
        raise ValueError("footprint must be 'affine' or 'spherical'")
    tail.append(1.0 if fp == "spherical" else 0.0)
    return np.array([settings["tile"], *vals, *tail], dtype=np.float64)


class _Args:
    def __init__(self, scene, cams, settings):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.keep = [f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacities), f(scene.sh),
                     f(cams.cams), np.ascontiguousarray(cams.wh, dtype=np.int32), settings_array(settings)]
        self.n = scene.means.shape[1]
        self.deg = scene.sh_degree
        self.V = cams.cams.shape[0]
        self.wh = cams.wh

    def tuple(self):
        m, s, q, o, sh, c, wh, st = self.keep
        return (_p(m), _p(s), _p(q), _p(o), _p(sh), self.n, self.deg, _p(c), _p(wh), self.V, _p(st))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def sh_basis(dirs: np.ndarray, K: int) -> np.ndarray:
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((d.shape[0], K))
    lib().oracle_sh_basis(_p(d), d.shape[0], K, _p(out))
    return out


def project(scene, cams, settings) -> np.ndarray:
    """Projection rows [V][N][NF] (see the field constants above)."""
    a = _Args(scene, cams, settings)
    out = np.zeros((a.V, a.n, NF))
    lib().oracle_project(*a.tuple(), _p(out))
    return out


def keys(scene, cams, settings):
    """Sorted (key uint64, gaussian index uint32) list over all views."""
    a = _Args(scene, cams, settings)
    P = lib().oracle_keys(*a.tuple(), None, None, 0)
    k = np.zeros(max(P, 1), dtype=np.uint64)
    v = np.zeros(max(P, 1), dtype=np.uint32)
    P2 = lib().oracle_keys(*a.tuple(), _p(k), _p(v), P)
    assert P2 == P
    return k[:P], v[:P]


def render(scene, cams, settings, mode: int = 32, band: bool = False, pix: np.ndarray | None = None):
    """Brute-force (or band) render.  Returns dict of rgb, T, ncontrib, margin, sig, depth (the
    alpha-weighted sort depth, sum of alpha_j T_j d_j over the contributors).

    Full image: rgb is [V][3][H][W] flattened and concatenated over views, the others [V][H][W].
    With ``pix`` (int32 [n][3] rows of view, x, y): rgb [n][3], the others [n].
    """
    a = _Args(scene, cams, settings)
    if pix is None:
        npx = int(np.sum(a.wh[:, 0].astype(np.int64) * a.wh[:, 1]))
        pp = None
        rgb = np.zeros(3 * npx)
    else:
        pp = np.ascontiguousarray(pix, dtype=np.int32)
        npx = pp.shape[0]
        rgb = np.zeros((npx, 3))
    T = np.zeros(npx)
    nc = np.zeros(npx, dtype=np.int32)
    margin = np.zeros(npx)
    sig = np.zeros(npx, dtype=np.uint64)
    depth = np.zeros(npx)
    lib().oracle_render(*a.tuple(), mode, int(band), _p(pp), npx if pp is not None else 0,
                        _p(rgb), _p(T), _p(nc), _p(margin), _p(sig), _p(depth))
    return dict(rgb=rgb, T=T, ncontrib=nc, margin=margin, sig=sig, depth=depth)


def spherical(settings) -> bool:
    return settings.get("footprint", "affine") == "spherical"


def backward(scene, cams, settings, dL: np.ndarray, mode: int = 32, pix: np.ndarray | None = None,
             want_g2d: bool = False, band: bool = False):
    """Gradient of sum(dL * rgb) w.r.t. every parameter (float64), and optionally the per-item
    gradients of the compositor's inputs: affine footprint g2d [V][N][9] (u, v, conic a, b, c,
    opacity, r, g, b); spherical footprint g2d [V][N][13] (mu^, A, opacity, rgb) and g2d_kernel
    [V][N][13] (mu^, Sigma~, opacity, rgb; the reverse compositor's layout).  mode 32 or 64 as
    in render; mode 33: mode 32's contributors with each alpha taken at the float pass's own
    exponent.  band: candidates from the tile lists instead of every kept Gaussian (the same
    contributor lists, much faster)."""
    a = _Args(scene, cams, settings)
    n, K = a.n, (a.deg + 1) ** 2
    gm, gs, gq = np.zeros((3, n)), np.zeros((3, n)), np.zeros((4, n))
    go, gsh = np.zeros(n), np.zeros((K * 3, n))
    sph = spherical(settings)
    g2d = np.zeros((a.V, n, 13 if sph else 9)) if want_g2d else None
    g2dk = np.zeros((a.V, n, 13)) if (want_g2d and sph) else None
    d = np.ascontiguousarray(dL, dtype=np.float64)
    pp = None if pix is None else np.ascontiguousarray(pix, dtype=np.int32)
    lib().oracle_backward(*a.tuple(), mode, _p(pp), 0 if pp is None else pp.shape[0], _p(d),
                          _p(gm), _p(gs), _p(gq), _p(go), _p(gsh), _p(g2d), _p(g2dk), int(band))
    out = dict(means=gm, scales=gs, quats=gq, opacities=go, sh=gsh)
    if want_g2d:
        out["g2d"] = g2d
        if sph:
            out["g2d_kernel"] = g2dk
    return out


def sph_eval(scene, cams, settings, queries: np.ndarray) -> np.ndarray:
    """Spherical footprint at (view, x, y, gaussian) rows: [n][6] = (m by the definition,
    b = d^T A mu^, m by the tangent-frame form in double, float exponent (0 if rejected), float
    acceptance, kept)."""
    a = _Args(scene, cams, settings)
    q = np.ascontiguousarray(queries, dtype=np.int32).reshape(-1, 4)
    out = np.zeros((q.shape[0], 6))
    lib().oracle_sph_eval(*a.tuple(), _p(q), q.shape[0], _p(out))
    return out


def g2d_to_sigma(rows: np.ndarray, g2d: np.ndarray) -> np.ndarray:
    """Per-item 2D gradients with the shape entries taken w.r.t. the inverse covariance
    (a, b, c) -> the same w.r.t. the covariance (uu, uv, vv), both off-diagonals as one shared
    variable: with M = [[a, b], [b, c]] and G = [[ga, gb/2], [gb/2, gc]], dL/dSigma = -M G M."""
    a, b, c = (rows[..., F_CONIC + k] for k in range(3))
    ga, gb, gc = g2d[..., 2], 0.5 * g2d[..., 3], g2d[..., 4]
    # (M G)_{ij} then (M G M)
    mg00, mg01 = a * ga + b * gb, a * gb + b * gc
    mg10, mg11 = b * ga + c * gb, b * gb + c * gc
    s00 = mg00 * a + mg01 * b
    s01 = mg00 * b + mg01 * c
    s11 = mg10 * b + mg11 * c
    out = np.array(g2d, dtype=np.float64, copy=True)
    out[..., 2], out[..., 3], out[..., 4] = -s00, -2.0 * s01, -s11
    return out


def project_adjoint(scene, cams, settings, g2d_sigma: np.ndarray):
    """Parameter gradients from per-item gradients in the reverse compositor's layout, summed
    over views: affine [V][N][9] in covariance terms (u, v, Sigma_uu, Sigma_uv (shared),
    Sigma_vv, opacity, r, g, b); spherical footprint [V][N][13] (mu^, Sigma~ (shared off-diagonals),
    opacity, rgb)."""
    a = _Args(scene, cams, settings)
    n, K = a.n, (a.deg + 1) ** 2
    gm, gs, gq = np.zeros((3, n)), np.zeros((3, n)), np.zeros((4, n))
    go, gsh = np.zeros(n), np.zeros((K * 3, n))
    g = np.ascontiguousarray(g2d_sigma, dtype=np.float64)
    assert g.shape == (a.V, n, 13 if spherical(settings) else 9)
    lib().oracle_project_adjoint(*a.tuple(), _p(g), _p(gm), _p(gs), _p(gq), _p(go), _p(gsh))
    return dict(means=gm, scales=gs, quats=gq, opacities=go, sh=gsh)
