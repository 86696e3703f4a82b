"""Small helpers shared by the tests (scene construction only; no rasterizer arithmetic)."""
import numpy as np

from paper_2410_20686_amd import scenes


def make_scene(means, scales, quats=None, opac=None, sh=None, sh_degree=0, dtype=np.float64):
    means = np.asarray(means, dtype=np.float64).reshape(-1, 3).T
    n = means.shape[1]
    scales = np.broadcast_to(np.asarray(scales, dtype=np.float64).reshape(-1, 3), (n, 3)).T
    if quats is None:
        quats = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    quats = np.broadcast_to(np.asarray(quats, dtype=np.float64).reshape(-1, 4), (n, 4)).T
    if opac is None:
        opac = np.full(n, 0.5)
    opac = np.broadcast_to(np.asarray(opac, dtype=np.float64), (n,))
    K = (sh_degree + 1) ** 2
    if sh is None:
        sh = np.zeros((K * 3, n))
    sh = np.asarray(sh, dtype=np.float64).reshape(K * 3, n)
    c = lambda a: np.ascontiguousarray(a, dtype=dtype)
    return scenes.Scene(c(means), c(scales), c(quats), c(opac), c(sh), sh_degree)


def settings(**kw):
    s = dict(scenes.DEFAULT_SETTINGS)
    s.update(kw)
    return s


def cams_from(R_list, t_list, wh):
    cams = np.zeros((len(R_list), 12))
    for v, (R, t) in enumerate(zip(R_list, t_list)):
        cams[v, :9] = np.asarray(R).reshape(-1)
        cams[v, 9:] = t
    return scenes.Cameras(cams, np.asarray(wh, dtype=np.int32).reshape(-1, 2))


def image(rgb_flat, cams, v):
    """View v of a concatenated [V][3][H][W] buffer as an array [3][H][W]."""
    off = 0
    for u in range(v):
        off += 3 * int(cams.wh[u, 0]) * int(cams.wh[u, 1])
    w, h = int(cams.wh[v, 0]), int(cams.wh[v, 1])
    return np.asarray(rgb_flat[off:off + 3 * w * h]).reshape(3, h, w)


def plane(buf_flat, cams, v):
    """View v of a concatenated [V][H][W] buffer as an array [H][W]."""
    off = 0
    for u in range(v):
        off += int(cams.wh[u, 0]) * int(cams.wh[u, 1])
    w, h = int(cams.wh[v, 0]), int(cams.wh[v, 1])
    return np.asarray(buf_flat[off:off + w * h]).reshape(h, w)


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, -s], [0.0, 1.0, 0.0], [s, 0.0, c]])
