"""Oracle for the densification step of ODGS (Sec. 3.3 and the implementation details of the
appendix): per-Gaussian statistics gathered during the backward pass, and the clone / split /
prune step that consumes them.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/`` and nothing on the
GPU product path.

Readings (the paper states only the threshold rule and its constants; the rest is the 3DGS
densification the method says it follows):

* Statistic: for every view in which a Gaussian is visible (kept by the culling tests and covering
  at least one tile), add the length of the gradient of the loss with respect to its 2D mean,
  measured in normalised image units (u_ndc = 2u/W - 1, v_ndc = 2v/H - 1, so
  dL/du_ndc = dL/du * W/2), add that view's threshold tau, and count the view.
* Threshold (Sec. 3.3): tau = tau_min + (1 - cos theta) (tau_max - tau_min), theta the elevation of
  the Gaussian's mean seen from that view's camera (cos theta = sqrt(mu_x^2 + mu_z^2) / |mu|);
  tau_min = 2e-5, tau_max = 1e-4 (appendix).  A Gaussian is selected when its mean gradient
  reaches its mean threshold; both means share the view count, so the test is taken on the sums,
  grad_sum >= tau_sum, in float32 on both sides.
* Clone (selected, largest scale <= percent_dense * extent), split (selected, largest scale
  above it) into two children at m + R(q) (s * xi) with scales s / 1.6 and every other parameter
  copied, the split parent removed; prune every resulting Gaussian with opacity below
  min_opacity, or (when max_scale_frac > 0) with largest scale above max_scale_frac * extent.
  percent_dense = 1e-3 (appendix).  The random draws xi are inputs ([2][3][n], one per child).
* Output order: surviving originals, surviving clones, surviving first children, surviving second
  children, each in parent index order.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

TAU_MIN = 2e-5
TAU_MAX = 1e-4
PERCENT_DENSE = 1e-3
MIN_OPACITY = 0.005
SPLIT_SHRINK = 1.6  # children scales are the parent's divided by 0.8 * (number of children = 2)


def threshold(cos_theta, tau_min=TAU_MIN, tau_max=TAU_MAX):
    """Elevation-dependent gradient threshold of Sec. 3.3 (FP64)."""
    return tau_min + (1.0 - cos_theta) * (tau_max - tau_min)


def visibility(scene, cams, settings) -> np.ndarray:
    """[V][N] bool: kept by the culling tests and covering at least one tile of that view."""
    rows = O.project(scene, cams, settings)
    area = rows[..., O.F_RECT + 1] * rows[..., O.F_RECT + 3]
    return (rows[..., O.F_KEPT] > 0) & (area > 0)


def stats_from(rows: np.ndarray, g2d: np.ndarray, wh: np.ndarray, tau_min=TAU_MIN, tau_max=TAU_MAX):
    """Statistics from projection rows [V][N][NF] and per-item 2D gradients [V][N][9] (FP64).

    Returns grad_sum [N], tau_sum [N], count [N] (summed over views)."""
    area = rows[..., O.F_RECT + 1] * rows[..., O.F_RECT + 3]
    vis = (rows[..., O.F_KEPT] > 0) & (area > 0)
    W = wh[:, 0].astype(np.float64)[:, None]
    H = wh[:, 1].astype(np.float64)[:, None]
    gnorm = np.sqrt((g2d[..., 0] * (0.5 * W)) ** 2 + (g2d[..., 1] * (0.5 * H)) ** 2)
    mu = rows[..., O.F_MU:O.F_MU + 3]
    with np.errstate(invalid="ignore", divide="ignore"):
        cos_t = np.sqrt(mu[..., 0] ** 2 + mu[..., 2] ** 2) / rows[..., O.F_R]
    tau = threshold(cos_t, tau_min, tau_max)
    grad_sum = np.where(vis, gnorm, 0.0).sum(axis=0)
    tau_sum = np.where(vis, tau, 0.0).sum(axis=0)
    count = vis.sum(axis=0).astype(np.int32)
    return grad_sum, tau_sum, count


def stats(scene, cams, settings, dL, mode: int = 32, pix=None, tau_min=TAU_MIN, tau_max=TAU_MAX):
    """Densification statistics of one backward pass with upstream image gradient dL."""
    g = O.backward(scene, cams, settings, dL, mode=mode, pix=pix, want_g2d=True)
    rows = O.project(scene, cams, settings)
    return stats_from(rows, g["g2d"], np.asarray(cams.wh), tau_min, tau_max)


def _rotation(q):
    """Rotation matrices [n][3][3] from quaternions (w, x, y, z) [4][n], normalised (FP64)."""
    q = q / np.linalg.norm(q, axis=0, keepdims=True)
    w, x, y, z = q
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], axis=-1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], axis=-1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=-1),
    ], axis=-2)


def densify(means, scales, quats, opacities, sh, grad_sum, tau_sum, count, noise, extent,
            percent_dense=PERCENT_DENSE, min_opacity=MIN_OPACITY, max_scale_frac=0.0):
    """One clone / split / prune step.  Parameter arrays are SoA float32 ([3][n], [3][n], [4][n],
    [n], [K*3][n]); statistics float32 / int32; noise float32 [2][3][n].

    Returns dict with the new SoA arrays (float32; children positions computed in FP64 and
    rounded), ``src`` (int32 parent index of every output), and ``counts`` = (originals, clones,
    first children, second children)."""
    f32 = np.float32
    means, scales, quats = (np.asarray(a, dtype=f32) for a in (means, scales, quats))
    opacities, sh = np.asarray(opacities, dtype=f32), np.asarray(sh, dtype=f32)
    grad_sum, tau_sum = np.asarray(grad_sum, dtype=f32), np.asarray(tau_sum, dtype=f32)
    count = np.asarray(count, dtype=np.int32)
    n = means.shape[1]
    selected = (count > 0) & (grad_sum >= tau_sum)
    smax = scales.max(axis=0)
    big = f32(percent_dense) * f32(extent)
    clone = selected & (smax <= big)
    split = selected & (smax > big)
    child_scales = scales / f32(SPLIT_SHRINK)

    def pruned(op, smax_):
        p = op < f32(min_opacity)
        if max_scale_frac > 0:
            p = p | (smax_ > f32(max_scale_frac) * f32(extent))
        return p

    drop = pruned(opacities, smax)
    drop_child = pruned(opacities, child_scales.max(axis=0))
    idx = np.arange(n)
    seg = [idx[~split & ~drop], idx[clone & ~drop], idx[split & ~drop_child], idx[split & ~drop_child]]
    src = np.concatenate(seg).astype(np.int32)
    R = _rotation(quats.astype(np.float64))
    out_m = [means[:, seg[0]], means[:, seg[1]]]
    out_s = [scales[:, seg[0]], scales[:, seg[1]]]
    for c in (0, 1):
        p = seg[2 + c]
        local = scales[:, p].astype(np.float64) * noise[c][:, p].astype(np.float64)      # [3][k]
        off = np.einsum("kij,jk->ik", R[p], local)
        out_m.append((means[:, p].astype(np.float64) + off).astype(f32))
        out_s.append(child_scales[:, p])
    return dict(
        means=np.concatenate(out_m, axis=1), scales=np.concatenate(out_s, axis=1),
        quats=quats[:, src], opacities=opacities[src], sh=sh[:, src], src=src,
        counts=tuple(len(s) for s in seg),
    )
