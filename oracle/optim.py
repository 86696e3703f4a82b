"""Oracle for the on-device training step around the rasterizer: the L1 image loss and one Adam
update of the Gaussian parameters.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The paper trains with the 3DGS recipe (its implementation details keep the 3DGS
hyper-parameters): an image loss on the rendered panorama and Adam over the raw parameters,
with scales and opacities stored before their activations (scale = exp(raw), opacity =
sigmoid(raw)) and the rotation quaternion normalised inside the rasterizer.  Readings:

* Loss: L1 = mean over all rendered values (views, channels, pixels) of |C - C_target|; its
  gradient is sign(C - C_target) / count with sign(0) = 0.  (3DGS mixes in a D-SSIM term; only the
  L1 part is built here.)
* Adam (Kingma & Ba, in the form PyTorch's optimiser uses and 3DGS relies on): with t the step
  number after incrementing,
  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
  p = p - (lr / (1 - b1^t)) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
* Parameter groups and their learning rates: means, raw scales, quaternions, raw opacities, the
  SH DC planes (k = 0) and the remaining SH planes.
"""
from __future__ import annotations

import numpy as np

GROUPS = ("means", "scales", "quats", "opacities", "sh_dc", "sh_rest")


def l1_loss(rgb, target):
    """(loss, dL/drgb) of the mean absolute difference, in double."""
    d = np.asarray(rgb, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    n = d.size
    return float(np.abs(d).sum() / n), np.sign(d) / n


def activate(raw):
    """Activated parameters the rasterizer reads, from raw ones (dict of SoA arrays)."""
    return dict(means=raw["means"], scales=np.exp(raw["scales"]), quats=raw["quats"],
                opacities=1.0 / (1.0 + np.exp(-raw["opacities"])), sh=raw["sh"])


def raw_gradients(raw, grads):
    """Chain the gradients w.r.t. the activated parameters through the activations."""
    s = np.exp(raw["scales"])
    o = 1.0 / (1.0 + np.exp(-raw["opacities"]))
    return dict(means=grads["means"], scales=grads["scales"] * s, quats=grads["quats"],
                opacities=grads["opacities"] * o * (1.0 - o), sh=grads["sh"])


def adam_step(raw, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam update.  raw, grads (w.r.t. the activated parameters), m, v: dicts of SoA arrays
    (float64 copies are made); t: step number before this update; lr: six learning rates in the
    order of GROUPS.  Returns (raw, m, v) after the update."""
    t = t + 1
    g = raw_gradients(raw, grads)
    bc1, bc2 = 1.0 - beta1 ** t, 1.0 - beta2 ** t
    out_p, out_m, out_v = {}, {}, {}
    for name in ("means", "scales", "quats", "opacities", "sh"):
        gg = np.asarray(g[name], dtype=np.float64)
        mm = beta1 * np.asarray(m[name], dtype=np.float64) + (1.0 - beta1) * gg
        vv = beta2 * np.asarray(v[name], dtype=np.float64) + (1.0 - beta2) * gg * gg
        if name == "sh":
            rate = np.full(gg.shape, lr[5])
            rate[:3] = lr[4]
        else:
            rate = lr[GROUPS.index(name)]
        p = np.asarray(raw[name], dtype=np.float64) - (rate / bc1) * mm / (np.sqrt(vv) / np.sqrt(bc2) + eps)
        out_p[name], out_m[name], out_v[name] = p, mm, vv
    return out_p, out_m, out_v
