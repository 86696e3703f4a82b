"""Densification for omnidirectional images (Sec. 3.3): statistics gathered by the backward
pass and the clone / split / prune step, both in the HIP kernels of ``libodgs.so``.

The gradient threshold depends on the Gaussian's elevation seen from each camera,
tau = tau_min + (1 - cos theta) (tau_max - tau_min) (tau_min = 2e-5, tau_max = 1e-4 in the
paper's implementation details), which keeps Gaussians near the poles, drawn larger by the ERP
map, from being densified too eagerly.  The clone / split / prune rules are those of 3DGS that
the method keeps (percent_dense = 1e-3).
"""
from __future__ import annotations

import ctypes

import torch

from . import _odgs as B

TAU_MIN = 2e-5
TAU_MAX = 1e-4
PERCENT_DENSE = 1e-3
MIN_OPACITY = 0.005


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class DensifyStats:
    """Per-Gaussian accumulators: grad_sum (sum over visible views of the 2D-mean gradient
    length in normalised image units), tau_sum (sum of the per-view thresholds), count (visible
    views).  Pass to Rasterizer.render_bwd / project_bwd / TrainStep; clear with reset()."""

    def __init__(self, n: int, device="cuda", tau_min: float = TAU_MIN, tau_max: float = TAU_MAX):
        self.grad_sum = torch.zeros(n, dtype=torch.float32, device=device)
        self.tau_sum = torch.zeros(n, dtype=torch.float32, device=device)
        self.count = torch.zeros(n, dtype=torch.int32, device=device)
        self.tau_min, self.tau_max = float(tau_min), float(tau_max)
        self._acc = B.DensifyAcc(self.grad_sum.data_ptr(), self.tau_sum.data_ptr(), self.count.data_ptr(),
                                 self.tau_min, self.tau_max)

    @property
    def n(self) -> int:
        return int(self.grad_sum.shape[0])

    def acc(self, n: int) -> B.DensifyAcc:
        if n != self.n:
            raise ValueError("statistics hold %d Gaussians, the rasterizer %d" % (self.n, n))
        return self._acc

    def reset(self):
        self.grad_sum.zero_()
        self.tau_sum.zero_()
        self.count.zero_()


def densify(params, stats: DensifyStats, noise: torch.Tensor, extent: float, sh_degree: int,
            percent_dense: float = PERCENT_DENSE, min_opacity: float = MIN_OPACITY, max_scale_frac: float = 0.0):
    """One clone / split / prune step.

    params: (means [3,N], scales [3,N], quats [4,N], opacities [N], sh [K*3,N]) float32 device
    tensors; noise: float32 [2, 3, N] standard normal draws for the two children of a split.
    Returns (new params tuple with M columns, src int32 [M] parent indices, counts tuple of
    (originals, clones, first children, second children)).  Synchronises once to read M."""
    means, scales, quats, opac, sh = params
    n = int(means.shape[1])
    dev = means.device
    for t in (*params, stats.grad_sum, stats.tau_sum, stats.count, noise):
        if not t.is_contiguous() or t.device != dev:
            raise ValueError("all tensors must be contiguous and on one device")
    if tuple(noise.shape) != (2, 3, n) or noise.dtype != torch.float32:
        raise ValueError("noise must be float32 [2, 3, %d]" % n)
    stats.acc(n)
    cap = max(2 * n, 1)
    out = (torch.empty((3, cap), dtype=torch.float32, device=dev), torch.empty((3, cap), dtype=torch.float32, device=dev),
           torch.empty((4, cap), dtype=torch.float32, device=dev), torch.empty(cap, dtype=torch.float32, device=dev),
           torch.empty((sh.shape[0], cap), dtype=torch.float32, device=dev))
    src = torch.empty(cap, dtype=torch.int32, device=dev)
    counts = torch.empty(4, dtype=torch.int64, device=dev)
    ws_bytes = B.odgs_densify_workspace_bytes(n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    p = B.DensifyParams(float(extent), float(percent_dense), float(min_opacity), float(max_scale_frac))
    B.odgs_densify(n, sh_degree, *[_ptr(t) for t in params], _ptr(stats.grad_sum), _ptr(stats.tau_sum),
                   _ptr(stats.count), _ptr(noise), p, cap, *[_ptr(t) for t in out], _ptr(src), _ptr(counts),
                   _ptr(ws), ws_bytes, _stream())
    c = tuple(int(x) for x in counts.cpu())
    m = sum(c)
    new = tuple(t[..., :m].contiguous() for t in out)
    return new, src[:m], c
