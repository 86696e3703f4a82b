"""Training step around the rasterizer on the device: L1 image loss and Adam (the 3DGS recipe the
paper trains with), both in the HIP kernels of ``libodgs.so``.

Parameters are kept raw (log-scales, opacity logits) as 3DGS stores them; the Adam kernel chains
the rasterizer's gradients through the activations and rewrites the activated tensors the
rasterizer reads, so one captured HIP graph (``LossTrainStep``) is a whole training iteration:
bin, forward, loss, backward, optimiser update.
"""
from __future__ import annotations

import ctypes

import torch

from . import _odgs as B
from .rasterizer import Rasterizer, TrainStep

# 3DGS defaults: position 1.6e-4 (times the scene extent), scaling 5e-3, rotation 1e-3,
# opacity 5e-2, SH DC 2.5e-3 and higher SH 2.5e-3 / 20.
DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 2.5e-3 / 20)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pp(ts) -> B.ParamPtrs:
    return B.ParamPtrs(*[t.data_ptr() for t in ts])


class GaussianParams:
    """Raw parameters, their activated copies (what the rasterizer reads), Adam moments, learning
    rates (device float[6]) and the device step counter."""

    def __init__(self, means, log_scales, quats, logit_opacities, sh, sh_degree: int, lr=DEFAULT_LR,
                 betas=(0.9, 0.999), eps=1e-15):
        self.raw = tuple(t.detach().float().contiguous().clone() for t in (means, log_scales, quats, logit_opacities, sh))
        self.sh_degree = int(sh_degree)
        self.n = int(self.raw[0].shape[1])
        dev = self.raw[0].device
        # initial activation (set-up only; afterwards the Adam kernel keeps these current)
        self.act = (self.raw[0].clone(), torch.exp(self.raw[1]), self.raw[2].clone(), torch.sigmoid(self.raw[3]),
                    self.raw[4].clone())
        self.m = tuple(torch.zeros_like(t) for t in self.raw)
        self.v = tuple(torch.zeros_like(t) for t in self.raw)
        self.lr = torch.tensor(lr, dtype=torch.float32, device=dev)
        self.step_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.hyper = B.AdamHyper(float(betas[0]), float(betas[1]), float(eps))
        self._p = [_pp(self.raw), _pp(self.act), None, _pp(self.m), _pp(self.v)]

    def adam_step(self, grads):
        """One update from gradients w.r.t. the activated parameters (as the rasterizer returns)."""
        for g, a in zip(grads, self.act):
            if g.shape != a.shape or not g.is_contiguous() or g.dtype != torch.float32:
                raise ValueError("gradients must match the parameters (contiguous float32)")
        B.odgs_adam_step(self.n, self.sh_degree, self._p[0], self._p[1], _pp(grads), self._p[3], self._p[4],
                         _ptr(self.lr), _ptr(self.step_count), self.hyper, _stream())


class L1Loss:
    """mean |rgb - target| and its gradient, with preallocated outputs (graph-capturable)."""

    def __init__(self, count: int, device="cuda"):
        self.count = int(count)
        self.dL = torch.empty(self.count, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.ws_bytes = B.odgs_l1_loss_workspace_bytes(self.count)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def __call__(self, rgb: torch.Tensor, target: torch.Tensor):
        if rgb.numel() != self.count or target.numel() != self.count:
            raise ValueError("expected %d values" % self.count)
        B.odgs_l1_loss(_ptr(rgb), _ptr(target), self.count, _ptr(self.dL), _ptr(self.loss), _ptr(self.ws),
                       self.ws_bytes, _stream())
        return self.loss, self.dL


class LossTrainStep(TrainStep):
    """A whole training iteration over all views: bin, forward, L1 loss against `target`, reverse
    compositing, projection adjoint and the Adam update of `params`.  Capture once, replay per
    iteration (targets and poses can be rewritten in place between replays)."""

    def __init__(self, rast: Rasterizer, params: GaussianParams, cams: torch.Tensor, target: torch.Tensor,
                 stats=None):
        self.loss_fn = L1Loss(3 * rast.pixels, device=rast.device)
        super().__init__(rast, params.act, cams, self.loss_fn.dL, stats=stats)
        self.gp = params
        self.target = target

    def run(self):
        self.bin()
        self.fwd()
        self.loss_fn(self.rgb, self.target)
        self.composite_bwd()
        self.project_bwd()
        self.gp.adam_step(self.grads)

    @property
    def loss(self) -> torch.Tensor:
        return self.loss_fn.loss
