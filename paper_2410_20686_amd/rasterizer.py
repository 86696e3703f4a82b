"""PyTorch front end of the gfx950 omnidirectional rasterizer.

PyTorch only provides device memory and the stream: every step of the rasterizer runs in the
HIP kernels of ``libodgs.so``, reached through the C ABI (``_odgs``).  There is no CPU path.

Tensor conventions (float32, contiguous, on the GPU):
  means [3, N], scales [3, N] (linear, > 0), quats [4, N] (w, x, y, z), opacities [N] in (0, 1),
  sh [K*3, N] with K = (degree+1)^2, cams [V, 12] (world-to-camera R row-major, then t).
Outputs: rgb flat [sum_v 3 H_v W_v] (view after view, each [3, H, W]) and T flat [sum_v H_v W_v].
"""
from __future__ import annotations

import ctypes

import torch

from . import _odgs as B

DEFAULT_SETTINGS = dict(tile=16, batch=0, batch_bwd=0, count_work=False, pinhole=None, footprint="affine",
                        schedule="queue", binning="auto", near=0.2, far=1.0e4, dilation=0.3, pole_eps=1.0e-4,
                        bg=(0.0, 0.0, 0.0))


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Rasterizer:
    """Plan and workspace of one workload shape: N Gaussians of one SH degree seen by views of
    the given sizes.  One forward may be in flight per rasterizer (the backward reads what the
    forward left in the workspace)."""

    def __init__(self, n: int, sh_degree: int, wh, settings: dict | None = None, pair_capacity: int | None = None,
                 device: str | torch.device = "cuda"):
        self.n = int(n)
        self.sh_degree = int(sh_degree)
        self.wh = [(int(w), int(h)) for w, h in wh]
        self.settings = dict(DEFAULT_SETTINGS)
        if settings:
            self.settings.update({k: v for k, v in settings.items() if k in DEFAULT_SETTINGS})
        self.device = torch.device(device)
        if pair_capacity is None:
            pair_capacity = max(1 << 16, 8 * self.n * len(self.wh))
        self.generation = 0
        self._alloc(int(pair_capacity))

    def _make_plan(self, capacity: int) -> B.Plan:
        """Plan for the current settings; settings["pinhole"] = {view: (fx, fy, cx, cy)} marks
        perspective views (the others are equirectangular)."""
        st = {k: v for k, v in self.settings.items() if k != "pinhole"}
        plan = B.odgs_plan_init(self.n, self.sh_degree, self.wh, B.make_settings(**st), capacity)
        for view, (fx, fy, cx, cy) in sorted((self.settings.get("pinhole") or {}).items()):
            B.odgs_plan_set_pinhole(plan, view, fx, fy, cx, cy)
        return plan

    def _alloc(self, capacity: int):
        self.capacity = min(capacity, (1 << 31) - 1)
        self.plan = self._make_plan(self.capacity)
        self.ws_bytes = B.odgs_workspace_bytes(self.plan)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        if self.ws.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")
        self.pixels = int(self.plan.pix_base[len(self.wh)])
        self.status_offset = B.odgs_status_offset(self.plan)

    def set_batches(self, batch: int, batch_bwd: int, count_work: bool | None = None):
        """Change the compositors' LDS batch sizes (and whether the forward records its work
        counters); the workspace, whose layout depends on neither, and its contents stay valid."""
        self.settings.update(batch=int(batch), batch_bwd=int(batch_bwd))
        if count_work is not None:
            self.settings["count_work"] = bool(count_work)
        plan = self._make_plan(self.capacity)
        if B.odgs_workspace_bytes(plan) != self.ws_bytes:
            raise RuntimeError("workspace layout changed with the batch sizes")
        self.plan = plan

    # ---------------------------------------------------------------------------------------
    def status(self) -> dict:
        """Read the device status record (synchronises with the current stream)."""
        raw = self.ws[self.status_offset:self.status_offset + ctypes.sizeof(B.Status)].cpu().numpy().tobytes()
        st = B.Status.from_buffer_copy(raw)
        return dict(flags=st.flags, n_pairs=st.n_pairs, n_pairs_stored=st.n_pairs_stored, n_visible=st.n_visible,
                    n_culled=st.n_culled, n_nonfinite=st.n_nonfinite, bin_gen=st.bin_gen, fwd_gen=st.fwd_gen)

    def _check_inputs(self, means, scales, quats, opac, sh, cams):
        K = (self.sh_degree + 1) ** 2
        shapes = ((means, (3, self.n)), (scales, (3, self.n)), (quats, (4, self.n)), (opac, (self.n,)),
                  (sh, (K * 3, self.n)), (cams, (len(self.wh), 12)))
        for t, shp in shapes:
            if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.ws.device:
                raise ValueError("expected contiguous float32 %s on %s, got %s %s on %s"
                                 % (shp, self.ws.device, tuple(t.shape), t.dtype, t.device))

    def bin(self, means, scales, quats, opac, sh, cams):
        """odgs_preprocess + odgs_bin_sort (no synchronisation)."""
        self._check_inputs(means, scales, quats, opac, sh, cams)
        s = _stream()
        B.odgs_preprocess(self.plan, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac), _ptr(sh), _ptr(cams),
                          _ptr(self.ws), self.ws_bytes, s)
        B.odgs_bin_sort(self.plan, _ptr(self.ws), self.ws_bytes, s)
        self.generation += 1  # new pair lists: no backward may use an earlier forward's state

    def bin_checked(self, means, scales, quats, opac, sh, cams) -> dict:
        """Bin, then read the status; on pair-list overflow grow the capacity and bin again."""
        self.bin(means, scales, quats, opac, sh, cams)
        st = self.status()
        if st["flags"] & B.STATUS_OVERFLOW:
            self._alloc(int(st["n_pairs"] * 1.25) + 1024)
            self.bin(means, scales, quats, opac, sh, cams)
            st = self.status()
            if st["flags"] & B.STATUS_OVERFLOW:
                raise RuntimeError("pair list still overflows after growing to %d" % self.capacity)
        return st

    def render_fwd(self, out_rgb: torch.Tensor | None = None, out_T: torch.Tensor | None = None, want_T=True,
                   out_depth: torch.Tensor | None = None):
        """Images (and final transmittance, whose complement is the accumulated alpha).  Pass
        out_depth (float32 [pixels]) to also get the alpha-weighted depth sum_j alpha_j T_j d_j."""
        if out_rgb is None:
            out_rgb = torch.empty(3 * self.pixels, dtype=torch.float32, device=self.device)
        if out_T is None and want_T:
            out_T = torch.empty(self.pixels, dtype=torch.float32, device=self.device)
        B.odgs_render_fwd(self.plan, _ptr(self.ws), self.ws_bytes, _ptr(out_rgb), _ptr(out_T), _ptr(out_depth),
                          _stream())
        self.generation += 1
        return out_rgb, out_T

    def render_bwd(self, means, scales, quats, opac, sh, cams, dL_drgb, grads=None, stats=None):
        """Parameter gradients (overwritten into ``grads`` if given); ``stats`` (a
        densify.DensifyStats) also accumulates the densification statistics."""
        self._check_inputs(means, scales, quats, opac, sh, cams)
        if dL_drgb.shape != (3 * self.pixels,) or dL_drgb.dtype != torch.float32 or not dL_drgb.is_contiguous():
            raise ValueError("dL_drgb must be contiguous float32 [%d]" % (3 * self.pixels))
        if grads is None:
            grads = tuple(torch.empty_like(t) for t in (means, scales, quats, opac, sh))
        B.odgs_render_bwd(self.plan, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac), _ptr(sh), _ptr(cams),
                          _ptr(self.ws), self.ws_bytes, _ptr(dL_drgb), *[_ptr(g) for g in grads],
                          None if stats is None else stats.acc(self.n), _stream())
        return grads

    # ---- inspection ---------------------------------------------------------------------------
    def records(self) -> torch.Tensor:
        out = torch.empty((self.n * len(self.wh), 12), dtype=torch.float32, device=self.device)
        B.odgs_debug_records(self.plan, _ptr(self.ws), _ptr(out), _stream())
        return out

    def keys(self):
        st = self.status()
        m = st["n_pairs_stored"]
        keys = torch.empty(max(m, 1), dtype=torch.int64, device=self.device)
        gauss = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        B.odgs_debug_keys(self.plan, _ptr(self.ws), m, _ptr(keys), _ptr(gauss), _stream())
        return keys[:m], gauss[:m]


    def composite_bwd(self, dL_drgb):
        B.odgs_composite_bwd(self.plan, _ptr(self.ws), self.ws_bytes, _ptr(dL_drgb), _stream())

    def project_bwd(self, means, scales, quats, opac, sh, cams, grads, stats=None):
        B.odgs_project_bwd(self.plan, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac), _ptr(sh), _ptr(cams),
                           _ptr(self.ws), self.ws_bytes, *[_ptr(g) for g in grads],
                           None if stats is None else stats.acc(self.n), _stream())

    def g2d(self) -> torch.Tensor:
        """[items, G] per-item gradients left by composite_bwd (item = view * N + gaussian).  Affine
        footprint, G = 9: d/du, d/dv, d/dSigma_uu, d/dSigma_uv (shared), d/dSigma_vv, d/dopacity,
        d/dr, d/dg, d/db.  Spherical footprint, G = 13: d/dmu^ (3), d/dSigma~ (xx, xy, xz, yy, yz,
        zz; shared off-diagonals), d/dopacity, d/d(r, g, b)."""
        out = torch.empty((self.n * len(self.wh), int(self.plan.g2d_stride)), dtype=torch.float64, device=self.device)
        B.odgs_debug_g2d(self.plan, _ptr(self.ws), _ptr(out), _stream())
        return out

    def pixel_counts(self) -> torch.Tensor:
        """[pixels, 4] int32 of the last forward: list position after the last contributor,
        contributors, entries evaluated, and entries evaluated up to the last contributor (the
        last two count only entries whose footprint reaches the pixel's 8x8 quadrant; the last
        three need a forward with the count_work setting)."""
        out = torch.empty((self.pixels, 4), dtype=torch.int32, device=self.device)
        B.odgs_debug_pixel_counts(self.plan, _ptr(self.ws), _ptr(out), _stream())
        return out


class TrainStep:
    """One forward + backward step over every view with preallocated outputs, so that it can be
    captured once into a HIP graph and replayed.  Parameters, camera poses and the upstream
    gradient are read from the given device tensors at every replay (update them in place)."""

    def __init__(self, rast: Rasterizer, params, cams: torch.Tensor, dL_drgb: torch.Tensor, stats=None):
        self.rast = rast
        self.stats = stats
        self.params = tuple(params)
        self.cams = cams
        self.dL = dL_drgb
        self.rgb = torch.empty(3 * rast.pixels, dtype=torch.float32, device=rast.device)
        self.grads = tuple(torch.empty_like(x) for x in self.params)
        self.graph = None

    def bin(self):
        self.rast.bin(*self.params, self.cams)

    def fwd(self):
        self.rast.render_fwd(self.rgb, None, want_T=False)

    def composite_bwd(self):
        self.rast.composite_bwd(self.dL)

    def project_bwd(self):
        self.rast.project_bwd(*self.params, self.cams, self.grads, self.stats)

    def run(self):
        self.bin()
        self.fwd()
        self.composite_bwd()
        self.project_bwd()

    def capture(self):
        """Record run() into a HIP graph (after one eager run on the capture stream)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        self.graph.replay()


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opac, sh, cams, rast):
        rast.bin_checked(means, scales, quats, opac, sh, cams)
        rgb, T = rast.render_fwd()
        ctx.rast = rast
        ctx.generation = rast.generation
        ctx.save_for_backward(means, scales, quats, opac, sh, cams)
        ctx.mark_non_differentiable(T)
        return rgb, T

    @staticmethod
    def backward(ctx, g_rgb, g_T):
        rast = ctx.rast
        if rast.generation != ctx.generation:
            raise RuntimeError("the rasterizer ran another forward (or binning) before this backward; its "
                               "workspace no longer holds this forward's lists")
        means, scales, quats, opac, sh, cams = ctx.saved_tensors
        grads = rast.render_bwd(means, scales, quats, opac, sh, cams, g_rgb.contiguous())
        return (*grads, None, None)


def render(means, scales, quats, opacities, sh, cams, rast: Rasterizer):
    """Differentiable render of every view.  Returns (rgb flat, T flat); T is not differentiable."""
    return _RenderFn.apply(means, scales, quats, opacities, sh, cams, rast)


def split_views(flat: torch.Tensor, wh, channels: int):
    """Views of a flat output buffer as a list of [channels, H, W] tensors."""
    out, off = [], 0
    for w, h in wh:
        out.append(flat[off:off + channels * w * h].view(channels, h, w))
        off += channels * w * h
    return out
