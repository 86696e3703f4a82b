"""Helpers for the GPU parity tests: run the HIP path through the C ABI on numpy inputs."""
import numpy as np

# Tolerances: colours 1e-4 absolute per pixel, gradients 1e-3 relative per element.
RGB_ATOL = 1e-4
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-3 * 1e-3   # absolute floor, times the largest |gradient| of the tensor
# Pixels whose early-termination test lies within this relative margin of the 1e-4 threshold can
# legitimately terminate one step earlier or later on either side (float exp differs by a few
# ulp between host and device); they are excluded from the strict comparison and counted.
TERM_MARGIN = 2e-5


def to_gpu(scene, cams, device="cuda"):
    import torch
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return [f(scene.means), f(scene.scales), f(scene.quats), f(scene.opacities), f(scene.sh), f(cams.cams)]


def run_gpu(scene, cams, settings, dL=None, pair_capacity=None, return_rast=False, split_bwd=False):
    import torch
    from paper_2410_20686_amd.rasterizer import Rasterizer
    wh = [tuple(int(x) for x in r) for r in cams.wh]
    rast = Rasterizer(scene.n, scene.sh_degree, wh, settings, pair_capacity=pair_capacity)
    t = to_gpu(scene, cams)
    st = rast.bin_checked(*t)
    rgb, T = rast.render_fwd()
    out = dict(rgb=rgb.cpu().numpy(), T=T.cpu().numpy(), status=st)
    if dL is not None:
        dLg = torch.from_numpy(np.ascontiguousarray(dL, dtype=np.float32)).cuda()
        if split_bwd:
            # the two backward stages separately, with the per-item 2D gradients in between
            rast.composite_bwd(dLg)
            out["g2d"] = rast.g2d().cpu().numpy().reshape(len(wh), scene.n, -1)
            g = tuple(torch.empty_like(x) for x in t[:5])
            rast.project_bwd(*t, g)
        else:
            g = rast.render_bwd(*t, dLg)
        torch.cuda.synchronize()
        out["grads"] = dict(zip(("means", "scales", "quats", "opacities", "sh"), (x.cpu().numpy() for x in g)))
    if return_rast:
        out["rast"] = rast
        out["tensors"] = t
    return out


def assert_grads_close(gpu, ref, names=("means", "scales", "quats", "opacities", "sh"), rtol=GRAD_RTOL,
                       floor=GRAD_FLOOR, per_gaussian_floor=None):
    """|gpu - ref| <= rtol |ref| + floor * max|ref| (over the tensor), plus optionally, for the
    tensors named in per_gaussian_floor, that fraction of the largest |ref| component of the same
    Gaussian (for quantities whose small components are cancellations of the large ones)."""
    report = {}
    for k in names:
        a, b = np.asarray(gpu[k], dtype=np.float64), np.asarray(ref[k], dtype=np.float64)
        gmax = np.abs(b).max() if b.size else 0.0
        err = np.abs(a - b)
        lim = rtol * np.abs(b) + floor * gmax
        if per_gaussian_floor and k in per_gaussian_floor and b.ndim == 2 and b.size:
            lim = lim + per_gaussian_floor[k] * np.abs(b).max(axis=0, keepdims=True)
        bad = ~(err <= lim)  # NaN counts as out of tolerance
        report[k] = (int(bad.sum()), float((err / np.maximum(lim, 1e-300)).max()) if b.size else 0.0)
        assert not bad.any(), "%s: %d elements out of tolerance, worst ratio %.3g, example gpu=%r ref=%r" % (
            k, bad.sum(), report[k][1], a[bad][:3], b[bad][:3])
    return report


def strict_pixels(margin, threshold=TERM_MARGIN):
    return np.asarray(margin) > threshold
