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
                       floor=GRAD_FLOOR, slack=None):
    """|gpu - ref| <= rtol |ref| + floor * max|ref| (over the tensor), plus, per element, the
    tensors' entries in `slack` when given (float_exponent_slack)."""
    report = {}
    for k in names:
        a, b = np.asarray(gpu[k], dtype=np.float64), np.asarray(ref[k], dtype=np.float64)
        gmax = np.abs(b).max() if b.size else 0.0
        err = np.abs(a - b)
        lim = rtol * np.abs(b) + floor * gmax
        if slack is not None:
            lim = lim + np.asarray(slack[k], dtype=np.float64)
        bad = ~(err <= lim)  # NaN counts as out of tolerance
        report[k] = (int(bad.sum()), float((err / np.maximum(lim, 1e-300)).max()) if b.size else 0.0)
        assert not bad.any(), "%s: %d elements out of tolerance, worst ratio %.3g, example gpu=%r ref=%r" % (
            k, bad.sum(), report[k][1], a[bad][:3], b[bad][:3])
    return report


def float_exponent_slack(scene, cams, settings, dL, ref, pix=None):
    """Per-element distance between the oracle's gradient (mode 32: float contributor decisions,
    double arithmetic) and the same derivative taken at the exponents as the float pass evaluated
    them (mode 33).  A float32 renderer composites with float exponents, so its gradient can sit
    this far from the double-exponent reference before any error of its own; the spherical
    footprint's exponent of a needle-like Gaussian (axis ratios ~800:1) is where this reaches the
    1e-3 scale.  Keys: the five parameter tensors, plus "g2d" (kernel layout) for the spherical
    footprint."""
    from oracle import oracle as O
    alt = O.backward(scene, cams, settings, dL, mode=33, pix=pix, want_g2d="g2d_kernel" in ref)
    out = {k: np.abs(ref[k] - alt[k]) for k in ("means", "scales", "quats", "opacities", "sh")}
    if "g2d_kernel" in ref:
        out["g2d"] = np.abs(ref["g2d_kernel"] - alt["g2d_kernel"])
    return out


def strict_pixels(margin, threshold=TERM_MARGIN):
    return np.asarray(margin) > threshold
