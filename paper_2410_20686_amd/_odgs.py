"""ctypes binding of ``libodgs.so`` (the C ABI of include/odgs.h).

Argument marshalling only: every function here forwards plain pointers and sizes to the
library of the same name.  Loading fails loudly when the library has not been built; there is
no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libodgs.so")

MAX_VIEWS = 64
OK, EINVAL, ENOSPACE, EHIP, ETOOBIG = 0, -1, -2, -3, -4
L1_NOALLOC_MAX_COUNT = 65536 * 4096
STATUS_OVERFLOW = 1
STATUS_STALE_FORWARD = 2
FLAG_COUNT_WORK = 1
FLAG_SPHERICAL = 2
FLAG_SCHED_PERSISTENT = 4
FLAG_SCHED_TILE_ID = 8
SCHEDULES = {"queue": 0, "persistent": FLAG_SCHED_PERSISTENT, "tile_id": FLAG_SCHED_TILE_ID}
FLAG_BIN_COARSE = 16
FLAG_BIN_DIRECT = 32
BINNINGS = {"auto": 0, "coarse": FLAG_BIN_COARSE, "direct": FLAG_BIN_DIRECT}

EXPORTS = ("odgs_plan_init", "odgs_plan_set_pinhole", "odgs_workspace_bytes", "odgs_preprocess", "odgs_bin_sort", "odgs_render_fwd",
           "odgs_render_bwd", "odgs_composite_bwd", "odgs_project_bwd", "odgs_status_offset", "odgs_strerror",
           "odgs_densify", "odgs_densify_workspace_bytes", "odgs_l1_loss", "odgs_l1_loss_workspace_bytes",
           "odgs_l1_loss_noalloc",
           "odgs_adam_step",
           "odgs_plan_size", "odgs_debug_records", "odgs_debug_keys", "odgs_debug_pixel_counts", "odgs_debug_g2d")


class Settings(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("batch", ctypes.c_int32), ("batch_bwd", ctypes.c_int32), ("near_r", ctypes.c_float),
                ("far_r", ctypes.c_float), ("dilation", ctypes.c_float), ("pole_eps", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("flags", ctypes.c_int32)]


class DensifyAcc(ctypes.Structure):
    _fields_ = [("grad_sum", ctypes.c_void_p), ("tau_sum", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("tau_min", ctypes.c_float), ("tau_max", ctypes.c_float)]


class ParamPtrs(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class AdamHyper(ctypes.Structure):
    _fields_ = [("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class DensifyParams(ctypes.Structure):
    _fields_ = [("extent", ctypes.c_float), ("percent_dense", ctypes.c_float), ("min_opacity", ctypes.c_float),
                ("max_scale_frac", ctypes.c_float)]


class Status(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_int32), ("n_pairs_stored", ctypes.c_int32), ("n_pairs", ctypes.c_int64),
                ("n_visible", ctypes.c_int64), ("bin_gen", ctypes.c_uint32), ("fwd_gen", ctypes.c_uint32),
                ("n_culled", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64)]


_OFFSETS = ["off_status", "off_rec", "off_rect", "off_count", "off_depth", "off_dkey0", "off_dkey1", "off_did0", "off_did1", "off_srect",
            "off_blocksum", "off_pkey0", "off_pkey1", "off_pval0", "off_pval1", "off_hist", "off_digit",
            "off_ranges", "off_T", "off_last", "off_ncontrib", "off_neval", "off_lasteval", "off_g2d", "off_srec",
            "off_cone", "off_dirs", "off_queue"]


class Plan(ctypes.Structure):
    _fields_ = ([("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("n_views", ctypes.c_int32),
                 ("s", Settings), ("width", ctypes.c_int32 * MAX_VIEWS), ("height", ctypes.c_int32 * MAX_VIEWS),
                 ("tile_base", ctypes.c_int32 * (MAX_VIEWS + 1)), ("pix_base", ctypes.c_int64 * (MAX_VIEWS + 1)),
                 ("pinhole", (ctypes.c_float * 4) * MAX_VIEWS),
                 ("items", ctypes.c_int64), ("pair_capacity", ctypes.c_int64), ("tile_bits", ctypes.c_int32),
                 ("item_blocks", ctypes.c_int32), ("pair_blocks", ctypes.c_int32), ("g2d_stride", ctypes.c_int32)]
                + [(name, ctypes.c_size_t) for name in _OFFSETS]
                + [("depth_final", ctypes.c_int32), ("pair_final", ctypes.c_int32), ("coarse", ctypes.c_int32),
                   ("coarse_bits", ctypes.c_int32), ("tile_base32", ctypes.c_int32 * (MAX_VIEWS + 1)),
                   ("ws_bytes", ctypes.c_size_t)])


_lib = None


def lib():
    """Load libodgs.so (raises if it is missing or does not match these declarations)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libodgs.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2410_20686_amd.build): %s" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, c_i64, c_i32, c_sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        pp = ctypes.POINTER(Plan)
        L.odgs_plan_size.restype = c_sz
        L.odgs_plan_init.argtypes = [pp, c_i64, c_i32, c_i32, P, ctypes.POINTER(Settings), c_i64]
        L.odgs_plan_init.restype = c_i32
        c_f = ctypes.c_float
        L.odgs_plan_set_pinhole.argtypes = [pp, c_i32, c_f, c_f, c_f, c_f]
        L.odgs_plan_set_pinhole.restype = c_i32
        L.odgs_workspace_bytes.argtypes = [pp]
        L.odgs_workspace_bytes.restype = c_sz
        L.odgs_status_offset.argtypes = [pp]
        L.odgs_status_offset.restype = c_sz
        L.odgs_preprocess.argtypes = [pp, P, P, P, P, P, P, P, c_sz, P]
        L.odgs_preprocess.restype = c_i32
        L.odgs_bin_sort.argtypes = [pp, P, c_sz, P]
        L.odgs_bin_sort.restype = c_i32
        L.odgs_render_fwd.argtypes = [pp, P, c_sz, P, P, P, P]
        L.odgs_render_fwd.restype = c_i32
        L.odgs_render_bwd.argtypes = [pp, P, P, P, P, P, P, P, c_sz, P, P, P, P, P, P, P, P]
        L.odgs_render_bwd.restype = c_i32
        L.odgs_composite_bwd.argtypes = [pp, P, c_sz, P, P]
        L.odgs_composite_bwd.restype = c_i32
        L.odgs_project_bwd.argtypes = [pp, P, P, P, P, P, P, P, c_sz, P, P, P, P, P, P, P]
        L.odgs_project_bwd.restype = c_i32
        L.odgs_densify_workspace_bytes.argtypes = [c_i64]
        L.odgs_densify_workspace_bytes.restype = c_sz
        L.odgs_densify.argtypes = [c_i64, c_i32] + [P] * 9 + [ctypes.POINTER(DensifyParams), c_i64] + [P] * 8 + [c_sz, P]
        L.odgs_densify.restype = c_i32
        L.odgs_l1_loss_workspace_bytes.argtypes = [c_i64]
        L.odgs_l1_loss_workspace_bytes.restype = c_sz
        L.odgs_l1_loss.argtypes = [P, P, c_i64, P, P, P, c_sz, P]
        L.odgs_l1_loss.restype = c_i32
        L.odgs_l1_loss_noalloc.argtypes = [P, P, c_i64, P, P, P]
        L.odgs_l1_loss_noalloc.restype = c_i32
        pptr = ctypes.POINTER(ParamPtrs)
        L.odgs_adam_step.argtypes = [c_i64, c_i32, pptr, pptr, pptr, pptr, pptr, P, P, ctypes.POINTER(AdamHyper), P]
        L.odgs_adam_step.restype = c_i32
        L.odgs_debug_pixel_counts.argtypes = [pp, P, P, P]
        L.odgs_debug_g2d.argtypes = [pp, P, P, P]
        L.odgs_debug_g2d.restype = c_i32
        L.odgs_debug_pixel_counts.restype = c_i32
        L.odgs_strerror.argtypes = [c_i32]
        L.odgs_strerror.restype = ctypes.c_char_p
        L.odgs_debug_records.argtypes = [pp, P, P, P]
        L.odgs_debug_records.restype = c_i32
        L.odgs_debug_keys.argtypes = [pp, P, c_i64, P, P, P]
        L.odgs_debug_keys.restype = c_i32
        if L.odgs_plan_size() != ctypes.sizeof(Plan):
            raise ImportError("odgs_plan layout mismatch: library %d bytes, binding %d bytes"
                              % (L.odgs_plan_size(), ctypes.sizeof(Plan)))
        _lib = L
    return _lib


class OdgsError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != OK:
        raise OdgsError("%s failed: %s (%d)" % (what, lib().odgs_strerror(rc).decode(), rc))


def make_settings(tile=16, batch=0, batch_bwd=0, near=0.2, far=1e4, dilation=0.3, pole_eps=1e-4,
                  bg=(0.0, 0.0, 0.0), count_work=False, footprint="affine", schedule="queue",
                  binning="auto") -> Settings:
    """footprint: "affine" (the paper's local affine approximation) or "spherical"
    (ODGS_FLAG_SPHERICAL: the exact per-ray maximum of each 3D Gaussian).  schedule: the
    compositors' tile scheduling, "queue" (one workgroup per tile, longest list first),
    "persistent" (device-filling workgroups claiming tiles from that queue) or "tile_id" (one
    workgroup per tile in tile id order).  binning (16x16 tiles): "auto" (by 32x32 tile, then
    split into the 16x16 lists, from 16384 tiles on; else directly), "coarse" or "direct"."""
    if footprint not in ("affine", "spherical"):
        raise ValueError("footprint must be 'affine' or 'spherical'")
    if schedule not in SCHEDULES:
        raise ValueError("schedule must be one of %s" % sorted(SCHEDULES))
    if binning not in BINNINGS:
        raise ValueError("binning must be one of %s" % sorted(BINNINGS))
    s = Settings()
    s.tile, s.batch, s.batch_bwd = int(tile), int(batch), int(batch_bwd)
    s.near_r, s.far_r, s.dilation, s.pole_eps = float(near), float(far), float(dilation), float(pole_eps)
    for k in range(3):
        s.bg[k] = float(bg[k])
    s.flags = ((FLAG_COUNT_WORK if count_work else 0) | (FLAG_SPHERICAL if footprint == "spherical" else 0)
               | SCHEDULES[schedule] | BINNINGS[binning])
    return s


def odgs_plan_init(n: int, sh_degree: int, wh, settings: Settings, pair_capacity: int) -> Plan:
    plan = Plan()
    flat = (ctypes.c_int32 * (2 * len(wh)))(*[int(x) for pair in wh for x in pair])
    rc = lib().odgs_plan_init(ctypes.byref(plan), int(n), int(sh_degree), len(wh), ctypes.cast(flat, ctypes.c_void_p),
                              ctypes.byref(settings), int(pair_capacity))
    _check(rc, "odgs_plan_init")
    return plan


def odgs_plan_set_pinhole(plan: Plan, view: int, fx: float, fy: float, cx: float, cy: float):
    _check(lib().odgs_plan_set_pinhole(ctypes.byref(plan), int(view), float(fx), float(fy), float(cx), float(cy)),
           "odgs_plan_set_pinhole")


def odgs_workspace_bytes(plan: Plan) -> int:
    return int(lib().odgs_workspace_bytes(ctypes.byref(plan)))


def odgs_status_offset(plan: Plan) -> int:
    return int(lib().odgs_status_offset(ctypes.byref(plan)))


def odgs_preprocess(plan, means, scales, quats, opac, sh, cams, ws, ws_bytes, stream):
    _check(lib().odgs_preprocess(ctypes.byref(plan), means, scales, quats, opac, sh, cams, ws, ws_bytes, stream),
           "odgs_preprocess")


def odgs_bin_sort(plan, ws, ws_bytes, stream):
    _check(lib().odgs_bin_sort(ctypes.byref(plan), ws, ws_bytes, stream), "odgs_bin_sort")


def odgs_render_fwd(plan, ws, ws_bytes, out_rgb, out_T, out_depth, stream):
    _check(lib().odgs_render_fwd(ctypes.byref(plan), ws, ws_bytes, out_rgb, out_T, out_depth, stream), "odgs_render_fwd")


def _acc_ref(acc):
    return None if acc is None else ctypes.byref(acc)


def odgs_render_bwd(plan, means, scales, quats, opac, sh, cams, ws, ws_bytes, dL, d_means, d_scales, d_quats,
                    d_opac, d_sh, acc, stream):
    """acc: DensifyAcc or None."""
    _check(lib().odgs_render_bwd(ctypes.byref(plan), means, scales, quats, opac, sh, cams, ws, ws_bytes, dL, d_means,
                                 d_scales, d_quats, d_opac, d_sh, _acc_ref(acc), stream), "odgs_render_bwd")


def odgs_composite_bwd(plan, ws, ws_bytes, dL, stream):
    _check(lib().odgs_composite_bwd(ctypes.byref(plan), ws, ws_bytes, dL, stream), "odgs_composite_bwd")


def odgs_project_bwd(plan, means, scales, quats, opac, sh, cams, ws, ws_bytes, d_means, d_scales, d_quats, d_opac,
                     d_sh, acc, stream):
    """acc: DensifyAcc or None."""
    _check(lib().odgs_project_bwd(ctypes.byref(plan), means, scales, quats, opac, sh, cams, ws, ws_bytes, d_means,
                                  d_scales, d_quats, d_opac, d_sh, _acc_ref(acc), stream), "odgs_project_bwd")


def odgs_l1_loss_workspace_bytes(count: int) -> int:
    return int(lib().odgs_l1_loss_workspace_bytes(int(count)))


def odgs_l1_loss(rgb, target, count, dL, loss, ws, ws_bytes, stream):
    _check(lib().odgs_l1_loss(rgb, target, int(count), dL, loss, ws, ws_bytes, stream), "odgs_l1_loss")


def odgs_l1_loss_noalloc(rgb, target, count, dL, loss, stream):
    _check(lib().odgs_l1_loss_noalloc(rgb, target, int(count), dL, loss, stream), "odgs_l1_loss_noalloc")


def odgs_adam_step(n, sh_degree, raw: ParamPtrs, act: ParamPtrs, grad: ParamPtrs, m: ParamPtrs, v: ParamPtrs, lr, step,
                   hyper: AdamHyper, stream):
    _check(lib().odgs_adam_step(int(n), int(sh_degree), ctypes.byref(raw), ctypes.byref(act), ctypes.byref(grad),
                                ctypes.byref(m), ctypes.byref(v), lr, step, ctypes.byref(hyper), stream),
           "odgs_adam_step")


def odgs_densify_workspace_bytes(n: int) -> int:
    return int(lib().odgs_densify_workspace_bytes(int(n)))


def odgs_densify(n, sh_degree, means, scales, quats, opac, sh, grad_sum, tau_sum, count, noise, params: DensifyParams,
                 capacity, out_means, out_scales, out_quats, out_opac, out_sh, out_src, out_counts, ws, ws_bytes, stream):
    _check(lib().odgs_densify(int(n), int(sh_degree), means, scales, quats, opac, sh, grad_sum, tau_sum, count, noise,
                              ctypes.byref(params), int(capacity), out_means, out_scales, out_quats, out_opac, out_sh,
                              out_src, out_counts, ws, ws_bytes, stream), "odgs_densify")


def odgs_debug_pixel_counts(plan, ws, out, stream):
    _check(lib().odgs_debug_pixel_counts(ctypes.byref(plan), ws, out, stream), "odgs_debug_pixel_counts")


def odgs_debug_g2d(plan, ws, out, stream):
    _check(lib().odgs_debug_g2d(ctypes.byref(plan), ws, out, stream), "odgs_debug_g2d")


def odgs_debug_records(plan, ws, out, stream):
    _check(lib().odgs_debug_records(ctypes.byref(plan), ws, out, stream), "odgs_debug_records")


def odgs_debug_keys(plan, ws, cap, keys, gauss, stream):
    _check(lib().odgs_debug_keys(ctypes.byref(plan), ws, int(cap), keys, gauss, stream), "odgs_debug_keys")


def odgs_strerror(code: int) -> str:
    return lib().odgs_strerror(int(code)).decode()
