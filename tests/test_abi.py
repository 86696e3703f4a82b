"""The C ABI library loads, exports every entry point declared in include/odgs.h, and rejects
bad arguments on the host before enqueuing anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2410_20686_amd import _odgs as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "odgs.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2410_20686_amd import build
        build.build()
    return B.lib()


def test_every_declared_symbol_is_exported(lib):
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(odgs_[a-z_0-9]+)\s*\(", text, re.M))
    assert {"odgs_preprocess", "odgs_bin_sort", "odgs_render_fwd", "odgs_render_bwd"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(B.EXPORTS) == declared


def test_plan_layout(lib):
    p = B.odgs_plan_init(12345, 3, [(1024, 512), (2048, 1024), (64, 32)], B.make_settings(tile=16), 1_000_003)
    assert p.n_views == 3 and p.items == 3 * 12345
    assert list(p.tile_base[:4]) == [0, 2048, 2048 + 8192, 2048 + 8192 + 8]
    assert p.pix_base[3] == 1024 * 512 + 2048 * 1024 + 64 * 32
    assert p.tile_bits == 14 and p.s.batch == 64 and p.s.batch_bwd == 64
    sph_only = ("off_srec", "off_cone", "off_dirs")  # empty regions (at the end) without the spherical flag
    offs = sorted(getattr(p, n) for n in B._OFFSETS if n not in sph_only)
    assert all(o % 256 == 0 for o in offs)
    assert len(set(offs)) == len(offs)
    assert B.odgs_workspace_bytes(p) == p.ws_bytes >= offs[-1]
    assert all(getattr(p, n) == p.ws_bytes for n in sph_only)
    assert B.odgs_status_offset(p) == p.off_status
    assert p.g2d_stride == 9


def test_binning_choice(lib):
    """Coarse binning (32x32-tile sort, then the 16x16 lists) by default from 16384 tiles on, only
    at tile 16 with every side a multiple of 32; the flags force either path."""
    big = [(2048, 1024)] * 2  # 16,384 tiles of 16x16
    small = [(256, 128), (512, 256)]
    plan = lambda wh, **kw: B.odgs_plan_init(1000, 0, wh, B.make_settings(**kw), 100_000)
    p = plan(big)
    assert p.coarse == 1 and p.coarse_bits == 12 and list(p.tile_base32[:3]) == [0, 2048, 4096]
    assert p.pair_final == (((p.coarse_bits + 7) // 8) % 2) ^ 1  # sort passes, then refined into the other buffer
    assert plan(big[:1] + [(1024, 512)]).coarse == 0  # 10,240 tiles
    assert plan(big, binning="direct").coarse == 0
    assert plan(big, tile=8).coarse == 0 and plan(big, tile=32).coarse == 0
    assert plan(small).coarse == 0
    q = plan(small, binning="coarse")
    assert q.coarse == 1 and list(q.tile_base32[:3]) == [0, 32, 160]
    assert plan([(256, 128), (80, 48)], binning="coarse").coarse == 0  # 80 and 48: not multiples of 32
    st = B.make_settings()
    st.flags = B.FLAG_BIN_COARSE | B.FLAG_BIN_DIRECT
    with pytest.raises(B.OdgsError):
        B.odgs_plan_init(1000, 0, small, st, 100_000)
    with pytest.raises(ValueError):
        B.make_settings(binning="fine")


def test_spherical_plan_layout(lib):
    wh = [(1024, 512), (64, 32)]
    p = B.odgs_plan_init(12345, 3, wh, B.make_settings(tile=16, footprint="spherical"), 1_000_003)
    q = B.odgs_plan_init(12345, 3, wh, B.make_settings(tile=16), 1_000_003)
    assert p.g2d_stride == 13 and p.s.flags == B.FLAG_SPHERICAL
    offs = sorted(getattr(p, n) for n in B._OFFSETS)
    assert len(set(offs)) == len(offs) and all(o % 256 == 0 for o in offs)
    items = 2 * 12345
    assert p.off_cone - p.off_srec >= 64 * items and p.off_dirs - p.off_cone >= 64 * items
    assert p.ws_bytes - p.off_dirs >= 16 * (1024 + 512 + 64 + 32)
    assert p.ws_bytes > q.ws_bytes + (4 * 4 + 64 + 64) * items
    # the spherical footprint is defined for equirectangular views and has no work counters
    with pytest.raises(B.OdgsError):
        B.odgs_plan_set_pinhole(p, 0, 100.0, 100.0, 32.0, 16.0)
    with pytest.raises(B.OdgsError):
        B.odgs_plan_init(10, 0, [(64, 32)], B.make_settings(footprint="spherical", count_work=True), 100)
    # no densification statistics with it (rejected before anything is enqueued)
    nul, fake = None, ctypes.c_void_p(256 * 1024)
    acc = B.DensifyAcc(256 * 1024, 256 * 1024, 256 * 1024, 2e-5, 1e-4)
    p = B.odgs_plan_init(10, 0, [(64, 32)], B.make_settings(footprint="spherical"), 100)
    assert lib.odgs_project_bwd(ctypes.byref(p), fake, fake, fake, fake, fake, fake, fake, p.ws_bytes, fake, fake,
                                fake, fake, fake, ctypes.byref(acc), nul) == B.EINVAL
    assert lib.odgs_render_bwd(ctypes.byref(p), fake, fake, fake, fake, fake, fake, fake, p.ws_bytes, fake, fake,
                               fake, fake, fake, fake, ctypes.byref(acc), nul) == B.EINVAL


@pytest.mark.parametrize("kw,wh", [
    (dict(tile=12), [(64, 32)]),
    (dict(tile=16), [(100, 64)]),
    (dict(tile=32, batch=32), [(64, 32)]),
    (dict(tile=16, batch=100), [(64, 32)]),
    (dict(tile=16), [(64, 32)] * 65),
    (dict(tile=8), [(32768, 16384)] * 64),  # 2^29 tiles: four compositing tasks per tile overflow a grid
    (dict(tile=16, far=0.1), [(64, 32)]),
])
def test_plan_rejects_bad_settings(lib, kw, wh):
    with pytest.raises(B.OdgsError):
        B.odgs_plan_init(10, 0, wh, B.make_settings(**kw), 100)


@pytest.mark.parametrize("n,deg,cap", [(-1, 0, 10), (10, 4, 10), (10, -1, 10), (10, 0, 1 << 31), (1 << 31, 0, 10)])
def test_plan_rejects_bad_sizes(lib, n, deg, cap):
    with pytest.raises(B.OdgsError):
        B.odgs_plan_init(n, deg, [(64, 32)], B.make_settings(), cap)


def test_entry_points_validate_on_host(lib):
    p = B.odgs_plan_init(10, 0, [(64, 32)], B.make_settings(), 100)
    nul = None
    fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: validation fails first
    assert lib.odgs_preprocess(ctypes.byref(p), fake, fake, fake, fake, fake, fake, nul, p.ws_bytes, nul) == B.EINVAL
    assert lib.odgs_bin_sort(ctypes.byref(p), fake, p.ws_bytes - 1, nul) == B.ENOSPACE
    assert lib.odgs_render_fwd(ctypes.byref(p), fake, p.ws_bytes, nul, nul, nul, nul) == B.EINVAL
    misaligned = ctypes.c_void_p(256 * 1024 + 2)
    assert lib.odgs_preprocess(ctypes.byref(p), misaligned, fake, fake, fake, fake, fake, fake, p.ws_bytes,
                               nul) == B.EINVAL
    assert lib.odgs_render_bwd(ctypes.byref(p), fake, fake, fake, fake, fake, fake, fake, p.ws_bytes, nul, fake,
                               fake, fake, fake, fake, nul, nul) == B.EINVAL
    # statistics requested with a null accumulator array
    acc = B.DensifyAcc(None, 256 * 1024, 256 * 1024, 2e-5, 1e-4)
    assert lib.odgs_project_bwd(ctypes.byref(p), fake, fake, fake, fake, fake, fake, fake, p.ws_bytes, fake, fake,
                                fake, fake, fake, ctypes.byref(acc), nul) == B.EINVAL
    for code in (B.OK, B.EINVAL, B.ENOSPACE, B.EHIP):
        assert B.odgs_strerror(code)


def test_densify_validates_on_host(lib):
    fake = ctypes.c_void_p(256 * 1024)
    nul = None
    n = 100
    ws = B.odgs_densify_workspace_bytes(n)
    assert ws >= 3 * 4 and ws % 256 == 0
    dp = B.DensifyParams(10.0, 1e-3, 0.005, 0.0)
    ins = [fake] * 9
    outs = [fake] * 8

    def call(n=n, deg=3, cap=2 * n, dp=dp, ws_bytes=ws, ins=ins, outs=outs):
        return lib.odgs_densify(n, deg, *ins, ctypes.byref(dp), cap, *outs, ws_bytes, nul)

    assert call(cap=2 * n - 1) == B.EINVAL          # capacity below the largest result
    assert call(deg=4) == B.EINVAL
    assert call(n=-1) == B.EINVAL
    assert call(ws_bytes=ws - 1) == B.ENOSPACE
    assert call(ins=[fake] * 8 + [nul]) == B.EINVAL  # noise missing
    assert call(outs=[fake] * 6 + [ctypes.c_void_p(256 * 1024 + 4), fake]) == B.EINVAL  # misaligned counts
    assert call(dp=B.DensifyParams(float("nan"), 1e-3, 0.005, 0.0)) == B.EINVAL
    assert call(dp=B.DensifyParams(10.0, 1e-3, 0.005, -1.0)) == B.EINVAL


def test_noalloc_l1_rejects_sizes_beyond_its_scratch(lib):
    """Checked on the host before anything is enqueued (no device memory is touched)."""
    fake = 1 << 20  # 256-aligned stand-ins: never dereferenced on these paths
    rc = lib.odgs_l1_loss_noalloc(fake, fake, B.L1_NOALLOC_MAX_COUNT + 1, fake, fake, None)
    assert rc == B.ETOOBIG
    assert b"scratch" in lib.odgs_strerror(rc)
    assert lib.odgs_l1_loss_noalloc(fake, fake, -1, fake, fake, None) == B.EINVAL
    assert lib.odgs_l1_loss_noalloc(fake, fake, 10, fake, None, None) == B.EINVAL
