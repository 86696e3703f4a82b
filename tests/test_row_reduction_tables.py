"""The lane-to-value tables of the compositors' 16-lane row reductions (kRowSlot for the nine
affine gradient values, kSphRowSlot for the thirteen spherical ones), checked against a model of
the DPP exchange pattern the kernels use: partners 15-i (row_mirror), (i & 8) | (7 - (i & 7))
(row_half_mirror), (i & ~3) | (3 - (i & 3)) (quad_perm [3,2,1,0]) and i ^ 1 (quad_perm [1,0,3,2]).
A lane keeping one slot of a pair (by a bit of its index) adds the partner's copy of the same slot;
values summed in place add the partner's copy of themselves.  Host-only."""
import os
import re

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_20686_amd", "csrc")

PARTNER = {
    "mirror": lambda i: 15 - i,
    "half_mirror": lambda i: (i & 8) | (7 - (i & 7)),
    "quad_rev": lambda i: (i & ~3) | (3 - (i & 3)),
    "pair": lambda i: i ^ 1,
}


def _read(ctrl, x):
    return np.array([x[PARTNER[ctrl](i)] for i in range(16)])


def _bfly(ctrl, lo, hi, bit):
    bits = np.array([(i & bit) != 0 for i in range(16)])
    send = np.where(bits, lo, hi)
    return np.where(bits, hi, lo) + _read(ctrl, send)


def _const(fname, name):
    src = open(os.path.join(CSRC, fname)).read()
    return int(re.search(name + r"\s*=\s*(0x[0-9A-Fa-f]+)ull", src).group(1), 16)


def _check(table, out, totals, nvalues):
    seen = set()
    for lane in range(16):
        q = (table >> (4 * lane)) & 0xF
        if q < nvalues:
            assert out[lane] == totals[q], (lane, q)
            seen.add(q)
    assert seen == set(range(nvalues))


def test_nine_value_table():
    rng = np.random.default_rng(5)
    g = rng.integers(0, 10**6, size=(9, 16))
    a = [_bfly("mirror", g[j], g[4 + j], 8) for j in range(4)]
    s8 = g[8] + _read("mirror", g[8])
    c = [_bfly("half_mirror", a[j], a[2 + j], 4) for j in range(2)]
    s8 = s8 + _read("half_mirror", s8)
    d = _bfly("quad_rev", c[0], c[1], 2)
    s8 = s8 + _read("quad_rev", s8)
    out = _bfly("pair", d, s8, 1)
    _check(_const("render.hip", "kRowSlot"), out, g.sum(axis=1), 9)


def test_thirteen_value_table():
    rng = np.random.default_rng(6)
    g = rng.integers(0, 10**6, size=(13, 16))
    regs = [_bfly("mirror", g[j], g[8 + j], 8) for j in range(5)]
    regs += [g[j] + _read("mirror", g[j]) for j in (5, 6, 7)]
    c = [_bfly("half_mirror", regs[2 * j], regs[2 * j + 1], 4) for j in range(4)]
    e = [_bfly("quad_rev", c[2 * j], c[2 * j + 1], 2) for j in range(2)]
    out = _bfly("pair", e[0], e[1], 1)
    _check(_const("render_sph.hip", "kSphRowSlot"), out, g.sum(axis=1), 13)
