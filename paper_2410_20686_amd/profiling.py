"""Summaries of rocprofv3 runs of ``bench.py``: per-kernel time, calibrated HBM traffic and rates
against the MI355X peaks, VALU issue and lane use, LDS activity.

Inputs are the CSV outputs of one ``--kernel-trace --stats`` run and of several ``--pmc`` runs of
the same command (one counter group each; rocprofv3 does not split counters over passes).  HBM
bytes come from ``FETCH_SIZE`` and ``WRITE_SIZE`` (KiB per dispatch), each scaled by what the same
counter reads for a device-to-device copy of known size in the same run (``bench.py
--copy-calibration MIB``).

Usage (the profiled commands are written into the summary's header):
    python -m paper_2410_20686_amd.profiling --trace DIR --pmc DIR [DIR ...] --calib-mib 256 \
        --out profiles/NAME.txt --cmd-trace "..." --cmd-pmc "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
from collections import defaultdict

HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
CUS, SIMDS_PER_CU, CLOCK = 256, 4, 2.4e9
LANE_OPS_PEAK = CUS * 64 * CLOCK   # non-packed FP32 lane-operations per second
LDS_BYTES_PER_CLK_CU = 128   # 32 banks x 4 bytes per clock (the CDNA LDS width)
LDS_PEAK = CUS * LDS_BYTES_PER_CLK_CU * CLOCK
COPY_KERNEL = "__amd_rocclr_copyBuffer"

SOURCES = ("paper_2410_20686_amd/csrc/render.hip", "paper_2410_20686_amd/csrc/common.h",
           "paper_2410_20686_amd/csrc/wave.h")


def source_hash(root: str) -> str:
    """Hash of the compositor sources a counter summary was taken from."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _csv(dirname: str, suffix: str):
    files = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def kernel_stats(trace_dir: str):
    """{kernel: (calls, average ns)} from the --stats output."""
    out = {}
    for r in _csv(trace_dir, "kernel_stats.csv"):
        out[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]))
    return out


def counters(pmc_dir: str):
    """{kernel: {counter: [value per dispatch]}} from a --pmc output."""
    per = defaultdict(lambda: defaultdict(dict))
    for r in _csv(pmc_dir, "counter_collection.csv"):
        per[r["Kernel_Name"]][r["Counter_Name"]][r["Dispatch_Id"]] = \
            per[r["Kernel_Name"]][r["Counter_Name"]].get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return {k: {c: list(d.values()) for c, d in v.items()} for k, v in per.items()}


def short(name: str) -> str:
    """Kernel name without return type, anonymous namespace and argument list."""
    name = name.replace("(anonymous namespace)::", "").strip()
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0].strip()


def summarize(trace_dir, pmc_dirs, calib_mib, out_path, cmd_trace, cmd_pmc, root, key_kernel, cmd_summary=""):
    stats = kernel_stats(trace_dir)
    pmc = defaultdict(dict)
    for d in pmc_dirs:
        for k, cs in counters(d).items():
            pmc[k].update(cs)
    # calibration: the largest copy dispatch is the known-size one
    copy = pmc.get(COPY_KERNEL, {})
    kib = calib_mib * 1024.0
    f_fetch = kib / max(copy.get("FETCH_SIZE", [kib])) if copy.get("FETCH_SIZE") else 1.0
    f_write = kib / max(copy.get("WRITE_SIZE", [kib])) if copy.get("WRITE_SIZE") else 1.0
    mean = lambda xs: sum(xs) / len(xs) if xs else float("nan")
    rows = []
    for name, (calls, avg_ns) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        c = pmc.get(name, {})
        dur = avg_ns * 1e-9
        fetch = mean(c.get("FETCH_SIZE", [])) * 1024 * f_fetch
        write = mean(c.get("WRITE_SIZE", [])) * 1024 * f_write
        traffic = fetch + write
        valu = mean(c.get("SQ_INSTS_VALU", []))
        act_valu = mean(c.get("SQ_ACTIVE_INST_VALU", []))
        thr_valu = mean(c.get("SQ_THREAD_CYCLES_VALU", []))
        lds_active = mean(c.get("SQ_LDS_IDX_ACTIVE", []))
        lds_conf = mean(c.get("SQ_LDS_BANK_CONFLICT", []))
        # bytes moved by LDS instructions (64-byte units, active lanes only)
        lds_units = sum(mean(c.get(k, [])) if c.get(k) else 0.0 for k in
                        ("SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH", "SQ_INSTS_LDS_ATOMIC_BANDWIDTH"))
        has_ldsbw = any(c.get(k) for k in ("SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH"))
        rows.append(dict(
            kernel=short(name), calls=calls, avg_us=avg_ns / 1e3, total_ms=calls * avg_ns / 1e6,
            traffic_gb=traffic / 1e9, hbm_gbs=traffic / dur / 1e9 if dur > 0 else float("nan"),
            hbm_frac=traffic / dur / HBM_PEAK if dur > 0 else float("nan"),
            valu_insts=valu,
            # one wave64 VALU instruction occupies its SIMD for 4 cycles (no packed FP32 here)
            valu_issue_frac=valu * 4 / (CUS * SIMDS_PER_CU * CLOCK) / dur if dur > 0 else float("nan"),
            lane_util=thr_valu / (act_valu * 64) if act_valu and act_valu == act_valu else float("nan"),
            lds_frac=lds_active / (CUS * CLOCK * dur) if dur > 0 else float("nan"),
            lds_gbs=lds_units * 64 / dur / 1e9 if (dur > 0 and has_ldsbw) else float("nan"),
            lds_bw_frac=lds_units * 64 / dur / LDS_PEAK if (dur > 0 and has_ldsbw) else float("nan"),
            lds_conflict=lds_conf / lds_active if lds_active else float("nan"),
            full=name))
    total_ms = sum(r["total_ms"] for r in rows)
    lines = []
    lines.append("# rocprofv3 summary (bench.py), produced by paper_2410_20686_amd/profiling.py")
    lines.append("#")
    lines.append("# kernel trace:  " + cmd_trace)
    for c in cmd_pmc:
        lines.append("# counters:      " + c)
    if cmd_summary:
        lines.append("# summary:       " + cmd_summary)
    lines.append("#")
    lines.append("# peaks (MI355X): HBM 8 TB/s; VALU issue 1,024 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction;")
    lines.append("#   LDS %d B per clock per CU (32 banks x 4 B) x 256 CUs x 2.4 GHz = %.1f TB/s" %
                 (LDS_BYTES_PER_CLK_CU, LDS_PEAK / 1e12))
    lines.append("# hbm_frac = calibrated (FETCH_SIZE + WRITE_SIZE) bytes / avg duration / 8 TB/s")
    lines.append("# valu_issue = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz) / avg duration")
    lines.append("# lane_util = SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU): active lanes per VALU instruction")
    lines.append("# lds_busy = SQ_LDS_IDX_ACTIVE / (256 CUs x 2.4 GHz x avg duration): fraction of cycles the LDS is busy")
    lines.append("# LDS_GB/s = 64 B x (SQ_INSTS_LDS_LOAD_BANDWIDTH + _STORE_ + _ATOMIC_BANDWIDTH) / avg duration: bytes the")
    lines.append("#   LDS instructions moved (active lanes); lds_bw = that / LDS peak; ldscf = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE")
    lines.append("")
    lines.append("## HBM traffic calibration: one %d MiB device-to-device copy (%s)" % (calib_mib, COPY_KERNEL))
    lines.append("factor_fetch %.4f  factor_write %.4f  (bytes = counter KiB * 1024 * factor)" % (f_fetch, f_write))
    lines.append("")
    lines.append("## per kernel (averages per dispatch)")
    hdr = ("%-44s %5s %9s %7s %8s %8s %6s %10s %6s %6s %8s %8s %6s %6s" %
           ("kernel", "calls", "avg_us", "pct", "traffic", "HBM_GB/s", "hbm", "VALU_inst", "valu", "lanes", "lds_busy",
            "LDS_GB/s", "lds_bw", "ldscf"))
    lines.append(hdr)
    fmt = lambda x, f: ("%" + f) % x if x == x else "-"
    for r in rows:
        lines.append("%-44s %5d %9.1f %6.1f%% %8s %8s %6s %10s %6s %6s %8s %8s %6s %6s" % (
            r["kernel"][:44], r["calls"], r["avg_us"], 100 * r["total_ms"] / total_ms, fmt(r["traffic_gb"], ".4f"),
            fmt(r["hbm_gbs"], ".0f"), fmt(r["hbm_frac"], ".3f"), fmt(r["valu_insts"], ".3e"),
            fmt(r["valu_issue_frac"], ".3f"), fmt(r["lane_util"], ".3f"), fmt(r["lds_frac"], ".3f"),
            fmt(r["lds_gbs"], ".0f"), fmt(r["lds_bw_frac"], ".3f"), fmt(r["lds_conflict"], ".3f")))
    key = next((r for r in rows if r["kernel"] == key_kernel), None)
    lines.append("")
    lines.append("## machine-readable (read by bench.py)")
    lines.append("source_sha256_16: %s" % source_hash(root))
    for r in rows:
        if r["traffic_gb"] == r["traffic_gb"]:
            lines.append("kernel: %s | avg_us %.3f | traffic_bytes %.0f | hbm_frac %.4f | valu_issue %.4f | lanes %.4f"
                         " | lds_busy %.4f | lds_gbs %.1f | lds_bw_frac %.4f" % (
                             r["kernel"], r["avg_us"], r["traffic_gb"] * 1e9, r["hbm_frac"], r["valu_issue_frac"],
                             r["lane_util"], r["lds_frac"], r["lds_gbs"], r["lds_bw_frac"]))
    if key is None:
        lines.append("# note: key kernel %s not found" % key_kernel)
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def read_summary(path: str):
    """{kernel: {avg_us, traffic_bytes, hbm_frac, ...}} and the source hash of a summary, or
    (None, None) when it is missing."""
    try:
        with open(path) as f:
            text = f.read().splitlines()
    except OSError:
        return None, None
    src, out = None, {}
    for line in text:
        if line.startswith("source_sha256_16:"):
            src = line.split(":", 1)[1].strip()
        elif line.startswith("kernel: "):
            parts = [p.strip() for p in line[len("kernel: "):].split("|")]
            d = {}
            for p in parts[1:]:
                k, v = p.split(" ", 1)
                d[k] = float(v)
            out[parts[0]] = d
    return out, src


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--pmc", nargs="+", default=[])
    ap.add_argument("--calib-mib", type=int, default=256)
    ap.add_argument("--out", required=True)
    ap.add_argument("--cmd-trace", default="")
    ap.add_argument("--cmd-pmc", action="append", default=[])
    ap.add_argument("--key-kernel", default="")
    ap.add_argument("--cmd-summary", default="")
    a = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    summarize(a.trace, a.pmc, a.calib_mib, a.out, a.cmd_trace, a.cmd_pmc, root, a.key_kernel, a.cmd_summary)


if __name__ == "__main__":
    main()
