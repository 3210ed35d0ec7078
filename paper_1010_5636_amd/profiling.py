"""Summaries of rocprofv3 output for the stencil kernels.

    python -m paper_1010_5636_amd.profiling stats   <out.txt> <cmd> <label>=<trace_dir> ...
    python -m paper_1010_5636_amd.profiling traffic <out.json> <copy_bytes> <cmd> <block,xcd>=<fetch_dir>,<write_dir> ...

``stats`` condenses ``*kernel_stats.csv`` (from ``rocprofv3 --kernel-trace
--stats``) of one or more runs into a short text table, one section per run.
``traffic`` reads the per-dispatch FETCH_SIZE and WRITE_SIZE counters (KiB,
from two ``rocprofv3 --pmc`` runs per launch shape), calibrates each run
against a plain device-to-device copy of ``copy_bytes`` bytes each way
recorded in the same run, and writes the HBM bytes per launch of every
even/odd dslash instantiation and launch shape (block, XCD remap), tagged
with the hash of the kernel source.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1010_5636_amd/csrc/wilson.hip", "paper_1010_5636_amd/csrc/wilson.h",
                  "paper_1010_5636_amd/csrc/ndq_device.h"]
_FMT = re.compile(r"k_wilson(_dirsplit)?<(\d+), (\d+), (\d+)")
_PREC = {0: "f64", 1: "f32", 2: "f16"}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def format_name(kernel: str):
    """'f32-r12' style name of a stencil instantiation (spinor prec, recon), or None."""
    m = _FMT.search(kernel)
    if not m:
        return None
    sp, lp, recon = int(m.group(2)), int(m.group(3)), int(m.group(4))
    name = f"{_PREC[sp]}-r{recon}"
    if lp != sp:
        name += f"-l{_PREC[lp]}"
    return name


def _csvs(d: str, suffix: str):
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def kernel_stats(trace_dir: str):
    rows = []
    for path in _csvs(trace_dir, "kernel_stats.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                rows.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                             "min_ns": float(r.get("MinNs", 0) or 0), "max_ns": float(r.get("MaxNs", 0) or 0)})
    return rows


def stats_text(runs, command: str) -> str:
    """runs: [(label, trace_dir)]."""
    lines = ["# rocprofv3 kernel statistics", f"# command: {command}"]
    for label, trace_dir in runs:
        rows = sorted(kernel_stats(trace_dir), key=lambda r: -r["calls"] * r["avg_ns"])
        lines += ["", f"## {label}", f"{'format':<14}{'calls':>8}{'avg_us':>10}{'min_us':>10}{'max_us':>10}  kernel"]
        for r in rows:
            fmt = format_name(r["name"]) or "-"
            lines.append(f"{fmt:<14}{r['calls']:>8}{r['avg_ns'] / 1e3:>10.3f}{r['min_ns'] / 1e3:>10.3f}"
                         f"{r['max_ns'] / 1e3:>10.3f}  {r['name'][:110]}")
    return "\n".join(lines) + "\n"


def counters(pmc_dir: str, counter: str):
    """{kernel name: [per-dispatch value]} for one counter."""
    out = {}
    for path in _csvs(pmc_dir, "counter_collection.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _copy_reading(vals: dict, copy_bytes: int):
    """Counter reading (KiB) of the calibration copy: the largest-reading
    dispatch of a runtime copy kernel."""
    best = None
    for name, v in vals.items():
        if "copy" in name.lower() or "Copy" in name:
            m = max(v)
            best = m if best is None else max(best, m)
    return best


def traffic(runs, copy_bytes: int, command: str):
    """runs: [(launch dict, fetch_dir, write_dir)].  Returns the summary with
    one entry per (format, launch shape)."""
    rec = {"kernel_hash": kernel_hash(), "command": command, "copy_bytes": copy_bytes, "formats": {}}
    for launch, fetch_dir, write_dir in runs:
        fetch = counters(fetch_dir, "FETCH_SIZE")
        write = counters(write_dir, "WRITE_SIZE")
        cf = _copy_reading(fetch, copy_bytes)
        cw = _copy_reading(write, copy_bytes)
        if not cf or not cw:
            raise RuntimeError("calibration copy kernel not found in the counter output")
        sf = copy_bytes / cf   # bytes per counter unit
        sw = copy_bytes / cw
        for name, v in fetch.items():
            fmt = format_name(name)
            w = write.get(name)
            if fmt is None or not w:
                continue
            fb = sf * sorted(v)[len(v) // 2]
            wb = sw * sorted(w)[len(w) // 2]
            rec["formats"].setdefault(fmt, []).append(
                {"launch": launch, "kernel": name[:120], "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                 "bytes_per_launch": fb + wb, "dispatches": len(v), "fetch_scale_bytes_per_unit": sf,
                 "write_scale_bytes_per_unit": sw})
    return rec


def lookup(rec: dict, fmt: str, launch: dict):
    """HBM bytes per launch of format ``fmt`` at ``launch``, or None."""
    if rec.get("kernel_hash") != kernel_hash():
        return None
    for ent in rec.get("formats", {}).get(fmt, []):
        if ent.get("launch") == launch:
            return ent.get("bytes_per_launch")
    return None


def _launch(text: str) -> dict:
    b, x = (int(t) for t in text.split(","))
    return {"block": b, "xcd_remap": x}


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        runs = [tuple(a.split("=", 1)) for a in argv[3:]]
        txt = stats_text(runs, argv[2])
        with open(argv[1], "w") as fh:
            fh.write(txt)
        print(txt)
        return 0
    if len(argv) >= 5 and argv[0] == "traffic":
        runs = []
        for a in argv[4:]:
            launch, dirs = a.split("=", 1)
            fd, wd = dirs.split(",", 1)
            runs.append((_launch(launch), fd, wd))
        rec = traffic(runs, int(argv[2]), argv[3])
        with open(argv[1], "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec, indent=1))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
