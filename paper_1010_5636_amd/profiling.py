"""Summaries of rocprofv3 output for the stencil kernels, and the workloads they profile.

    python -m paper_1010_5636_amd.profiling stats   <out.txt> <cmd> <label>=<trace_dir> ...
    python -m paper_1010_5636_amd.profiling traffic <out.json> <copy_bytes> <cmd> <block,xcd>=<fetch_dir>,<write_dir> ...
    python -m paper_1010_5636_amd.profiling kernels <out.txt> <copy_bytes> <cmd> <trace_dir> <fetch_dir> <write_dir>
    python -m paper_1010_5636_amd.profiling run <workload>[,<workload>...] [reps]
    python -m paper_1010_5636_amd.profiling dispatches <out.txt> <copy_bytes> <cmd> <pattern> <trace_dir> <counter>=<dir> ...

``run`` executes fixed, seeded workloads of the solve and batching legs for the
profiler (``WORKLOADS`` below), each a few launches of the kernels it names,
followed by a device copy of 512 MiB for the counter calibration.  ``kernels``
joins one kernel-trace run and one FETCH_SIZE and one WRITE_SIZE run of the
same command into a per-kernel table: average duration, and HBM bytes per
dispatch (median) scaled by the calibration copy.

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
# the sources of the stencil kernels (the dslash traffic record is valid while they are unchanged)
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


def _dbs(d: str):
    return sorted(glob.glob(os.path.join(d, "**", "*results.db"), recursive=True))


def kernel_stats(trace_dir: str):
    """Per-kernel calls and durations from a kernel-trace run (CSV statistics,
    or the rocpd SQLite database that rocprofv3 writes by default)."""
    rows = []
    for path in _dbs(trace_dir):
        import sqlite3
        con = sqlite3.connect(path)
        q = "select name, count(*), avg(duration), min(duration), max(duration) from kernels group by name"
        for name, n, avg, mn, mx in con.execute(q):
            rows.append({"name": name, "calls": int(n), "avg_ns": float(avg), "min_ns": float(mn), "max_ns": float(mx)})
        con.close()
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
    for path in _dbs(pmc_dir):
        import sqlite3
        con = sqlite3.connect(path)
        q = "select kernel_name, value from counters_collection where counter_name = ? order by dispatch_id"
        for name, val in con.execute(q, (counter,)):
            out.setdefault(name, []).append(float(val))
        con.close()
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


def kernels_text(trace_dir: str, fetch_dir: str, write_dir: str, copy_bytes: int, command: str) -> str:
    """Per-kernel time and HBM traffic of one workload (see the module docstring)."""
    stats = {r["name"]: r for r in kernel_stats(trace_dir)}
    fetch = counters(fetch_dir, "FETCH_SIZE")
    write = counters(write_dir, "WRITE_SIZE")
    cf = _copy_reading(fetch, copy_bytes)
    cw = _copy_reading(write, copy_bytes)
    if not cf or not cw:
        raise RuntimeError("calibration copy kernel not found in the counter output")
    sf, sw = copy_bytes / cf, copy_bytes / cw
    lines = ["# rocprofv3 kernel time and HBM traffic per dispatch", f"# command: {command}",
             f"# kernel source hash: {kernel_hash()}",
             f"# counter scale from a {copy_bytes}-byte device copy: {sf:.2f} bytes per FETCH_SIZE unit, "
             f"{sw:.2f} per WRITE_SIZE unit", "",
             f"{'calls':>7}{'avg_us':>11}{'fetch_MB':>11}{'write_MB':>11}{'GB/s':>9}  kernel"]
    rows = sorted(stats.values(), key=lambda r: -r["calls"] * r["avg_ns"])
    for r in rows:
        f = fetch.get(r["name"])
        w = write.get(r["name"])
        fb = sf * sorted(f)[len(f) // 2] if f else float("nan")
        wb = sw * sorted(w)[len(w) // 2] if w else float("nan")
        gbs = (fb + wb) / r["avg_ns"] if f and w else float("nan")
        lines.append(f"{r['calls']:>7}{r['avg_ns'] / 1e3:>11.3f}{fb / 1e6:>11.3f}{wb / 1e6:>11.3f}{gbs:>9.1f}  "
                     f"{r['name'][:120]}")
    return "\n".join(lines) + "\n"


# ---- profiled workloads -------------------------------------------------------

def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _fullq24(reps):
    """Full Q on 24^3 x 48 (the solve lattice) in the solver's formats: F32
    spinors with 12-real F32 links, F16 spinors with 12-real F16 links, F64 with
    18-real links; two rotating field sets per format."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dims = (48, 24, 24, 24)
    g = ndq.Geometry(dims)
    u = torch.from_numpy(synthetic.gauge_field(dims)).cuda()
    psi = torch.from_numpy(synthetic.spinor(g.volume)).cuda()
    for sp, lp, recon in ((ndq.F32, ndq.F32, 12), (ndq.F16, ndq.F16, 12), (ndq.F64, ndq.F64, 18)):
        sets = []
        for k in range(2):
            U = ndq.GaugeField.pack(g, u, lp, recon)
            x = ndq.SpinorField.pack(g, psi * (1 + 0.1 * k), sp, ndq.FULL)
            sets.append((U, x, x.like()))
        for i in range(reps):
            U, x, y = sets[i % 2]
            ndq.apply_Q(g, U, -1.4, x, y)
        torch.cuda.synchronize()
        _log(f"fullq24: format ({sp}, {lp}, {recon}) done")
        del sets


def _mrhs32(reps):
    """The 12 spin-colour point sources on 32^3 x 64 (F32 spinors, 18-real F32
    links) in one multi-RHS Q apply."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dims = (64, 32, 32, 32)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, torch.from_numpy(synthetic.gauge_field(dims)).cuda(), ndq.F32, 18)
    canon = torch.zeros((12, g.volume, 4, 3), dtype=torch.complex128, device="cuda")
    for s in range(4):
        for c in range(3):
            canon[3 * s + c, 0, s, c] = 1.0
    x = ndq.SpinorField.pack(g, canon, ndq.F32, ndq.FULL)
    del canon
    y = x.like()
    for _ in range(reps):
        ndq.apply_Q(g, U, -1.4, x, y)
    torch.cuda.synchronize()
    _log("mrhs32: done")


def _filter24(reps):
    """The low-mode filter's block apply: Q on 60 FP64 fields (18-real links) on 24^3 x 48."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dims = (48, 24, 24, 24)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, torch.from_numpy(synthetic.gauge_field(dims)).cuda(), ndq.F64, 18)
    x = ndq.SpinorField(g, ndq.F64, ndq.FULL, 60)
    one = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(g.volume)).cuda(), ndq.F64, ndq.FULL)
    rb = g.spinor_bytes(ndq.F64, ndq.FULL, 1)
    for r in range(60):
        x.buf[r * rb:(r + 1) * rb].copy_(one.buf)
    y = x.like()
    for _ in range(reps):
        ndq.apply_Q(g, U, -1.4, x, y)
    torch.cuda.synchronize()
    _log("filter24: done")


def _modes24(reps):
    """The low-mode projection of Eq. 11 with 20 FP64 modes on 24^3 x 48: sign
    applies with a degree-1 polynomial (so the projection kernels dominate) on
    F32 and F64 fields."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    import numpy as np
    dims = (48, 24, 24, 24)
    g = ndq.Geometry(dims)
    u = torch.from_numpy(synthetic.gauge_field(dims)).cuda()
    nev = 20
    modes = ndq.SpinorField(g, ndq.F64, ndq.FULL, nev)
    one = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(g.volume)).cuda(), ndq.F64, ndq.FULL)
    rb = g.spinor_bytes(ndq.F64, ndq.FULL, 1)
    for r in range(nev):
        modes.buf[r * rb:(r + 1) * rb].copy_(one.buf)
    nu = np.linspace(-0.5, 0.5, nev) + 0.01
    ap = ndq.Approx(ndq.MINMAX_POLY, 0.01, 1)
    for sp, lp, recon in ((ndq.F32, ndq.F32, 12), (ndq.F64, ndq.F64, 18)):
        U = ndq.GaugeField.pack(g, u, lp, recon)
        ov = ndq.Overlap(g, -1.4, ap, 6.6, modes=modes, nu=nu)
        x = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(g.volume)).cuda(), sp, ndq.FULL)
        y = x.like()
        for _ in range(reps):
            ndq.apply_sign(g, U, ov, x, y)
        torch.cuda.synchronize()
    _log("modes24: done")


def _batch24(reps):
    """The batched sign of the point-source solves: a degree-4 polynomial sign
    (Clenshaw on the multi-RHS stencil) with 20 FP64 modes on a block of 12 F32
    fields (12-real F32 links) on 24^3 x 48, sandwich projection (block Gram
    products on the matrix cores, one-pass rank-20 update)."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    import numpy as np
    dims = (48, 24, 24, 24)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, torch.from_numpy(synthetic.gauge_field(dims)).cuda(), ndq.F32, 12)
    nev = 20
    modes = ndq.SpinorField(g, ndq.F64, ndq.FULL, nev)
    one = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(g.volume)).cuda(), ndq.F64, ndq.FULL)
    rb = g.spinor_bytes(ndq.F64, ndq.FULL, 1)
    for r in range(nev):
        modes.buf[r * rb:(r + 1) * rb].copy_(one.buf)
    nu = np.linspace(-0.5, 0.5, nev) + 0.01
    ov = ndq.Overlap(g, -1.4, ndq.Approx(ndq.MINMAX_POLY, 0.01, 4), 6.6, modes=modes, nu=nu, form=ndq.SANDWICH)
    x = ndq.SpinorField(g, ndq.F32, ndq.FULL, 12)
    x1 = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(g.volume)).cuda(), ndq.F32, ndq.FULL)
    rb = g.spinor_bytes(ndq.F32, ndq.FULL, 1)
    for r in range(12):
        x.buf[r * rb:(r + 1) * rb].copy_(x1.buf)
    y = x.like()
    for _ in range(reps):
        ndq.apply_sign(g, U, ov, x, y)
    torch.cuda.synchronize()
    _log("batch24: done")


# Work orders of the multi-RHS stencil compared by ``_orders32`` (fields per
# workgroup, group-major, tile chunk): the default, the tuned orders and the
# one-field-per-group extreme.
ORDERS32 = [(0, 0, -1), (6, 1, 16), (4, 1, 16), (2, 1, 16), (1, 1, 16), (12, 0, 16)]


def _orders32(reps):
    """The 12-field Q apply of ``_mrhs32`` (random fields) in each work order
    of ORDERS32, `reps` applies each, in that order (for per-dispatch counters)."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    from paper_1010_5636_amd import ndq as nb
    dims = (64, 32, 32, 32)
    g = ndq.Geometry(dims)
    U = ndq.GaugeField.pack(g, torch.from_numpy(synthetic.gauge_field(dims)).cuda(), ndq.F32, 18)
    x = ndq.SpinorField(g, ndq.F32, ndq.FULL, 12)
    gen = torch.Generator(device="cuda").manual_seed(1002)
    x.buf.view(torch.float32).normal_(generator=gen)   # in place: no copy kernel besides the calibration
    y = x.like()
    for rg, gm, ch in ORDERS32:
        nb.set_mrhs_launch(g, ndq.F32, ndq.F32, 18, 12, 2, rg, bool(gm), ch, True, -1)
        for _ in range(reps):
            ndq.apply_Q(g, U, -1.4, x, y)
        torch.cuda.synchronize()
        _log(f"orders32: rg={rg} group_major={gm} chunk={ch} done")


WORKLOADS = {"fullq24": _fullq24, "mrhs32": _mrhs32, "filter24": _filter24, "modes24": _modes24, "batch24": _batch24,
             "orders32": _orders32}


def dispatches_text(trace_dir: str, pmc_dirs, copy_bytes: int, pattern: str, labels, command: str) -> str:
    """Per-dispatch duration and counters of the kernels whose name contains
    `pattern`, in dispatch order, grouped `len(dispatches) / len(labels)` per
    label.  pmc_dirs: [(counter, dir)]; FETCH_SIZE and WRITE_SIZE are scaled to
    bytes by the calibration copy, other counters are printed as read."""
    import sqlite3
    durs = []
    for path in _dbs(trace_dir):
        con = sqlite3.connect(path)
        durs += [d for (d,) in con.execute("select duration from kernels where name like ? order by id",
                                           (f"%{pattern}%",))]
        con.close()
    cols = []
    for counter, d in pmc_dirs:
        vals = counters(d, counter)
        seq = [v for name, vs in vals.items() if pattern in name for v in vs]
        scale = 1.0
        if counter in ("FETCH_SIZE", "WRITE_SIZE"):
            c = _copy_reading(vals, copy_bytes)
            scale = copy_bytes / c / 1e6 if c else float("nan")
        cols.append((counter, [v * scale for v in seq]))
    per = max(1, len(durs) // max(1, len(labels)))
    lines = ["# rocprofv3 per-dispatch kernel time and counters", f"# command: {command}",
             f"# kernel source hash: {kernel_hash()}", f"# kernels matching: {pattern}",
             "# FETCH_SIZE / WRITE_SIZE in MB (scaled by a device copy of %d bytes); other counters raw" % copy_bytes,
             "", f"{'label':<28}{'us':>10}" + "".join(f"{c:>16}" for c, _ in cols)]
    for i, lab in enumerate(labels):
        sl = slice(i * per, (i + 1) * per)
        t = sorted(durs[sl])
        if not t:
            continue
        row = f"{str(lab):<28}{t[len(t) // 2] / 1e3:>10.1f}"
        for _, v in cols:
            vv = sorted(v[sl]) if len(v) >= (i + 1) * per else []
            row += f"{vv[len(vv) // 2]:>16.1f}" if vv else f"{'-':>16}"
        lines.append(row)
    return "\n".join(lines) + "\n"
CALIBRATION_BYTES = 512 * 1024 * 1024


def run(names, reps: int) -> int:
    import torch
    from . import ndq
    ndq.lib()
    for name in names:
        _log(f"workload {name}: {reps} reps")
        WORKLOADS[name](reps)
    src = torch.empty(CALIBRATION_BYTES, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    _log("calibration copy done")
    return 0


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
    if len(argv) >= 2 and argv[0] == "run":
        sys.path.insert(0, ROOT)
        return run(argv[1].split(","), int(argv[2]) if len(argv) > 2 else 10)
    if len(argv) == 7 and argv[0] == "kernels":
        txt = kernels_text(argv[4], argv[5], argv[6], int(argv[2]), argv[3])
        with open(argv[1], "w") as fh:
            fh.write(txt)
        print(txt)
        return 0
    if len(argv) >= 6 and argv[0] == "dispatches":
        # dispatches <out.txt> <copy_bytes> <cmd> <pattern> <trace_dir> <counter>=<dir> ...
        pmc = [tuple(a.split("=", 1)) for a in argv[6:]]
        labels = [f"rg={a} gm={b} chunk={c}" for a, b, c in ORDERS32]
        txt = dispatches_text(argv[5], pmc, int(argv[2]), argv[4], labels, argv[3])
        with open(argv[1], "w") as fh:
            fh.write(txt)
        print(txt)
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
