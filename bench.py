"""Benchmark of the Wilson-Dirac hot path on one MI355X.

Workload (the dslash benchmark): even/odd Wilson dslash on a 16^3 x 32
lattice (V = 131072, 65536 output sites per apply), m = -1.4, random SU(3)
links (su(3) generator width 0.3, re-unitarised), complex Gaussian spinors,
link storage 18/12/8 reals in FP32 and 18 reals in FP64 (plus FP16 storage).

One step = one even/odd dslash apply (1320 flop per output site).  Steps
alternate D_oe and D_eo over NSETS independent (U, psi_e, psi_o) sets whose
total size exceeds 512 MB, so consecutive applies cannot reuse each other's
data from the 256 MB Infinity Cache: the timed applies stream from HBM.
The timed region is K back-to-back launches between two HIP events on the
launch stream (optionally replayed from a HIP graph with --graph).

Prints one JSON line.  `value` is GFLOP/s of the headline format; the
`roofline` object is for the headline dslash kernel (algorithmic bytes per
launch / average launch time over the timed region; `traffic` is the HBM
bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary
when it was taken on the current kernel source); `variants` lists every format; `cpu_baseline` times the FP64 oracle
on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (32, 16, 16, 16)
M = -1.4
FLOP_PER_SITE = 1320
HBM_PEAK_GBS = 8000.0
ROTATE_BYTES = 600e6
# (name, spinor prec, link prec, recon); the first entry is the headline
FORMATS = [("f32-r12", 1, 1, 12), ("f32-r18", 1, 1, 18), ("f32-r8", 1, 1, 8), ("f64-r18", 0, 0, 18),
           ("f16-r12", 2, 2, 12)]
SPINOR_BYTES = {0: 192, 1: 96, 2: 52}
LINK_REAL_BYTES = {0: 8, 1: 4, 2: 2}

def bytes_per_site(sp, lp, recon):
    """Algorithmic bytes per output site of one even/odd dslash: 8 links
    (each of the 4V links is read once per pair of parities), the input
    spinor once, the output spinor once."""
    return 8 * recon * LINK_REAL_BYTES[lp] + 2 * SPINOR_BYTES[sp]


def kernel_name(launch):
    """Name of the dslash kernel that the launch shape selects (as rocprofv3 lists it)."""
    if launch["block"] == 0:
        return "k_wilson_dirsplit (even/odd dslash, 4 wavefronts per 64 sites)"
    return f"k_wilson (even/odd dslash, {launch['block']}-lane workgroups)"


def read_traffic(fmt_name, launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source at this launch shape; else None."""
    path = os.path.join(ROOT, "profiles", "dslash_16c32_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_1010_5636_amd.profiling import lookup
    return lookup(rec, fmt_name, launch)


def cpu_baseline(max_seconds=20.0):
    """The FP64 oracle's even/odd dslash on the host, on as many applies as fit
    in ~max_seconds (at least 2), with BLAS/OpenMP pools limited to 1 thread."""
    import synthetic
    from oracle import dirac
    from threadpoolctl import threadpool_limits
    v = int(np.prod(DIMS))
    with threadpool_limits(1):
        u = synthetic.gauge_field(DIMS)
        psi = synthetic.spinor(v // 2)
        dirac.dslash(u, psi, DIMS, 1)  # warm-up
        n, t0 = 0, time.perf_counter()
        while True:
            psi = dirac.dslash(u, psi, DIMS, (n + 1) % 2)   # even -> odd -> even ...
            n += 1
            el = time.perf_counter() - t0
            if (n >= 2 and el > max_seconds) or n >= 50:
                break
    gflops = FLOP_PER_SITE * (v // 2) * n / el / 1e9
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    # per output site of one dslash; a full Q is two dslashes (both parities) plus the
    # site term, so about 2 x this per site of the lattice
    us_site = el / n / (v // 2) * 1e6
    return {"value": round(gflops, 4), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} even/odd dslash applies of the FP64 numpy oracle on the 16^3x32 lattice "
                      f"({el:.1f} s, one thread)",
            "host": {"cpu": cpu, "nproc": os.cpu_count()}, "us_per_site_dslash": round(us_site, 4)}


def cpu_tau(reps=5):
    """The paper's unit measured on the oracle: seconds per site per step of the
    polynomial recurrence (two FP64 Q applies of the oracle on 16^3 x 32 plus the
    recurrence's vector updates, t_{j+1} = 2 Z t_j - t_{j-1}, acc += c_j t_{j+1},
    Z = (2 Q^2 / lam^2 - (1 + eps)) / (1 - eps)), median of `reps` steps after one
    warm-up step, with the BLAS/OpenMP pools at one thread and at all threads."""
    import synthetic
    from oracle import dirac
    from threadpoolctl import threadpool_info, threadpool_limits
    v = int(np.prod(DIMS))
    u = synthetic.gauge_field(DIMS)
    t_prev = synthetic.spinor(v, seed=11)
    t_cur = synthetic.spinor(v, seed=12)
    acc = np.zeros_like(t_cur)
    lam, eps = 6.6, 0.01

    def step(tp, tc, a):
        z = (2.0 * dirac.apply_Q(u, dirac.apply_Q(u, tc, M, DIMS), M, DIMS) / lam ** 2 - (1.0 + eps) * tc) / (1.0 - eps)
        tn = 2.0 * z - tp
        a += 0.1 * tn
        return tc, tn

    out = {"unit": "microseconds per site per recurrence step (2 Q applies + vector updates)",
           "lattice": "16^3x32", "reps": reps,
           "blas": [{"api": i.get("internal_api"), "threads": i.get("num_threads")} for i in threadpool_info()]}
    for label, limit in (("one_thread", 1), ("all_threads", None)):
        with threadpool_limits(limit):
            tp, tc = step(t_prev, t_cur, acc)
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                tp, tc = step(tp, tc, acc)
                times.append(time.perf_counter() - t0)
        out[label] = {"tau_us": round(float(np.median(times)) / v * 1e6, 4),
                      "step_s_median": round(float(np.median(times)), 3),
                      "threads": 1 if limit else os.cpu_count()}
    return out


def extrapolated_cpu(base, solve):
    """Oracle times the CPU could not run in a bounded sample, extrapolated from the
    measured per-site dslash time (labelled as such): the paper's tau (time per site per
    Clenshaw step = 2 full Q applies, vector work ignored), and one plain FP64 solve on
    24^3x48 from the GPU run's count of Q applies."""
    t_q_site = 2 * base["us_per_site_dslash"]
    v = int(np.prod(SOLVE_DIMS))
    out = {"kind": "extrapolated from the measured oracle dslash rate (one thread); the measured tau is "
                   "cpu_baseline.tau_measured"}
    if solve:
        out["fp64_solve_24c48_s"] = round(solve["runs"]["fp64"]["q_applies"] * t_q_site * v * 1e-6, 1)
        out["fp64_solve_gpu_s"] = solve["runs"]["fp64"]["seconds"]
    return out


SOLVE_DIMS = (48, 24, 24, 24)
SOLVE_MQ = 0.05
SOLVE_NEV = 20
LAM_MAX = 6.6


def poly_for(ndq, eps, target):
    """Smallest-degree minimax polynomial (library Remez) with delta <= target."""
    n = max(8, int(0.8 * np.log(2.0 / target) / (2.0 * np.sqrt(eps))))
    while True:
        a = ndq.Approx(ndq.MINMAX_POLY, eps, n)
        if a.delta <= target:
            return a
        n += max(4, n // 10)


def solve_leg(log, sectors_fp64=False):
    """D_N^m solves on the 24^3 x 48 lattice: mixed precision (F32 arithmetic on
    F32 or F16 storage, FP64 defect correction) vs plain FP64, to a 1e-10 true
    relative residual.  Setup (fields, 20 FP64 low modes, approximants) is timed
    separately and excluded from solves/s."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    g = ndq.Geometry(SOLVE_DIMS)
    v = g.volume
    u = torch.from_numpy(synthetic.gauge_field(SOLVE_DIMS)).to(dev)
    # FP64 links in the 12-real form (c = (a x b)^*, Eq. 3): exact for SU(3) to FP64 rounding,
    # a third fewer link bytes for the FP64 operator, the low-mode filter and the plain solve
    U64 = ndq.GaugeField.pack(g, u, ndq.F64, 12)
    U32 = ndq.GaugeField.pack(g, u, ndq.F32, 12)
    U16 = ndq.GaugeField.pack(g, u, ndq.F16, 12)
    del u
    start = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.start_vector(v)).to(dev), ndq.F64, ndq.FULL)
    b = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(v)).to(dev), ndq.F64, ndq.FULL)
    torch.cuda.synchronize()
    t_fields = time.perf_counter() - t0
    log(f"solve leg: fields {t_fields:.1f} s")
    # work order of the 12-field multi-RHS stencil of the batched solves
    tuned = {}
    t0 = time.perf_counter()
    for name, sp, Uf in (("f32-r12", ndq.F32, U32), ("f16-r12", ndq.F16, U16)):
        r = ndq.ndq.autotune_mrhs(g, Uf, sp, 12, ny=2, reps=5)
        tuned[name + "_12rhs"] = {k: r[k] for k in ("rg", "group_major", "chunk", "us_best", "us_previous")}
    log(f"solve leg: launch tuning {time.perf_counter() - t0:.1f} s: {tuned}")
    t0 = time.perf_counter()
    # a block of 20 + 40 vectors: the 20 lowest modes sit in a dense cluster, and
    # the larger block converges in fewer filter steps (measured 36 s vs 55 s with 20 + 8);
    # the filter of the early restarts on the F32 links (FP64 Rayleigh-Ritz throughout)
    modes, nu, rho, info = ndq.lowmodes_compute(g, U64, M, LAM_MAX, start, SOLVE_NEV, nextra=40, tol=1e-11,
                                                U_lo=U32)
    t_modes = time.perf_counter() - t0
    log(f"solve leg: low modes {t_modes:.1f} s, {info['q_applies']} Q applies, lam_next {info['lam_next']:.5f}")
    k = (info["lam_next"] - info["rho_next"]) / LAM_MAX
    eps = k * k
    t0 = time.perf_counter()
    ap64 = poly_for(ndq, eps, 1e-12)
    ap_lo = poly_for(ndq, eps, 1e-6)
    t_approx = time.perf_counter() - t0
    ov64 = ndq.Overlap(g, M, ap64, LAM_MAX, modes=modes, nu=nu, mq=SOLVE_MQ)
    ov_lo = ndq.Overlap(g, M, ap_lo, LAM_MAX, modes=modes, nu=nu, mq=SOLVE_MQ)
    out = {"workload": "D_N^m x = b, 24^3x48, m=-1.4, mq=0.05, 20 exact low modes (block Chebyshev-filtered subspace iteration, FP64 Rayleigh-Ritz and residues, the filter of the early restarts on F32 links), "
                       "complex Gaussian b (and a chiral point source for the inner-solver comparison), true relative "
                       "residual 1e-10 with the FP64 operator",
           "dims": list(SOLVE_DIMS), "setup_s": {"fields": round(t_fields, 2), "lowmodes": round(t_modes, 2),
                                                 "approximants": round(t_approx, 2)},
           "lowmodes": {"nev": SOLVE_NEV, "nu_abs_min": float(np.abs(nu).min()), "nu_abs_max": float(np.abs(nu).max()),
                        "lam_next": info["lam_next"], "max_rho": info["max_rho"], "kappa_plus": info["kappa_plus"],
                        "kappa_minus": info["kappa_minus"], "q_applies": info["q_applies"],
                        "restarts": info["restarts"], "restarts_f32_filter": info["restarts_lo"],
                        "cheb_degree": info["cheb_degree"], "block": SOLVE_NEV + 40},
           "launch_tuning": tuned,
           "approximant": {"kind": "minimax polynomial (Clenshaw)", "eps": eps, "degree_fp64": ap64.n,
                           "delta_fp64": ap64.delta, "degree_inner": ap_lo.n, "delta_inner": ap_lo.delta}}
    runs = {}
    # Inner tolerances: the library's defaults (1e-5 for F32 storage; 8 units of
    # F16 rounding, 8 * 2^-11, for F16 storage).
    # a spin-colour point source (spin 2, colour 0 at site 0): chiral, so the
    # chirality-sector inner solver needs one sector
    point = torch.zeros((v, 4, 3), dtype=torch.complex128, device=dev)
    point[0, 2, 0] = 1.0
    b_point = ndq.SpinorField.pack(g, point, ndq.F64, ndq.FULL)
    del point
    cases = [("mixed_f32", ndq.F32, U32, ov_lo, 0.0, False, b),
             ("mixed_f16", ndq.F16, U16, ov_lo, 0.0, False, b),
             ("fp64", ndq.F64, None, None, 0.0, False, b),
             ("point_mixed_f32", ndq.F32, U32, ov_lo, 0.0, False, b_point),
             ("point_mixed_f32_sectors", ndq.F32, U32, ov_lo, 0.0, True, b_point)]
    if sectors_fp64:   # the plain-FP64 pair of the inner-solver comparison (38 s)
        cases += [("point_fp64", ndq.F64, None, None, 0.0, False, b_point),
                  ("point_fp64_sectors", ndq.F64, None, None, 0.0, True, b_point)]
    for name, prec, Ulo, ovlo, itol, sectors, rhs in cases:
        x = ndq.SpinorField(g, ndq.F64, ndq.FULL)
        x.buf.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ndq.solve_DN(g, U64, ov64, rhs, x, tol=1e-10, U_lo=Ulo, ov_lo=ovlo, inner_prec=prec, inner_tol=itol,
                          max_outer=30, sectors=sectors)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        runs[name] = {"seconds": round(el, 3), "solves_per_s": round(1.0 / el, 4), "residual": st["residual"],
                      "outer": st["outer"], "inner_cg_iterations": st["inner"], "q_applies": st["q_applies"],
                      "inner_solver": "chirality sectors" if sectors else "CGNE",
                      "source": "point (chiral)" if rhs is b_point else "complex Gaussian"}
        log(f"solve leg: {name} {el:.2f} s, residual {st['residual']:.2e}, outer {st['outer']}, "
            f"inner {st['inner']}, Q applies {st['q_applies']}")
        del x
    # the 12 spin-colour point sources at the origin solved as one block (every
    # stencil application of the recurrence serves all 12 fields) against the
    # same 12 sources solved one by one, mixed F32; and the block at F16 storage
    pts = torch.zeros((12, v, 4, 3), dtype=torch.complex128, device=dev)
    for s_ in range(4):
        for c_ in range(3):
            pts[3 * s_ + c_, 0, s_, c_] = 1.0
    b12 = ndq.SpinorField.pack(g, pts, ndq.F64, ndq.FULL)
    del pts
    rb = g.spinor_bytes(ndq.F64, ndq.FULL, 1)
    blk = {}
    for name, prec, Ulo in (("batched_mixed_f32", ndq.F32, U32), ("batched_mixed_f16", ndq.F16, U16)):
        x = ndq.SpinorField(g, ndq.F64, ndq.FULL, 12)
        x.buf.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ndq.solve_DN(g, U64, ov64, b12, x, tol=1e-10, U_lo=Ulo, ov_lo=ov_lo, inner_prec=prec, max_outer=30)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        blk[name] = {"seconds": round(el, 3), "solves_per_s": round(12 / el, 4), "residual_max": st["residual"],
                     "outer": st["outer"], "block_iterations": st["inner"], "q_applies": st["q_applies"]}
        log(f"solve leg: {name} 12 point sources {el:.2f} s, residual {st['residual']:.2e}, outer {st['outer']}, "
            f"block iterations {st['inner']}")
        del x
    x1 = ndq.SpinorField(g, ndq.F64, ndq.FULL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst, q1, it1 = 0.0, 0, 0
    for r in range(12):
        x1.buf.zero_()
        b1 = ndq.SpinorField(g, ndq.F64, ndq.FULL, 1, buffer=b12.buf[r * rb:(r + 1) * rb])
        st = ndq.solve_DN(g, U64, ov64, b1, x1, tol=1e-10, U_lo=U32, ov_lo=ov_lo, inner_prec=ndq.F32, max_outer=30)
        worst, q1, it1 = max(worst, st["residual"]), q1 + st["q_applies"], it1 + st["inner"]
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t0
    blk["single_mixed_f32"] = {"seconds": round(el1, 3), "solves_per_s": round(12 / el1, 4), "residual_max": worst,
                               "inner_cg_iterations": it1, "q_applies": q1}
    blk["speedup_batched_vs_single_f32"] = round(el1 / blk["batched_mixed_f32"]["seconds"], 3)
    blk["work_order"] = ndq.ndq.get_mrhs_launch(g, ndq.F32, ndq.F32, 12, 12, 2)
    log(f"solve leg: 12 single mixed F32 point-source solves {el1:.2f} s "
        f"(batched speed-up {blk['speedup_batched_vs_single_f32']:.2f}x)")
    out["point_sources_12"] = {"workload": "the 12 spin-colour point sources at the origin, 24^3x48, mq=0.05, "
                                           "20 exact low modes; true relative residual 1e-10 per source", **blk}
    del b12, x1
    torch.cuda.empty_cache()
    # algorithmic bytes of the Q applies alone (links once, spinor in and out
    # once per apply: 384 B/site F32-12, 200 F16-12, 768 F64-12), counted at the
    # inner precision for the mixed runs (the FP64 outer applies are ~2% of them)
    qbytes = {"mixed_f32": 384, "mixed_f16": 200, "fp64": 768}
    for name, r in runs.items():
        rb = r["q_applies"] * qbytes["mixed_f32" if "f32" in name else "fp64" if "fp64" in name else name] * v
        r["q_alg_bytes"] = rb
        r["q_roofline_s"] = round(rb / (HBM_PEAK_GBS * 1e9), 4)
        r["frac_of_roofline"] = round(rb / (HBM_PEAK_GBS * 1e9) / r["seconds"], 4)
    # the paper's unit: time per site per Clenshaw step (one step = 2 Q applies
    # with fused vector updates), on one polynomial sign apply
    tau = {}
    for name, prec, Uf, ap in (("f32", ndq.F32, U32, ap_lo), ("f64", ndq.F64, U64, ap64)):
        ov = ndq.Overlap(g, M, ap, LAM_MAX)
        xs = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(v)).to(dev), prec, ndq.FULL)
        ys = xs.like()
        ndq.apply_sign(g, Uf, ov, xs, ys)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ndq.apply_sign(g, Uf, ov, xs, ys)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 3
        tau[name] = {"degree": ap.n, "sign_ms": round(el * 1e3, 3), "tau_us": round(el / (ap.n * v) * 1e6, 6)}
        del ov, xs, ys
    out["clenshaw_tau"] = {"unit": "microseconds per site per Clenshaw step", **tau,
                           "paper_context": "GTX285: 0.038 (single), 0.090 (double); Core2 SSE2: 0.877 / 1.459, "
                                            "i.e. GPU over CPU about 23x (single) and 16x (double) (Sec. 3, Sec. 4); "
                                            "other hardware, context only"}
    out["runs"] = runs
    out["speedup_mixed_f32_vs_fp64"] = round(runs["fp64"]["seconds"] / runs["mixed_f32"]["seconds"], 3)
    out["speedup_mixed_f16_vs_fp64"] = round(runs["fp64"]["seconds"] / runs["mixed_f16"]["seconds"], 3)
    out["speedup_sectors_vs_cgne_point_source"] = {
        "mixed_f32": round(runs["point_mixed_f32"]["seconds"] / runs["point_mixed_f32_sectors"]["seconds"], 3)}
    if sectors_fp64:
        out["speedup_sectors_vs_cgne_point_source"]["fp64"] = round(
            runs["point_fp64"]["seconds"] / runs["point_fp64_sectors"]["seconds"], 3)
    return out


def _time_events(fn, reps):
    """Average milliseconds of fn() over reps calls between two events on the current stream."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_reference(nbytes, reps=400):
    """A plain device-to-device copy (torch) moving the same number of HBM bytes
    as one headline dslash (half read, half written), on rotating buffers:
    what a kernel with no arithmetic and no gathers achieves at this size."""
    import torch
    half = int(nbytes) // 2
    nsets = max(2, int(np.ceil(ROTATE_BYTES / (2 * half))))
    src = [torch.ones(half, dtype=torch.uint8, device="cuda") for _ in range(nsets)]
    dst = [torch.empty(half, dtype=torch.uint8, device="cuda") for _ in range(nsets)]
    it = {"k": 0}

    def one():
        k = it["k"] % nsets
        dst[k].copy_(src[k])
        it["k"] += 1

    for _ in range(2 * nsets):
        one()
    ms = _time_events(one, reps)
    return {"bytes": 2 * half, "us": round(ms * 1e3, 3), "gbs": round(2 * half / (ms * 1e-3) / 1e9, 1),
            "frac": round(2 * half / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def launch_floor(reps=1000):
    """Back-to-back launches of the smallest kernel (a one-element fill) timed as
    the headline is: the per-launch floor that any kernel pays in such a chain."""
    import torch
    t = torch.empty(1, dtype=torch.float32, device="cuda")
    f = lambda: t.fill_(1.0)  # noqa: E731
    for _ in range(20):
        f()
    return {"us": round(_time_events(f, reps) * 1e3, 3), "kernel": "one-element fill, back to back"}


BATCH_DIMS = (64, 32, 32, 32)
MULTI_DIMS = [(8, 8, 8, 8), (12, 12, 12, 12), (32, 16, 16, 16)]


def batch_leg(log):
    """Batching of the stencil.
    (i) The 12 spin-colour point sources on 32^3 x 64 with FP32 spinors and
        18-real FP32 links: one multi-RHS Q apply (links staged once per tile)
        against 12 single-RHS applies of the same data.  Algorithmic bytes per
        site: 12 x (96 in + 96 out) + 4 x 72 links = 2592 batched, 12 x 480 single.
    (ii) One persistent launch of Q over 8^4 + 12^4 + 16^3x32 at 4 RHS each
        (F32 spinors, 12-real links; 155904 sites x (4 x 192 + 4 x 48) B) against
        the three lattices launched one after the other, on 3 rotating copies."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dev = torch.device("cuda")
    out = {}
    t0 = time.perf_counter()
    g = ndq.Geometry(BATCH_DIMS)
    v = g.volume
    u = torch.from_numpy(synthetic.gauge_field(BATCH_DIMS)).to(dev)
    U = ndq.GaugeField.pack(g, u, ndq.F32, 18)
    # the even/odd dslash on the same 32^3x64 links in the headline format (F32
    # spinors, 12-real F32 links): 403 MB of links and 2 x 101 MB of spinors per
    # apply, beyond the 256 MB Infinity Cache, so every apply streams from HBM
    U12 = ndq.GaugeField.pack(g, u, ndq.F32, 12)
    del u
    e = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(v // 2)).to(dev), ndq.F32, ndq.EVEN)
    o = e.like(parity=ndq.ODD)
    tune = ndq.autotune(g, U12, ndq.F32, reps=50)
    par = {"k": 0}

    def dslash_big():
        if par["k"] % 2 == 0:
            ndq.apply_dslash(g, U12, e, o)
        else:
            ndq.apply_dslash(g, U12, o, e)
        par["k"] += 1

    for _ in range(10):
        dslash_big()
    ms_d = _time_events(dslash_big, 200)
    alg_d = 576 * (v // 2)
    out["dslash_32c64"] = {
        "workload": "even/odd dslash, 32^3x64, F32 spinors, 12-real F32 links, random SU(3) links (width 0.3)",
        "us": round(ms_d * 1e3, 3), "alg_bytes": alg_d, "gbs": round(alg_d / (ms_d * 1e-3) / 1e9, 1),
        "frac_hbm": round(alg_d / (ms_d * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "gflops": round(FLOP_PER_SITE * (v // 2) / (ms_d * 1e-3) / 1e9, 1),
        "launch": {"block": tune["block"], "xcd_remap": tune["xcd_remap"], "chunked_order": tune["order"]}}
    log(f"batch leg: dslash 32^3x64 {ms_d * 1e3:.2f} us ({out['dslash_32c64']['frac_hbm']:.3f} of HBM peak)")
    # the same with 18-real links (no reconstruction; 768 B per site)
    tune18 = ndq.autotune(g, U, ndq.F32, reps=50)
    par18 = {"k": 0}

    def dslash_big18():
        if par18["k"] % 2 == 0:
            ndq.apply_dslash(g, U, e, o)
        else:
            ndq.apply_dslash(g, U, o, e)
        par18["k"] += 1

    for _ in range(10):
        dslash_big18()
    ms_d18 = _time_events(dslash_big18, 200)
    alg_d18 = 768 * (v // 2)
    out["dslash_32c64_r18"] = {
        "workload": "even/odd dslash, 32^3x64, F32 spinors, 18-real F32 links, random SU(3) links (width 0.3)",
        "us": round(ms_d18 * 1e3, 3), "alg_bytes": alg_d18, "gbs": round(alg_d18 / (ms_d18 * 1e-3) / 1e9, 1),
        "frac_hbm": round(alg_d18 / (ms_d18 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "gflops": round(FLOP_PER_SITE * (v // 2) / (ms_d18 * 1e-3) / 1e9, 1),
        "launch": {"block": tune18["block"], "xcd_remap": tune18["xcd_remap"], "chunked_order": tune18["order"]}}
    log(f"batch leg: dslash 32^3x64 18-real {ms_d18 * 1e3:.2f} us "
        f"({out['dslash_32c64_r18']['frac_hbm']:.3f} of HBM peak)")
    del e, o, U12
    canon = torch.zeros((12, v, 4, 3), dtype=torch.complex128, device=dev)
    for s in range(4):
        for c in range(3):
            canon[3 * s + c, 0, s, c] = 1.0
    x = ndq.SpinorField.pack(g, canon, ndq.F32, ndq.FULL)
    del canon
    y = x.like()
    rb = g.spinor_bytes(ndq.F32, ndq.FULL, 1)
    xs = [ndq.SpinorField(g, ndq.F32, ndq.FULL, 1, buffer=x.buf[r * rb:(r + 1) * rb]) for r in range(12)]
    ys = [ndq.SpinorField(g, ndq.F32, ndq.FULL, 1, buffer=y.buf[r * rb:(r + 1) * rb]) for r in range(12)]
    torch.cuda.synchronize()
    log(f"batch leg: 32^3x64 fields {time.perf_counter() - t0:.1f} s")

    tuned = ndq.ndq.autotune_mrhs(g, U, ndq.F32, 12, ny=2, reps=5)

    def batched():
        ndq.apply_Q(g, U, M, x, y)

    def singles():
        for r in range(12):
            ndq.apply_Q(g, U, M, xs[r], ys[r])

    batched()
    singles()
    ms_b = _time_events(batched, 10)
    ms_s = _time_events(singles, 5)
    alg_b = 2592 * v
    out["point_sources_32c64"] = {
        "workload": "Q on 12 point-source right-hand sides, 32^3x64, F32 spinors, 18-real F32 links",
        "batched_ms": round(ms_b, 4), "single_rhs_ms": round(ms_s, 4), "speedup": round(ms_s / ms_b, 3),
        "alg_bytes_batched": alg_b, "alg_bytes_single": 12 * 480 * v,
        "batched_hbm_gbs": round(alg_b / (ms_b * 1e-3) / 1e9, 1),
        "batched_frac_hbm": round(alg_b / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "single_hbm_gbs": round(12 * 480 * v / (ms_s * 1e-3) / 1e9, 1)}
    out["point_sources_32c64"]["work_order"] = ndq.ndq.get_mrhs_launch(g, ndq.F32, ndq.F32, 18, 12, 2)
    out["point_sources_32c64"]["autotune_mrhs"] = {k: tuned[k] for k in ("nshapes", "us_best", "us_previous")}
    log(f"batch leg: 12 point sources batched {ms_b:.3f} ms vs single {ms_s:.3f} ms")
    del x, y, xs, ys, U
    torch.cuda.empty_cache()

    sets = []
    nsites = 0
    for copy in range(3):
        jobs = []
        for k, d in enumerate(MULTI_DIMS):
            gg = ndq.Geometry(d)
            if copy == 0:
                nsites += gg.volume
            uu = torch.from_numpy(synthetic.gauge_field(d, seed=1001 + k)).to(dev)
            UU = ndq.GaugeField.pack(gg, uu, ndq.F32, 12)
            xx = ndq.SpinorField.pack(gg, torch.from_numpy(synthetic.spinor(gg.volume, nrhs=4, seed=1002 + k)).to(dev),
                                      ndq.F32, ndq.FULL)
            jobs.append((gg, UU, M, xx, xx.like()))
        sets.append(jobs)
    it = {"k": 0}

    def multi():
        ndq.apply_Q_multi(sets[it["k"] % 3])
        it["k"] += 1

    def separate():
        for (gg, UU, m, xx, yy) in sets[it["k"] % 3]:
            ndq.apply_Q(gg, UU, m, xx, yy)
        it["k"] += 1

    multi()
    separate()
    # the persistent grid (a multiple of the resident workgroups) picked by its autotuner
    grid_tune = ndq.ndq.autotune_multi(sets[0], reps=20)
    ms_m = _time_events(multi, 30)
    ms_sep = _time_events(separate, 30)
    alg_m = nsites * (4 * 192 + 4 * 48)
    out["multi_lattice"] = {
        "workload": "Q on 8^4 + 12^4 + 16^3x32 at 4 RHS each, F32 spinors, 12-real F32 links",
        "sites": nsites, "persistent_ms": round(ms_m, 4), "separate_ms": round(ms_sep, 4),
        "speedup": round(ms_sep / ms_m, 3), "alg_bytes": alg_m,
        "persistent_hbm_gbs": round(alg_m / (ms_m * 1e-3) / 1e9, 1),
        "grid_factor": grid_tune["factor"],
        "autotune_grid_us": {str(f): round(u, 2) for f, u in grid_tune["us"].items()}}
    log(f"batch leg: multi-lattice persistent {ms_m:.4f} ms (grid factor {grid_tune['factor']}) vs separate "
        f"{ms_sep:.4f} ms")
    return out


def graph_leg(log):
    """Rational sign(Q) (Zolotarev, 12 shifts, no low modes, FP64) applied with
    each block of 8 multi-shift iterations launched eagerly or replayed from a
    captured HIP graph; wall time per apply (host synchronised)."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dev = torch.device("cuda")
    out = {}
    for d in ((8, 8, 8, 8), (32, 16, 16, 16)):
        g = ndq.Geometry(d)
        U = ndq.GaugeField.pack(g, torch.from_numpy(synthetic.gauge_field(d)).to(dev), ndq.F64, 18)
        x = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(g.volume)).to(dev), ndq.F64, ndq.FULL)
        y = x.like()
        ap = ndq.Approx(ndq.ZOLOTAREV, 0.08, 12)
        res = {}
        for graph in (False, True):
            ov = ndq.Overlap(g, M, ap, LAM_MAX, tol=1e-10, check_every=8, graph=graph)
            st = ndq.apply_sign(g, U, ov, x, y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = 5
            for _ in range(n):
                st = ndq.apply_sign(g, U, ov, x, y)
            torch.cuda.synchronize()
            res["graph" if graph else "eager"] = {"ms": round((time.perf_counter() - t0) * 1e3 / n, 3),
                                                  "cg_iterations": st["iterations"]}
        res["speedup"] = round(res["eager"]["ms"] / res["graph"]["ms"], 3)
        out["x".join(str(k) for k in d[::-1])] = res
        log(f"graph leg: {d} eager {res['eager']['ms']} ms, graph {res['graph']['ms']} ms")
    return out


INDEX_DIMS = (32, 16, 16, 16)


def index_leg(log):
    """Index of the massless D_N by zero-mode counting (ndq_index_DN) on a
    16^3 x 32 background with quantised fluxes (q01, q23) = (1, 1) in the
    diag(e^{i phi}, e^{-i phi}, 1) embedding (topological charge 2), light noise
    (width 0.2) and a random gauge transformation; FP64 sign (minimax
    polynomial, delta <= 1e-10, 4 exact low modes) on 12-real FP64 links (the
    field is SU(3), so the third row is exact to rounding).  Expected index: -2."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    g = ndq.Geometry(INDEX_DIMS)
    u = synthetic.flux_gauge_field(INDEX_DIMS, 1, 1, noise=0.2, gauge_seed=synthetic.SEED_HAAR)
    U = ndq.GaugeField.pack(g, torch.from_numpy(u).to(dev), ndq.F64, 12)
    del u
    start = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.start_vector(g.volume)).to(dev), ndq.F64, ndq.FULL)
    modes, nu, _, lm = ndq.lowmodes_compute(g, U, M, LAM_MAX, start, 4, tol=1e-10)
    t_modes = time.perf_counter() - t0
    ap = poly_for(ndq, ((lm["lam_next"] - lm["rho_next"]) / LAM_MAX) ** 2, 1e-10)
    ov = ndq.Overlap(g, M, ap, LAM_MAX, modes=modes, nu=nu)
    torch.cuda.synchronize()
    r = ndq.index_DN(g, U, ov, start, block=8, zero_cut=1e-7)
    # one sign apply alone, for the cost per application
    x = start.like()
    y = start.like()
    x.buf.copy_(start.buf)
    ndq.apply_sign(g, U, ov, x, y)
    ms_sign = _time_events(lambda: ndq.apply_sign(g, U, ov, x, y), 5)
    out = {"workload": "index of the massless D_N, 16^3x32 flux background (q01 = q23 = 1, noise 0.2, gauge "
                       "transformed), FP64 polynomial sign (degree %d, delta %.1e), 4 exact low modes, 12-real FP64 links" % (ap.n, ap.delta),
           "n_plus": r["n_plus"], "n_minus": r["n_minus"], "index": r["index"], "index_expected": -2,
           "block": r["block"], "sweeps": r["sweeps"], "filter_degree": r["degree"], "sign_applies": r["sign_applies"],
           "seconds": round(r["seconds"], 3), "sign_ms": round(ms_sign, 3),
           "first_nonzero_theta": [r["theta_plus"][r["n_plus"]], r["theta_minus"][r["n_minus"]]],
           "setup_lowmodes_s": round(t_modes, 2)}
    log(f"index leg: index {r['index']} (n+ {r['n_plus']}, n- {r['n_minus']}), {r['sign_applies']} sign applies, "
        f"{r['seconds']:.1f} s")
    return out


def autograd_leg(log):
    """S = psi^H Q^2 psi on 16^3 x 32 in FP64 through the torch autograd function
    (forward Q, backward Q and the su(3) force kernel, canonical tensors in and
    out), and the force kernel alone (4 links + psi + g read, 4 x 8 reals written
    per site)."""
    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    dev = torch.device("cuda")
    g = ndq.Geometry(DIMS)
    v = g.volume
    links = torch.from_numpy(synthetic.gauge_field(DIMS)).to(dev).requires_grad_(True)
    psi = torch.from_numpy(synthetic.spinor(v)).to(dev).requires_grad_(True)

    def step():
        y = ndq.QFunction.apply(psi, links, g, M)
        s = (y.conj() * y).real.sum()
        s.backward()

    step()
    ms_step = _time_events(step, 10)
    U = ndq.GaugeField.pack(g, links.detach(), ndq.F64, 18)
    x = ndq.SpinorField.pack(g, psi.detach(), ndq.F64, ndq.FULL)
    gy = ndq.SpinorField.pack(g, torch.from_numpy(synthetic.spinor(v, seed=4)).to(dev), ndq.F64, ndq.FULL)
    f = torch.empty((v, 4, 8), dtype=torch.float64, device=dev)
    from paper_1010_5636_amd.ndq import lib, _ptr, _check
    import ctypes

    def force_only():
        _check(lib().ndq_gauge_force(g.handle, ctypes.byref(U.desc), ctypes.byref(x.desc), ctypes.byref(gy.desc),
                                     _ptr(f), None, None))

    force_only()
    ms_f = _time_events(force_only, 50)
    # per site: its 4 links, psi and g once each (the x + mu neighbours are
    # other sites' own values), 4 x 8 force components written
    bytes_site = 4 * 144 + 2 * 192 + 4 * 8 * 8
    # gradient error: dS along one random su(3) direction omega (U -> exp(i h omega.T) U)
    # by central differences of S = |Q psi|^2, against sum omega . F with F the force
    # of the cotangent 2 Q psi
    y0 = ndq.SpinorField(g, ndq.F64, ndq.FULL)
    ndq.apply_Q(g, U, M, x, y0)
    gy2 = ndq.SpinorField.pack(g, 2.0 * y0.unpack()[0], ndq.F64, ndq.FULL)
    force = ndq.gauge_force(g, U, x, gy2)[0]
    om = torch.from_numpy(synthetic.su3_directions(v, 1, seed=synthetic.SEED_DIRECTIONS)[0]).to(dev)
    analytic = float((om * force).sum())
    gen = torch.from_numpy(synthetic.su3_generators()).to(dev)
    hmat = torch.einsum("vma,aij->vmij", om.to(torch.complex128), gen)
    h = 1e-5

    def action(sgn):
        up = torch.linalg.matrix_exp(1j * sgn * h * hmat) @ links.detach()
        Uh = ndq.GaugeField.pack(g, up.contiguous(), ndq.F64, 18)
        yh = ndq.SpinorField(g, ndq.F64, ndq.FULL)
        ndq.apply_Q(g, Uh, M, x, yh)
        return float((yh.buf.view(torch.float64) ** 2).sum())

    fd = (action(1) - action(-1)) / (2 * h)
    grad_err = abs(fd - analytic) / abs(analytic)
    out = {"workload": "S = psi^H Q^2 psi, 16^3x32, FP64, 18-real links",
           "autograd_step_ms": round(ms_step, 4), "force_kernel_us": round(ms_f * 1e3, 2),
           "gradient_check": {"direction": "random su(3), seed 1004", "h": h, "central_difference": fd,
                              "analytic": analytic, "rel_error": grad_err},
           "force_alg_bytes": bytes_site * v,
           "force_hbm_gbs": round(bytes_site * v / (ms_f * 1e-3) / 1e9, 1)}
    log(f"autograd leg: step {ms_step:.3f} ms, force kernel {ms_f * 1e3:.1f} us, gradient rel. error {grad_err:.1e}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--formats", default="all", help="comma list of format names or 'all'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--warm-cache", action="store_true", help="reuse one buffer set (data stays in cache)")
    ap.add_argument("--graph", action="store_true", help="replay the timed launches from a HIP graph")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run a device-to-device copy of BYTES bytes (counter calibration)")
    ap.add_argument("--no-solve", action="store_true", help="skip the 24^3x48 D_N solve leg")
    ap.add_argument("--sectors-fp64", action="store_true",
                    help="also run the plain-FP64 CGNE / chirality-sector comparison on a point source")
    ap.add_argument("--no-extra", action="store_true", help="skip the batching, graph and autograd legs")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--launch", default="", metavar="BLOCK,XCD",
                    help="force one launch shape for every format (no autotuning), e.g. 0,1")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: multi-GPU runs are not supported "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    import synthetic
    import paper_1010_5636_amd as ndq
    from paper_1010_5636_amd.ndq import lib

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    lib()  # fails loudly if libndq.so is missing
    dev = torch.device("cuda")
    g = ndq.Geometry(DIMS)
    vh = g.volume // 2
    u_canon = torch.from_numpy(synthetic.gauge_field(DIMS)).to(dev)
    psi_canon = torch.from_numpy(synthetic.spinor(vh)).to(dev)

    fmts = FORMATS if args.formats == "all" else [f for f in FORMATS if f[0] in args.formats.split(",")]
    results = {}
    for name, sp, lp, recon in fmts:
        bps = bytes_per_site(sp, lp, recon)
        set_bytes = g.gauge_bytes(lp, recon) + 2 * g.spinor_bytes(sp, ndq.EVEN, 1)
        nsets = 1 if args.warm_cache else max(2, int(np.ceil(ROTATE_BYTES / set_bytes)))
        sets = []
        for s in range(nsets):
            U = ndq.GaugeField.pack(g, u_canon, lp, recon)
            e = ndq.SpinorField.pack(g, psi_canon * (1.0 + 0.01 * s), sp, ndq.EVEN)
            o = e.like(parity=ndq.ODD)
            sets.append((U, e, o))
        torch.cuda.synchronize()
        if args.launch:
            b, x = (int(t) for t in args.launch.split(","))
            ndq.set_launch_for(sp, lp, recon, b, bool(x))
            tune = None
        elif args.no_autotune:
            tune = None
        else:
            tune = ndq.autotune(g, sets[0][0], sp, reps=200, rotate_bytes=int(ROTATE_BYTES))
        launch = ndq.ndq.get_launch_lattice(g, sp, lp, recon, 1)

        def step(k):
            U, e, o = sets[k % nsets]
            if (k // nsets) % 2 == 0:
                ndq.apply_dslash(g, U, e, o)
            else:
                ndq.apply_dslash(g, U, o, e)

        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        # Timed region: K back-to-back launches on the current stream between two
        # HIP events; the per-launch average is that elapsed time over K (the
        # queue hides dispatch latency, as in a solver's dependent chain).
        # With --graph the K launches are replayed from a captured graph.
        graph = None
        gsize = 2 * nsets
        if args.graph:
            graph = torch.cuda.CUDAGraph()
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                with torch.cuda.graph(graph, stream=stream):
                    for k in range(gsize):
                        step(k)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            reps, rem = divmod(args.steps, gsize)
        else:
            reps, rem = 0, args.steps
        t_start = torch.cuda.Event(enable_timing=True)
        t_stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t_start.record()
        for _ in range(reps):
            graph.replay()
        for k in range(rem):
            step(k)
        t_stop.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms_total = t_start.elapsed_time(t_stop)
        k_avg = ms_total * 1e-3 / args.steps
        gflops = FLOP_PER_SITE * vh * args.steps / (ms_total * 1e-3) / 1e9
        alg_bytes = bps * vh
        # the no-reuse count (8 neighbour spinors and 8 links per output site,
        # plus the output), as GPU lattice codes often quote it
        noreuse = (8 * (SPINOR_BYTES[sp] + recon * LINK_REAL_BYTES[lp]) + SPINOR_BYTES[sp]) * vh
        results[name] = {
            "gflops": round(gflops, 1),
            "effective_gbs_no_reuse": noreuse / k_avg / 1e9,
            "ms_per_step": ms_total / args.steps,
            "wall_s": wall,
            "kernel_us_avg": k_avg * 1e6,
            "alg_bytes_per_launch": alg_bytes,
            "hbm_gbs": alg_bytes / k_avg / 1e9,
            "kernel_gflops": FLOP_PER_SITE * vh / k_avg / 1e9,
            "frac_hbm": alg_bytes / k_avg / 1e9 / HBM_PEAK_GBS,
            "nsets": nsets,
            "launch": launch,
            "autotune_us": None if tune is None else {k: round(t, 3) for k, t in tune["us"].items()},
        }
        if (name, sp, lp, recon) == fmts[0] and not args.warm_cache:
            # the same dslash on one buffer set (37.7 MB at F32-12, resident in the
            # 256 MB last-level cache): the cache-warm rate, next to the HBM-streamed one
            U0, e0, o0 = sets[0]
            warm = {"k": 0}

            def warm_step():
                if warm["k"] % 2 == 0:
                    ndq.apply_dslash(g, U0, e0, o0)
                else:
                    ndq.apply_dslash(g, U0, o0, e0)
                warm["k"] += 1

            for _ in range(20):
                warm_step()
            us_warm = _time_events(warm_step, args.steps) * 1e3
            results[name]["warm_cache"] = {"us": round(us_warm, 3),
                                           "gflops": round(FLOP_PER_SITE * vh / (us_warm * 1e-6) / 1e9, 1),
                                           "alg_gbs": round(alg_bytes / (us_warm * 1e-6) / 1e9, 1)}
        if (name, sp, lp, recon) == fmts[0] and not args.graph:
            # the even-site Schur operator Qhat_ee (two dslashes and the site
            # term) and the dslash replayed from a captured graph of 2 x nsets launches
            tmps = [e.like(parity=ndq.ODD) for (_, e, _) in sets]
            outs = [e.like() for (_, e, _) in sets]
            it = {"k": 0}

            def qhat():
                k = it["k"] % nsets
                U, e, _ = sets[k]
                ndq.apply_Qhat_ee(g, U, M, e, outs[k], tmps[k])
                it["k"] += 1

            for _ in range(nsets):
                qhat()
            results[name]["qhat_ee_us"] = _time_events(qhat, 500) * 1e3
            del tmps, outs
            gph = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            with torch.cuda.stream(cs):
                with torch.cuda.graph(gph, stream=cs):
                    for k in range(2 * nsets):
                        step(k)
            torch.cuda.synchronize()
            gph.replay()
            results[name]["graph_replay_us"] = _time_events(gph.replay, max(1, 1000 // (2 * nsets))) * 1e3 / (2 * nsets)
            del gph
        del sets, graph
        torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the shapes tuned on the dslash stay out of the legs below (their full-Q
    # applies run with the default shape)
    ndq.set_launch(0, True)
    head = fmts[0][0]
    hr = results[head]
    traffic = read_traffic(head, hr["launch"])
    out = {
        "metric": "Dslash GFLOP/s + HBM GB/s; D_N solves/s mixed vs FP64 at 1e-10 rel resid",
        "value": hr["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hr["ms_per_step"], 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fmts[0][1] != 0 else "f64",
        "data": "synthetic",
        "config": {"workload": "even/odd Wilson dslash, 16^3x32, m=-1.4, random SU(3) links (width 0.3), "
                               f"{head} ({'F16' if fmts[0][1] == 2 else 'F32' if fmts[0][1] == 1 else 'F64'} spinors, "
                               f"{fmts[0][3]}-real links), HBM-streamed (rotating buffer sets)"
                               if not args.warm_cache else f"{head}, warm cache",
                   "dims": list(DIMS), "flop_per_site": FLOP_PER_SITE, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(hr["hbm_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(hr["frac_hbm"], 4), "traffic": traffic,
                     "kernel": kernel_name(hr["launch"]), "alg_bytes_per_launch": hr["alg_bytes_per_launch"],
                     "kernel_us_avg": round(hr["kernel_us_avg"], 3),
                     "copy_same_bytes": copy_reference(hr["alg_bytes_per_launch"]),
                     "launch_floor": launch_floor()},
        "variants": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in r.items()}
                     for k, r in results.items()},
    }
    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731
    if not args.no_solve:
        out["dn_solve"] = solve_leg(log, args.sectors_fp64)
    if not args.no_extra:
        out["batching"] = batch_leg(log)
        out["graph_multishift"] = graph_leg(log)
        out["autograd"] = autograd_leg(log)
        out["index"] = index_leg(log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline"]["tau_measured"] = cpu_tau()
        out["cpu_baseline"]["extrapolated"] = extrapolated_cpu(out["cpu_baseline"], out.get("dn_solve"))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
