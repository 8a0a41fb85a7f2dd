#!/usr/bin/env python3
"""Benchmark of the initial-guess hot path on one MI355X.

Workload (defaults): 7-point Helmholtz (-Laplacian_h + 10 I) on a 256^3 grid
of the unit cube (16,777,216 unknowns), right-hand sides b_n = sum of 16
seeded plane-wave modes with amplitudes sin(w_k t_n + phi_k), dt = 0.005.
One step = one time step of the whole hot path for every method:
  b_n (device RHS kernel) -> guess_form -> Jacobi-PCG to ||r|| <= 1e-8 ||b||
  -> guess_update,
for least-squares extrapolation EXTRAP(2, 8) and A-orthonormal projection
PROJ(8), both with FP64 history.  W warm-up steps fill the histories first.

value = guess form+update HBM throughput in GB/s: algorithmic bytes of every
guess kernel in the timed steps divided by their device time (HIP events on
the library's stream).  PCG iterations and ms per step are reported per
method.  The JSON line also carries the roofline of the dominant guess kernel
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# kernels launched per call, in order (see include/libguess.h, guess_kernel_times)
KERNELS = {
    ("extrap", "form"): ["extrap_form"],
    ("extrap", "update"): ["ring_store"],
    ("last", "form"): ["extrap_form"],
    ("last", "update"): ["ring_store"],
    ("spextrap", "form"): ["extrap_form"],
    ("spextrap", "update"): ["ring_store"],
    ("proj", "form"): ["proj_dots", "proj_fin", "proj_combine"],
    ("proj", "update"): ["proj_apply", "proj_fin", "proj_reorth", "proj_fin", "proj_gs_write", "proj_fin"],
}
for _m in ("projqr", "proj_l2", "projqr_l2"):
    KERNELS[(_m, "form")] = KERNELS[("proj", "form")]
    KERNELS[(_m, "update")] = KERNELS[("proj", "update")]
for _m in ("proj_raw", "projqr_raw"):
    KERNELS[(_m, "form")] = ["raw_dots", "raw_solve", "raw_combine"]
    KERNELS[(_m, "update")] = ["raw_store", "raw_apply", "raw_fin"]
RING = ("extrap", "last", "spextrap")
RAW = ("proj_raw", "projqr_raw")


def kernel_names(method, call, dtype="f64"):
    """Kernels of one call in launch order; an FP16 ring store is followed by the kernel that
    stores the slot again when the solution's exponent differs from the previous one's."""
    if method in RING and call == "update" and dtype == "f16":
        return ["ring_store", "ring_fix"]
    if method in RAW and call == "update" and dtype == "f16":
        return ["raw_store", "raw_fix", "raw_apply", "raw_fin"]
    return KERNELS[(method, call)]


def kernel_rw(method, call, N, s, k_or_d, M, restart, faces=0, dtype="f64", fixed=False):
    """Algorithmic HBM bytes (read, written) of each kernel of one call (list, launch order).

    `faces`: bytes of the operator's face arrays, read by the fused operator
    apply of a variable-coefficient workload.  `fixed`: an FP16 ring store that
    had to store the slot again (the ring_fix kernel moved the same bytes)."""
    f16 = dtype == "f16"
    if method in RING:
        if call == "form":
            return [(N * k_or_d * s, N * 8)] if k_or_d > 0 else []
        if f16:
            return [(N * 8, N * s), (N * 8, N * s) if fixed else (0, 0)]
        return [(N * 8, N * s)]
    d = k_or_d
    if call == "form":
        return [(N * (d * s + 8), 0) if d > 0 else (0, 0), (0, 0), (N * d * s, N * 8)]
    if method in RAW:
        # store the solution; A on the stored vector fused with its Gram row against the nd
        # solutions that stay (a full history restarts, or drops its oldest)
        nd = d if d < M else (M - 1 if method == "projqr_raw" else 0)
        store = [(N * 8, N * s)] + ([(N * 8, N * s) if fixed else (0, 0)] if f16 else [])
        return store + [(N * (nd + 1) * s + faces, 0), (0, 0)]
    if restart and f16:
        # the apply pass reads x and writes A x with max |x|, |A x|; the write kernel stores the pair
        return [(N * 8 + faces, N * 8), (0, 0), (0, 0), (0, 0), (N * 16, N * 2 * s), (0, 0)]
    if restart:
        return [(N * 8 + faces, N * 2 * s), (0, 0), (0, 0), (0, 0), (0, 0), (0, 0)]
    if f16:
        reorth = N * (2 * d * s + 16)      # also forms x - X c1 for the pair's exponent
    else:
        reorth = N * ((1 if method.endswith("_l2") else 2) * d * s + 8)
    apply = (N * (8 + d * s) + faces, N * 8)
    if method.startswith("projqr") and d == M:      # rolling drop: every column rotated in place
        return [apply, (0, 0), (reorth, 0), (0, 0), (N * (2 * d * s + 16), N * 2 * d * s), (0, 0)]
    return [apply, (0, 0), (reorth, 0), (0, 0), (N * (2 * d * s + 16), N * 2 * s), (0, 0)]


def kernel_bytes(method, call, N, s, k_or_d, M, restart, faces=0, dtype="f64", fixed=False):
    """Algorithmic HBM bytes of each kernel of one call (list, launch order): read + written."""
    return [r + w for r, w in kernel_rw(method, call, N, s, k_or_d, M, restart, faces, dtype, fixed)]


def mixed_roof(read, write, read_roof, write_roof):
    """Bandwidth a kernel moving `read` and `write` bytes reaches at the measured read and
    write roofs: (read + write) / (read / R + write / W)."""
    if read + write <= 0:
        return None
    return (read + write) / (read / read_roof + write / write_roof)


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--n", type=int, default=256)
    p.add_argument("--workload", choices=("helmholtz", "varcoef"), default="helmholtz",
                   help="varcoef: -div(kappa grad u) + 10 u, kappa = exp(g), g a unit-variance Gaussian "
                        "field with correlation length 0.1 (the largest configuration: --n 384 --M 16)")
    p.add_argument("--M", type=int, default=8)
    p.add_argument("--degree", type=int, default=2)
    p.add_argument("--modes", type=int, default=16)
    p.add_argument("--dt", type=float, default=0.005)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--rtol", type=float, default=1e-8)
    p.add_argument("--eps-rel", type=float, default=0.0,
                   help="projection: relative rejection threshold of a new vector (<= 0: the library's "
                        "default for the storage format, 1e-6 for FP64)")
    p.add_argument("--precision-dtypes", default="f32,f16,bf16")
    p.add_argument("--precision-methods", default="extrap,proj,proj_raw,projqr_raw",
                   help="methods of the reduced-precision runs (proj_raw: reduced precision only)")
    p.add_argument("--progress", action="store_true", help="print a line to stderr after every step")
    p.add_argument("--fields", choices=("one", "ins"), default="one",
                   help="ins: per step three velocity components (shift --velocity-shift) and a pressure "
                        "(shift 0), each with its own right-hand sides and guess contexts")
    p.add_argument("--velocity-shift", type=float, default=2.0e4,
                   help="velocity Helmholtz shift, 1/(nu dt) for nu = 1e-2, dt = 5e-3")
    p.add_argument("--isolated", action="store_true",
                   help="only time each guess kernel in isolation (MALL evicted between launches)")
    p.add_argument("--reps", type=int, default=20)
    p.add_argument("--concurrent", action="store_true",
                   help="four independent fields (three velocity components, a pressure), each with its own "
                        "operator, guess context and HIP stream: the steps run field after field on one host "
                        "thread, then with one host thread per field; reports ms per step of both")
    p.add_argument("--adjoint", action="store_true",
                   help="time the differentiable sequence instead: forward solves and the reverse-time "
                        "adjoint solves, each with its own guess history, on --adjoint-n^3 for --adjoint-steps")
    p.add_argument("--adjoint-n", type=int, default=128)
    p.add_argument("--adjoint-steps", type=int, default=100)
    p.add_argument("--shard-nz", type=int, default=0,
                   help="with --isolated: time the kernels on an n x n x NZ slab (one z-slab of a "
                        "multi-GPU split) instead of the n^3 grid")
    p.add_argument("--stop-rule", choices=("rhs", "initresid"), default="rhs",
                   help="PCG stop: ||r|| <= rtol ||b|| or ||r|| < rtol max(||r0||, 1)")
    p.add_argument("--rhs", choices=("planewave", "gaussian"), default="planewave",
                   help="gaussian: a moving Gaussian source (solutions not confined to a low-rank space)")
    p.add_argument("--dtype", default="f64", choices=["f64", "f32", "f16", "bf16"])
    p.add_argument("--methods", default="extrap,proj")
    p.add_argument("--maxit", type=int, default=5000)
    p.add_argument("--cpu-baseline", dest="cpu", action="store_true", default=True)
    p.add_argument("--no-cpu-baseline", dest="cpu", action="store_false")
    p.add_argument("--cpu-steps", type=int, default=10)
    p.add_argument("--no-small-sequence", dest="small", action="store_false", default=True,
                   help="skip the 32^3 whole-sequence run (e.g. under a profiler)")
    p.add_argument("--precision-steps", type=int, default=10,
                   help="timed steps of each FP32/FP16/BF16 history run (0: skip)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run the plain copy kernel (1 GiB -> 1 GiB, 5 launches); used to scale "
                        "the FETCH_SIZE / WRITE_SIZE counters of a profiled run")
    p.add_argument("--traffic-summary", nargs=4, metavar=("FETCH", "WRITE", "FETCH_COPY", "WRITE_COPY"),
                   help="no GPU: write profiles/hbm_traffic.txt from four rocprofv3 --pmc output folders "
                        "(FETCH_SIZE and WRITE_SIZE of a profiled bench run whose JSON line is FETCH/bench.json, "
                        "and of --calibrate-copy)")
    return p.parse_args()


def copy_roof(L, nbytes=1 << 30, reps=5, mode=None):
    """Bandwidth of the library's plain copy kernel (nbytes read + nbytes written), or with
    `mode` of its read-only (nbytes read) or write-only (nbytes written) reference."""
    import torch

    mode = L.ROOF_COPY if mode is None else mode
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty(2048 if mode in (L.ROOF_READ, L.ROOF_READ_STREAMS) else nbytes // 8, dtype=torch.float64,
                      device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    L.guess_roof_kernel(mode, dst, src, nbytes, L.stream_handle())
    ts = []
    for _ in range(reps):
        ev[0].record()
        L.guess_roof_kernel(mode, dst, src, nbytes, L.stream_handle())
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    del src, dst
    t = sorted(ts)[len(ts) // 2]
    return (2 if mode == L.ROOF_COPY else 1) * nbytes / (t * 1e-3) / 1e9


def roofs(L, reps=9):
    """Measured copy, read-only and write-only bandwidths (GB/s), 1 GiB each, median of `reps`
    launches (single measurements vary by about 3 % between runs).  The read roof is the better
    of two patterns: one stream on 2048 workgroups, and 16 streams side by side on the
    reduction grid (what a Gram-Schmidt pass reads)."""
    one = copy_roof(L, reps=reps, mode=L.ROOF_READ)
    many = copy_roof(L, reps=reps, mode=L.ROOF_READ_STREAMS)
    return {"copy_roof_GBps": copy_roof(L, reps=reps), "read_roof_GBps": max(one, many),
            "read_roof_one_stream_GBps": one, "read_roof_16_streams_GBps": many,
            "write_roof_GBps": copy_roof(L, reps=reps, mode=L.ROOF_WRITE)}


def hbm_traffic(kernel):
    """(counter-measured HBM bytes, algorithmic bytes) per launch of `kernel` in the profiled
    run, if still valid.

    Read from profiles/hbm_traffic.txt (written from two rocprofv3 --pmc runs,
    FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel calibration); the
    entry is ignored (None) when the kernel sources changed since then.
    """
    import hashlib

    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in sorted(rec.get("sources", "").split(",")):
        if not f:
            continue
        fp = os.path.join(ROOT, f)
        if not os.path.exists(fp):
            return None
        h.update(open(fp, "rb").read())
    if rec.get("sha256") != h.hexdigest():
        return None
    v = rec.get(f"{kernel}.bytes_per_launch")
    a = rec.get(f"{kernel}.algorithmic_bytes_per_launch")
    return (float(v), float(a)) if v and a else None


# Kernel-name patterns of the counter CSVs -> bench kernel names; PCG's kernels with their
# algorithmic bytes per unknown (constant coefficient).
TRAFFIC_GUESS = [("extrap_form", "extrap_form_kernel"), ("ring_store", "ring_store_kernel"),
                 ("proj_dots", "proj_dots_kernel"), ("proj_combine", "proj_combine_kernel"),
                 ("proj_apply", "proj_apply_"), ("proj_reorth", "proj_reorth_kernel"),
                 ("proj_gs_write", "proj_gs_write_kernel")]
TRAFFIC_PCG = [("pcg_a_xupdate", "pcg_a_march_kernel<false, true>", 32, 24),
               ("pcg_a", "pcg_a_march_kernel<false, false>", 16, 16),
               ("pcg_b", "pcg_b_kernel<false>", 16, 8)]
TRAFFIC_SOURCES = ["paper_2009_10863_amd/_build.py", "paper_2009_10863_amd/csrc/common.h",
                   "paper_2009_10863_amd/csrc/extrap.hip", "paper_2009_10863_amd/csrc/launch.h",
                   "paper_2009_10863_amd/csrc/march.h", "paper_2009_10863_amd/csrc/pcg.hip",
                   "paper_2009_10863_amd/csrc/proj_impl.h", "paper_2009_10863_amd/csrc/proj_inst.hip",
                   "paper_2009_10863_amd/csrc/stencil.h"]


def traffic_summary(args):
    """profiles/hbm_traffic.txt from the counter runs: per kernel the mean FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads for the copy
    kernel moving 1 GiB -> 1 GiB, beside the algorithmic bytes per launch of the same run (the
    bench JSON line of the profiled command: every step timed, so its launches are the
    dispatches counted)."""
    import csv
    import glob
    import hashlib

    def counter(folder, name, pattern):
        # dispatches that moved data: a launch that returns at once (a projection call on an
        # empty history, PCG kernels of a batch after convergence) reads a few KiB
        vals = []
        for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                if row["Counter_Name"] == name and pattern in row["Kernel_Name"]:
                    vals.append(float(row["Counter_Value"]) * 1024.0)
        if not vals:
            return None, 0
        big = sorted(vals)[len(vals) // 2] * 0.01
        vals = [v for v in vals if v >= big]
        return sum(vals), len(vals)

    fdir, wdir, fcopy, wcopy = args.traffic_summary
    gib = float(1 << 30)
    fc, nfc = counter(fcopy, "FETCH_SIZE", "copy_kernel")
    wc, nwc = counter(wcopy, "WRITE_SIZE", "copy_kernel")
    fscale, wscale = gib / (fc / nfc), gib / (wc / nwc)
    run = json.loads(open(os.path.join(fdir, "bench.json")).read().strip().splitlines()[-1])
    N = run["config"]["n"] ** 3
    h = hashlib.sha256()
    for f in sorted(TRAFFIC_SOURCES):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    rows = []
    entries = [(k, pat, run["kernels"][k]["bytes_per_launch"], run["kernels"][k]["launches"], None, None)
               for k, pat in TRAFFIC_GUESS if k in run["kernels"]]
    entries += [(k, pat, (r + w) * N, None, r * N, w * N) for k, pat, r, w in TRAFFIC_PCG]
    for k, pat, alg, launches, ar, aw in entries:
        fb, nf = counter(fdir, "FETCH_SIZE", pat)
        wb, nw = counter(wdir, "WRITE_SIZE", pat)
        if fb is None or wb is None:
            continue
        # per launch: the run's totals over its launches that moved data (the bench's own count
        # for the guess kernels, whose launch on an empty history may only write)
        nl = launches if launches is not None else nf
        rd, wr = fb * fscale / nl, wb * wscale / nl
        rows.append(f"{k}.bytes_per_launch = {rd + wr:.0f}")
        rows.append(f"{k}.read_bytes_per_launch = {rd:.0f}")
        rows.append(f"{k}.write_bytes_per_launch = {wr:.0f}")
        rows.append(f"{k}.algorithmic_bytes_per_launch = {alg:.0f}")
        if ar is not None:
            rows.append(f"{k}.algorithmic_read_bytes_per_launch = {ar:.0f}")
            rows.append(f"{k}.algorithmic_write_bytes_per_launch = {aw:.0f}")
        rows.append(f"{k}.ratio = {(rd + wr) / alg:.4f}")
        rows.append(f"{k}.dispatches = {nf} fetch, {nw} write" +
                    (f" (bench launches {launches})" if launches is not None else ""))
    head = [
        f"# HBM bytes per launch, {run['config']['workload']}: FETCH_SIZE and WRITE_SIZE (KiB per dispatch,",
        "# one rocprofv3 --pmc run each), scaled by what the same counters read for the plain copy kernel",
        f"# moving 1 GiB -> 1 GiB (FETCH_SIZE x {fscale:.4f}, WRITE_SIZE x {wscale:.4f}); algorithmic bytes",
        "# of the guess kernels from the profiled run's own JSON line, of PCG's kernels per unknown",
        "# (pcg_a_xupdate: the odd iterations that also update x, 56 B; pcg_a: 32 B; pcg_b: 24 B).",
        "# Dispatches that return at once (reading < 1 % of the kernel's median) are left out.",
        "# Valid while the sources below hash to sha256.  Commands (from /tmp, TMPDIR=/tmp; the four",
        "# output folders as given to --traffic-summary):",
        "#   rocprofv3 --pmc FETCH_SIZE -f csv --kernel-include-regex \"extrap_form|ring_store|proj_|copy_kernel|pcg_\" "
        f"-d {fdir} -o bench -- python3 bench.py --steps 15 --warmup 0 --no-cpu-baseline "
        f"--no-small-sequence --precision-steps 0 > {fdir}/bench.json",
        f"#   (the same with WRITE_SIZE and {wdir})",
        f"#   rocprofv3 --pmc FETCH_SIZE -f csv --kernel-include-regex copy_kernel -d {fcopy} "
        "-o copy -- python3 bench.py --calibrate-copy",
        f"#   (the same with WRITE_SIZE and {wcopy})",
        f"#   python3 bench.py --traffic-summary {fdir} {wdir} {fcopy} {wcopy}",
        f"sources = {','.join(sorted(TRAFFIC_SOURCES))}",
        f"sha256 = {h.hexdigest()}",
        f"fetch_scale = {fscale:.6f}",
        f"write_scale = {wscale:.6f}",
    ]
    out = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    with open(out, "w") as f:
        f.write("\n".join(head + rows) + "\n")
    print(f"wrote {out}")


def cpu_baseline(args, s_bytes):
    """The oracle (NumPy FP64) timed on the host: guess form+update on a bounded sample of the
    benchmark's own workload.

    Sample: the plane-wave sequence of the benchmark (same seed, modes, dt, grid, M, degree),
    solutions exact (each one the same combination of the modes' DST-I solutions as its
    right-hand side is of the modes), histories filled over M untimed steps; then
    `cpu_steps` steps of EXTRAP(m, M) and PROJ(M) form+update are timed on one host thread
    and, from the same state, on all host cores (BLAS threads; NumPy's elementwise passes
    stay on one).  The oracle's own operator is applied once per projection update.
    Reported in the same algorithmic GB/s as the GPU value.  The oracle's guesses at the last
    two steps also serve as the FP64 reference of the library's guess error per history format
    (`guess_rel_err_vs_oracle`).
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    return _cpu_baseline(args, np, cores, threadpool_limits)


def _cpu_baseline(args, np, cores, threadpool_limits):
    import copy

    import synth
    from oracle import operator as oop
    from oracle.extrap import ExtrapHistory
    from oracle.projection import AOrthoProjection
    from oracle.sequence import run_sequence

    n, M, m = args.n, args.M, args.degree
    N = n ** 3
    Aop = oop.Operator(n)
    t_setup = time.perf_counter()
    p = synth.plane_wave_params(args.seed, args.modes)
    F = synth.plane_wave_modes(p, n)
    U = np.stack([oop.dst_solve(f, n, workers=cores) for f in F])      # A u_k = f_k
    amps = lambda step: synth.mode_amplitudes(p, step * args.dt)     # noqa: E731
    e = ExtrapHistory(M, m)
    P = AOrthoProjection(M, Aop, 1e-6)
    with threadpool_limits(limits=cores):
        for step in range(1, M + 1):
            x = amps(step) @ U
            e.update(x)
            P.update(x)
    setup_s = time.perf_counter() - t_setup
    state = copy.deepcopy((e, P))

    last = M + args.cpu_steps
    sample_steps = [s for s in (last - 1, last) if s > M]
    sampled = {}     # step -> (EXTRAP guess, PROJ guess) of the oracle

    def timed(threads, keep=False):
        ee, PP = copy.deepcopy(state)
        nbytes, secs = 0.0, 0.0
        with threadpool_limits(limits=threads):
            for step in range(M + 1, M + 1 + args.cpu_steps):
                a = amps(step)
                b, x = a @ F, a @ U
                t0 = time.perf_counter()
                ge = ee.form(N=N)
                ee.update(x)
                secs += time.perf_counter() - t0
                nbytes += N * (M * 8 + 8) + N * 16
                d = PP.d
                t0 = time.perf_counter()
                gp = PP.form(b)
                PP.update(x)
                secs += time.perf_counter() - t0
                restart = d == 0 or d >= M
                nbytes += 2 * N * (d * 8 + 8) + (N * (8 + 16) if restart else N * (5 * d * 8 + 16 + 40))
                if keep and step in sample_steps:
                    sampled[step] = (ge, gp)
        return nbytes / secs / 1e9, secs, PP.d

    one, one_s, d_end = timed(1)
    allc, all_s, _ = timed(cores, keep=True)
    vs_oracle = _precision_vs_oracle(args, np, n, M, m, F, U, amps, sampled) if args.precision_steps > 0 else None
    # the whole small sequence (32^3, 4 plane waves, 50 steps, dt = 0.01): guess -> PCG -> update
    n1 = 32
    op1 = oop.Operator(n1)
    p1 = synth.plane_wave_params(0, 4)
    rhs1 = [synth.plane_wave_rhs(p1, n1, 0.01 * (k + 1)) for k in range(50)]
    seq = {}
    with threadpool_limits(limits=1):
        for meth in ("zero", "last", "extrap", "proj"):
            t0 = time.perf_counter()
            r = run_sequence(op1, rhs1, meth, M, m, rtol=args.rtol)
            seq[meth] = {"wall_s": round(time.perf_counter() - t0, 3), "pcg_iters": int(sum(r["iters"]))}
    return {
        "value": allc,
        "unit": "GB/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{args.cpu_steps} steps (after {M} that fill the histories) of EXTRAP({m},{M}) + PROJ({M}) "
                  f"form+update on the benchmark's {args.modes}-mode plane-wave sequence at {n}^3, exact "
                  f"solutions; FP64 NumPy with {cores} BLAS threads, {all_s:.1f} s timed "
                  f"(setup {setup_s:.0f} s); projection history at d = {d_end} at the end",
        "one_thread": {"value": one, "unit": "GB/s", "cores": 1, "timed_s": round(one_s, 2)},
        "guess_rel_err_vs_oracle": vs_oracle,
        "small_sequence": {"workload": f"{n1}^3, 4 plane-wave modes, 50 steps, dt = 0.01, M = {M}, "
                                       f"EXTRAP({m},{M}) / PROJ({M}), guess -> PCG -> update, one thread",
                           "methods": seq},
    }


def _precision_vs_oracle(args, np, n, M, m, F, U, amps, sampled):
    """Guess error of the library against the FP64 oracle at the sampled steps of the
    cpu_baseline sequence (the same exact solutions and right-hand sides): one library context
    per history format and method is fed the whole sequence, and at each sampled step its guess
    x0 is compared with the oracle's FP64 guess g as max|x0 - g| / max|g| (EXTRAP(m, M) against
    the oracle's extrapolation, every projection form against its FP64 A-norm projection)."""
    import torch

    from paper_2009_10863_amd import libguess as L

    N = n ** 3
    dts = ["f64"] + [d.strip() for d in args.precision_dtypes.split(",") if d.strip() and d.strip() != "f64"]
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    ctx = {}
    try:
        for dt in dts:
            for name in ("extrap", "proj", "proj_raw"):
                if name == "proj_raw" and dt == "f64":
                    continue
                meth, _ = L.parse_method(name)
                ctx[dt, name] = L.guess_create_ex(N, M, meth, m if name == "extrap" else 0, L.DTYPES[dt],
                                                  args.eps_rel, A)
        bg = torch.empty(N, dtype=torch.float64, device="cuda")
        xg, x0 = torch.empty_like(bg), torch.empty_like(bg)
        err = {dt: {} for dt in dts}
        for step in range(1, max(sampled) + 1 if sampled else 0):
            a = amps(step)
            bg.copy_(torch.from_numpy(a @ F))
            xg.copy_(torch.from_numpy(a @ U))
            refs = None
            if step in sampled:
                refs = [torch.from_numpy(v).to("cuda") for v in sampled[step]]
            for (dt, name), g in ctx.items():
                if refs is not None:
                    L.guess_form(g, bg, x0)
                    ref = refs[0] if name == "extrap" else refs[1]
                    e = float((x0 - ref).abs().max() / ref.abs().max())
                    err[dt].setdefault(name, []).append(e)
                L.guess_update(g, xg)
        torch.cuda.synchronize()
    finally:
        for g in ctx.values():
            L.guess_destroy(g)
        L.guess_op_destroy(A)
    return {"steps": sorted(sampled), "reference": "oracle FP64 EXTRAP / PROJ (A-norm, classic) guesses",
            "dtypes": err}


def isolated(args, L):
    """Each guess kernel in isolation: median of `reps` launches at the benchmark grid, with a
    1 GiB scratch read between launches so that no operand is served from the 256 MB MALL.  The
    scratch is read, not written: a write would leave up to 256 MB of dirty lines whose write-back
    would then run inside the timed launch.
    Histories are random (well-conditioned); projection updates run at d = M - 1 (classic,
    rejected duplicates keep d) and at d = M (rolling drop)."""
    import torch

    n, M = args.n, args.M
    nz = args.shard_nz or n
    N = n * n * nz
    S = L.stream_handle()
    scratch = torch.ones(1 << 27, dtype=torch.float64, device="cuda")

    def evict():
        scratch.sum()
    A = L.guess_op_create(n, n, nz, float((n + 1) ** 2), 10.0, None)
    L.guess_op_set_stream(A, S)
    b = torch.randn(N, dtype=torch.float64, device="cuda")
    x0 = torch.empty_like(b)
    reps = args.reps
    out, us = {}, {}

    def med(v):
        return sorted(v)[len(v) // 2]

    for dt in ("f64", "f32", "f16", "bf16"):
        s = L.ELEM_BYTES[L.DTYPES[dt]]
        g = L.guess_create_ex(N, M, L.EXTRAP, args.degree, L.DTYPES[dt], 0.0, None, S)
        L.guess_profile(g, True)
        for _ in range(M):
            L.guess_update(g, torch.randn(N, dtype=torch.float64, device="cuda"))
        tf, tu = [], []
        for _ in range(reps):
            evict()
            L.guess_form(g, None, x0)
            tf.append(L.guess_kernel_times(g)[0])
            evict()
            L.guess_update(g, b)
            tu.append(sum(L.guess_kernel_times(g)))   # FP16: store + exponent check (same exponent: no re-store)
        out[f"extrap_form_{dt}"] = N * (M * s + 8) / (med(tf) * 1e-3) / 1e9
        out[f"ring_store_{dt}"] = N * (8 + s) / (med(tu) * 1e-3) / 1e9
        us[f"extrap_form_{dt}"] = med(tf) * 1e3
        us[f"ring_store_{dt}"] = med(tu) * 1e3
        L.guess_destroy(g)
    for meth in ("proj", "projqr"):
        for dt in ("f64", "f32"):
            s = L.ELEM_BYTES[L.DTYPES[dt]]
            g = L.guess_create_ex(N, M, L.METHODS[meth], 0, L.DTYPES[dt], 1e-6, A, S)
            L.guess_profile(g, True)
            keep = []
            for _ in range(M - 1 if meth == "proj" else M):
                keep.append(torch.randn(N, dtype=torch.float64, device="cuda"))
                L.guess_update(g, keep[-1])
            d = L.guess_get_info(g)["count"]
            tf, tu = [], []
            for _ in range(reps):
                evict()
                L.guess_form(g, b, x0)
                tf.append(L.guess_kernel_times(g))
                evict()
                L.guess_update(g, keep[-1] if meth == "proj" else torch.randn(N, dtype=torch.float64, device="cuda"))
                tu.append(L.guess_kernel_times(g))
            drop = meth == "projqr"
            fb = kernel_bytes(meth, "form", N, s, d, M, False)
            ub = kernel_bytes(meth, "update", N, s, d, M, False)
            for name, by, i in zip(KERNELS[(meth, "form")], fb, range(3)):
                if by:
                    out[f"{meth}_{name}_{dt}_d{d}"] = by / (med([t[i] for t in tf]) * 1e-3) / 1e9
                    us[f"{meth}_{name}_{dt}_d{d}"] = med([t[i] for t in tf]) * 1e3
            for name, by, i in zip(KERNELS[(meth, "update")], ub, range(6)):
                if by:
                    key = f"{meth}_{name}_{dt}_d{d}{'_drop' if drop else ''}"
                    out[key] = by / (med([t[i] for t in tu]) * 1e-3) / 1e9
                    us[key] = med([t[i] for t in tu]) * 1e3
            L.guess_destroy(g)
    # one Jacobi-PCG iteration at this shape (wall time of a fixed-count solve, host loop included)
    x = torch.zeros_like(b)
    L.pcg_solve(A, b, x, rtol=1e-300, maxit=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, its, _ = L.pcg_solve(A, b, x.zero_(), rtol=1e-300, maxit=100)
    torch.cuda.synchronize()
    us["pcg_iteration"] = (time.perf_counter() - t0) / max(its, 1) * 1e6
    L.guess_op_destroy(A)
    print(json.dumps({"isolated_GBps": {k: round(v, 1) for k, v in out.items()},
                      "isolated_us": {k: round(v, 2) for k, v in us.items()},
                      "grid": [n, n, nz], "M": M, "reps": reps,
                      **roofs(L), "peak_GBps": HBM_PEAK_GBS}), flush=True)


def small_sequence(args):
    """The whole small sequence (32^3, 4 plane waves, 50 steps, dt = 0.01) through the library,
    guess -> PCG -> update, per method: wall time and total PCG iterations (the oracle's run of the
    same sequence is cpu_baseline's small_sequence entry)."""
    import torch

    import synth
    from paper_2009_10863_amd.sequence import Operator, PlaneWaveRHS, run_sequence

    n1 = 32
    op1 = Operator(n1)
    rhs = PlaneWaveRHS(synth.plane_wave_params(0, 4), n1)
    res = {}
    try:
        for meth in ("zero", "last", "extrap", "proj"):
            run_sequence(op1, lambda k, out: rhs(0.01 * k, out), 5, meth, args.M, args.degree, rtol=args.rtol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = run_sequence(op1, lambda k, out: rhs(0.01 * k, out), 50, meth, args.M, args.degree,
                             rtol=args.rtol)
            torch.cuda.synchronize()
            res[meth] = {"wall_s": round(time.perf_counter() - t0, 4), "pcg_iters": int(sum(r["iters"]))}
    finally:
        op1.close()
    return {"workload": f"{n1}^3, 4 plane-wave modes, 50 steps, dt = 0.01, M = {args.M}, "
                        f"EXTRAP({args.degree},{args.M}) / PROJ({args.M}), guess -> PCG -> update",
            "methods": res}


def concurrent_run(args, L):
    """Independent sequences solved side by side.  Each field owns an operator, an EXTRAP context, its
    right-hand-side generator and a HIP stream; pcg_solve synchronises only its own stream, so one
    host thread per field keeps all four streams busy at once.  The same steps are first run field
    after field on one thread; iteration counts must agree between the two runs."""
    import threading

    import numpy as np
    import torch

    import synth
    from paper_2009_10863_amd.sequence import GuessSequence, Operator, PlaneWaveRHS

    n, T, W = args.n, args.steps, args.warmup
    N = n ** 3
    specs = [(f"vel{c}", args.velocity_shift, args.seed + 1 + c) for c in range(3)] + [("p", 0.0, args.seed + 4)]

    def make():
        fs = []
        for name, shift, seed in specs:
            st = torch.cuda.Stream()
            op = Operator(n, shift, None, st)
            fs.append({"name": name, "stream": st, "op": op,
                       "rhs": PlaneWaveRHS(synth.plane_wave_params(seed, args.modes), n, st),
                       "g": GuessSequence(N, args.M, "extrap", args.degree, "f64", 0.0, op, st),
                       "b": torch.empty(N, dtype=torch.float64, device="cuda"),
                       "x": torch.zeros(N, dtype=torch.float64, device="cuda"), "iters": []})
        torch.cuda.synchronize()
        return fs

    def steps(f, first, count):
        for step in range(first, first + count):
            f["rhs"](step * args.dt, f["b"])
            f["g"].form(f["b"], f["x"])
            stt, it, _ = f["op"].solve(f["b"], f["x"], args.rtol, args.maxit)
            if stt != L.OK:
                raise RuntimeError(f"PCG failed for field {f['name']} at step {step}: status {stt}")
            f["g"].update(f["x"])
            f["iters"].append(it)
        torch.cuda.synchronize(f["stream"])

    def close(fs):
        for f in fs:
            f["g"].close()
            f["op"].close()

    out = {}
    for mode in ("one_thread", "thread_per_field"):
        fs = make()
        try:
            for f in fs:
                steps(f, 1, W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "one_thread":
                for step in range(W + 1, W + T + 1):
                    for f in fs:
                        steps(f, step, 1)
            else:
                errs = []

                def work(f):
                    try:
                        steps(f, W + 1, T)
                    except Exception as e:  # noqa: BLE001
                        errs.append(e)
                th = [threading.Thread(target=work, args=(f,)) for f in fs]
                for t in th:
                    t.start()
                for t in th:
                    t.join()
                if errs:
                    raise errs[0]
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            out[mode] = {"ms_per_step": 1e3 * wall / T,
                         "pcg_iters_per_step": {f["name"]: float(np.mean(f["iters"][W:])) for f in fs},
                         "iters": {f["name"]: f["iters"] for f in fs}}
        finally:
            close(fs)
    same = out["one_thread"]["iters"] == out["thread_per_field"]["iters"]
    for v in out.values():
        del v["iters"]
    print(json.dumps({"mode": "concurrent", "workload": f"{n}^3: three velocity components (shift "
                                                       f"{args.velocity_shift}) and a pressure, {args.modes} "
                                                       f"plane-wave modes each, EXTRAP({args.degree},{args.M}), "
                                                       f"{T} timed steps after {W}",
                      "runs": out, "same_iterations": same,
                      "speedup": out["one_thread"]["ms_per_step"] / out["thread_per_field"]["ms_per_step"]}),
          flush=True)


def adjoint_run(args, L):
    """Differentiable sequence (loss sum_n ||x_n - y_n||^2, gradient with respect to the mode
    amplitudes c): forward solves, then the reverse-time adjoint solves, each sequence with its own
    guess history; the same with zero guesses for comparison.  Reports ms and PCG iterations per
    step for both directions and how far the two gradients differ (both solve to rtol)."""
    import numpy as np
    import torch

    import synth
    from paper_2009_10863_amd.autograd import GuessSolveFn, SolveSequence, plane_wave_modes
    from paper_2009_10863_amd.sequence import Operator

    n, T, K = args.adjoint_n, args.adjoint_steps, args.modes
    N = n ** 3
    S = L.stream_handle()
    params = synth.plane_wave_params(args.seed, K)
    tp = synth.target_params(args.seed + 99)
    ts = synth.step_times(T, args.dt)
    amps = np.stack([synth.mode_amplitudes(params, t) for t in ts])
    F = plane_wave_modes(params, n)
    Y = torch.empty((T, N), dtype=torch.float64, device="cuda")
    kv = [int(v) for v in tp["k"].reshape(-1)]
    for i, t in enumerate(ts):   # y(t) = scale sum_j sin(w_j t + phi_j) cos(2 pi k_j.x + theta_j)
        L.workload_plane_wave_rhs(n, kv, tp["theta"], tp["scale"] * np.sin(tp["w"] * t + tp["phi"]), Y[i], S)
    op = Operator(n)
    out = {}
    try:
        for method in ("extrap", "zero"):
            seq = SolveSequence(op, F, amps, method=method, M=args.M, degree=args.degree, rtol=args.rtol)
            c = torch.ones(K, dtype=torch.float64, requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X = GuessSolveFn.apply(c, seq)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss = ((X - Y) ** 2).sum()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            out[method] = {"forward_ms_per_step": 1e3 * (t1 - t0) / T, "adjoint_ms_per_step": 1e3 * (t2 - t1) / T,
                           "forward_iters_per_step": float(np.mean(seq.stats["forward_iters"])),
                           "adjoint_iters_per_step": float(np.mean(seq.stats["adjoint_iters"])),
                           "loss": float(loss.detach()), "grad": c.grad.tolist()}
            del X, loss
        ge, gz = np.array(out["extrap"]["grad"]), np.array(out["zero"]["grad"])
        rel = float(np.max(np.abs(ge - gz)) / np.max(np.abs(gz)))
    finally:
        op.close()
    print(json.dumps({"mode": "adjoint", "workload": f"{n}^3 Helmholtz, {K} plane-wave modes, {T} steps, dt={args.dt}, "
                                                    f"EXTRAP({args.degree},{args.M}) both directions vs zero guess, "
                                                    f"PCG rtol {args.rtol}",
                      "methods": out, "grad_rel_diff_extrap_vs_zero": rel}), flush=True)


def main():
    args = parse()
    if args.traffic_summary:
        traffic_summary(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout "
              "is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2009_10863_amd import libguess as L
    from paper_2009_10863_amd.sequence import Operator, PlaneWaveRHS

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        gbps = copy_roof(L, 1 << 30, 5)
        print(json.dumps({"copy_kernel_GBps": gbps, "bytes_read_per_launch": 1 << 30,
                          "bytes_written_per_launch": 1 << 30}), flush=True)
        return
    if args.isolated:
        isolated(args, L)
        return
    if args.adjoint:
        adjoint_run(args, L)
        return
    if args.concurrent:
        concurrent_run(args, L)
        return
    rf = roofs(L)
    roof = rf["copy_roof_GBps"]
    n, N, M = args.n, args.n ** 3, args.M
    methods = [m.strip() for m in args.methods.split(",") if m.strip()]
    kappa = None
    if args.workload == "varcoef":
        kappa = torch.from_numpy(np.exp(synth.gaussian_field(args.seed + 5, n))).cuda()
    op = Operator(n, 10.0, kappa)
    del kappa
    faces = 8 * 3 * (n + 1) * n * n if args.workload == "varcoef" else 0
    params = synth.plane_wave_params(args.seed, args.modes)
    if args.rhs == "planewave":
        rhs = PlaneWaveRHS(params, n)
    else:
        gp = synth.gaussian_source_params(args.seed)

        def rhs(t, out):
            L.workload_gaussian_rhs(n, synth.gaussian_center(gp, t), gp["sigma"], gp["amp"], out,
                                    L.stream_handle())
    # fields solved every step: one (the default), or the paper's incompressible-flow
    # pattern of three velocity components (Helmholtz, shift 1/(nu dt)) and a pressure
    # (Poisson), each with its own right-hand sides and its own guess contexts
    fields = [("u", op, rhs)]
    if args.fields == "ins":
        op_v = Operator(n, args.velocity_shift)
        op_p = Operator(n, 0.0)
        fields = [(f"vel{c}", op_v, PlaneWaveRHS(synth.plane_wave_params(args.seed + 1 + c, args.modes), n))
                  for c in range(3)]
        fields.append(("p", op_p, PlaneWaveRHS(synth.plane_wave_params(args.seed + 4, args.modes), n)))
    bufs = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in fields]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def run(dtype, steps, warmup, shadow=False, methods=methods):
        """Time `steps` steps after `warmup` untimed ones; with `shadow`, an FP64
        context per method is fed the same solutions, and the guess error of the
        reduced-precision history against it is recorded (the raw-solution projection,
        which takes reduced-precision histories only, against the FP64 Gram-Schmidt form
        with the same window rule)."""
        s = L.ELEM_BYTES[L.DTYPES[dtype]]
        ctx, xs, sh, x64 = {}, {}, {}, None
        for fi, (_, fop, _) in enumerate(fields):
            for m in methods:
                meth, inner = L.parse_method(m)
                ctx[fi, m] = L.guess_create_ex(N, 1 if m == "last" else M, meth,
                                               args.degree if m in ("extrap", "spextrap") else 0, L.DTYPES[dtype],
                                               args.eps_rel, fop.handle, L.stream_handle(), inner)
                L.guess_profile(ctx[fi, m], True)
                xs[fi, m] = torch.zeros(N, dtype=torch.float64, device="cuda")
                if shadow:
                    if m in RAW:
                        meth = L.PROJ_QR if m == "projqr_raw" else L.PROJ
                    sh[fi, m] = L.guess_create_ex(N, 1 if m == "last" else M, meth,
                                                  args.degree if m in ("extrap", "spextrap") else 0, L.F64,
                                                  args.eps_rel, fop.handle, L.stream_handle(), inner)
        if shadow:
            x64 = torch.empty(N, dtype=torch.float64, device="cuda")
        stats = {m: {"iters": [], "guess_ms": 0.0, "guess_bytes": 0.0, "solve_ms": 0.0, "relres": [],
                     "err": [], "field_iters": {f[0]: [] for f in fields}} for m in methods}
        kstat = {}    # kernel -> [launches, ms, bytes]

        def one_step(step, timed):
            t = step * args.dt
            for fi, (fname, fop, frhs) in enumerate(fields):
                b = bufs[fi]
                frhs(t, b)
                for m in methods:
                    field_step(step, timed, fi, fname, fop, b, m)

        def field_step(step, timed, fi, fname, op, b, m):
            g, x = ctx[fi, m], xs[fi, m]
            inf0 = L.guess_get_info(g)
            kd = inf0["count"]
            if m == "spextrap":
                kd_form = min(args.degree, kd - 1) + 1 if kd > 0 else 0    # slots read
            else:
                kd_form = kd if m.startswith("proj") else min(kd, M)
            L.guess_form(g, b, x)
            tf = L.guess_kernel_times(g)
            if shadow and timed:
                L.guess_form(sh[fi, m], b, x64)
                nrm = float(torch.linalg.vector_norm(x64))
                stats[m]["err"].append(float(torch.linalg.vector_norm(x - x64)) / nrm if nrm > 0 else 0.0)
            ev[0].record()
            st, it, rr = op.solve(b, x, args.rtol, args.maxit,
                                  L.STOP_RHS if args.stop_rule == "rhs" else L.STOP_INITRESID)
            ev[1].record()
            inf1 = L.guess_get_info(g)
            L.guess_update(g, x)
            tu = L.guess_kernel_times(g)
            fixed = False
            if dtype == "f16" and (m in RING or m in RAW) and timed:
                plain = sum(kernel_bytes(m, "update", N, s, inf1["count"], M, False, faces, dtype, False))
                fixed = L.guess_get_info(g)["update_bytes"] > plain + 0.5 * N * (8 + s)
            if shadow:
                L.guess_update(sh[fi, m], x)
            if st != L.OK:
                raise RuntimeError(f"PCG failed for {m} ({dtype}, field {fname}) at step {step}: status {st}")
            if not timed:
                return
            torch.cuda.synchronize()
            S = stats[m]
            S["iters"].append(it)
            S["field_iters"][fname].append(it)
            S["relres"].append(rr)
            S["solve_ms"] += ev[0].elapsed_time(ev[1])
            dd = inf1["count"]
            if m.startswith("projqr"):
                restart = dd == 0 or M == 1
            else:
                restart = m.startswith("proj") and (dd == 0 or dd >= M)
            for call, times, kdd in (("form", tf, kd_form), ("update", tu, inf1["count"])):
                names = kernel_names(m, call, dtype)
                rws = kernel_rw(m, call, N, s, kdd, M, restart, faces, dtype, fixed)
                for name, ms, (rb, wb) in zip(names, times, rws):
                    # every kernel of the call counts in the guess time; the
                    # per-kernel table keeps the streaming kernels that moved data
                    by = rb + wb
                    S["guess_ms"] += ms
                    S["guess_bytes"] += by
                    if by == 0:
                        continue
                    key = name if m in ("extrap", "proj") else f"{name}:{m}"
                    ks = kstat.setdefault(key, [0, 0.0, 0.0, 0.0, 0.0])
                    ks[0] += 1
                    ks[1] += ms
                    ks[2] += by
                    ks[3] += rb
                    ks[4] += wb

        try:
            for step in range(1, warmup + 1):
                one_step(step, False)
                if args.progress:
                    print(f"[bench] {dtype} warm-up step {step} done", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for step in range(warmup + 1, warmup + steps + 1):
                one_step(step, True)
                if args.progress:
                    print(f"[bench] {dtype} timed step {step} done", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            for m in methods:
                inf = L.guess_get_info(ctx[0, m])
                stats[m]["history"] = {k: inf[k] for k in ("count", "restarts", "drops", "rejects", "eps_rel")}
        finally:
            torch.cuda.synchronize()
            for g in list(ctx.values()) + list(sh.values()):
                L.guess_destroy(g)
        return stats, kstat, wall

    stats, kstat, wall = run(args.dtype, args.steps, args.warmup)
    s = L.ELEM_BYTES[L.DTYPES[args.dtype]]
    tot_bytes = sum(S["guess_bytes"] for S in stats.values())
    tot_ms = sum(S["guess_ms"] for S in stats.values())
    value = tot_bytes / (tot_ms * 1e-3) / 1e9
    dom = max(kstat.items(), key=lambda kv: kv[1][1])
    dname, (dl, dms, dby, drb, dwb) = dom
    achieved = (dby / dl) / (dms / dl * 1e-3) / 1e9
    per_method = {}
    for m, S in stats.items():
        per_method[m] = {
            "guess_GBps": S["guess_bytes"] / (S["guess_ms"] * 1e-3) / 1e9 if S["guess_ms"] else None,
            "guess_ms_per_step": S["guess_ms"] / args.steps,
            "pcg_iters_per_step": float(np.mean(S["iters"])),
            "pcg_ms_per_step": S["solve_ms"] / args.steps,
            # wall time of the solves (initial residual, iterations, host loop) per iteration
            "pcg_us_per_iteration": S["solve_ms"] * 1e3 / max(1.0, float(np.sum(S["iters"]))),
            "max_relres": float(np.max(S["relres"])),
            "history_after_run": S["history"],
        }
        if len(fields) > 1:
            per_method[m]["pcg_iters_per_step_by_field"] = {f: float(np.mean(v)) for f, v in S["field_iters"].items()}
    R, W = rf["read_roof_GBps"], rf["write_roof_GBps"]
    kernels = {}
    for k, v in sorted(kstat.items()):
        gbps = v[2] / (v[1] * 1e-3) / 1e9
        mr = mixed_roof(v[3], v[4], R, W)
        kernels[k] = {"launches": v[0], "avg_us": 1e3 * v[1] / v[0], "GBps": gbps, "bytes_per_launch": v[2] / v[0],
                      "read_fraction": v[3] / v[2], "mixed_roof_GBps": mr, "frac_of_mixed_roof": gbps / mr}
    # counter bytes of the profiled launches, scaled to this run's launches of the same kernel
    # (their mix of history sizes d differs with the number of steps)
    tr = hbm_traffic(dname)
    traffic_ratio = tr[0] / tr[1] if tr else None
    traffic = traffic_ratio * (dby / dl) if tr else None
    out = {
        "metric": "guess form+update HBM GB/s (256^3, M=8); PCG iters & ms/step vs FP64 plain",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{'helmholtz7' if args.workload == 'helmholtz' else 'varcoef7 kappa=exp(GRF l=0.1)'} "
                               f"{n}^3 ({N} unknowns), "
                               f"{str(args.modes) + ' plane-wave modes' if args.rhs == 'planewave' else 'moving Gaussian source'}"
                               f", dt={args.dt}, "
                               f"M={M}, EXTRAP({args.degree},{M}) + PROJ({M}), {args.dtype} history, PCG rtol {args.rtol}",
                   "n": n, "N": N, "M": M, "degree": args.degree, "methods": methods,
                   "history_dtype": args.dtype,
                   "eps_rel": next(iter(per_method.values()))["history_after_run"]["eps_rel"], "rtol": args.rtol,
                   "stop_rule": args.stop_rule, "rhs": args.rhs, "fields": [f[0] for f in fields],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_ratio": traffic_ratio,
                     "bytes_per_launch": dby / dl, "avg_us": 1e3 * dms / dl,
                     "copy_roof_GBps": roof, "frac_of_copy_roof": achieved / roof,
                     "read_roof_GBps": R, "read_roof_one_stream_GBps": rf["read_roof_one_stream_GBps"],
                     "read_roof_16_streams_GBps": rf["read_roof_16_streams_GBps"], "write_roof_GBps": W,
                     "mixed_roof_GBps": mixed_roof(drb, dwb, R, W),
                     "frac_of_mixed_roof": achieved / mixed_roof(drb, dwb, R, W)},
        "guess_mixed_roof_GBps": mixed_roof(sum(v[3] for v in kstat.values()), sum(v[4] for v in kstat.values()), R, W),
        "methods": per_method,
        "kernels": kernels,
    }
    if args.precision_steps > 0 and args.dtype == "f64":
        prec = {}
        for dt in [d.strip() for d in args.precision_dtypes.split(",") if d.strip()]:
            try:
                pm = [m.strip() for m in args.precision_methods.split(",") if m.strip()]
                st_, ks_, wall_ = run(dt, args.precision_steps, args.warmup, shadow=True, methods=pm)
            except RuntimeError as e:
                # a reduced-precision history can produce a guess PCG cannot start from
                # (e.g. FP16 overflow); that is a result of this sweep, not a bench failure
                prec[dt] = {"error": str(e)}
                continue
            gb = sum(S["guess_bytes"] for S in st_.values())
            gm = sum(S["guess_ms"] for S in st_.values())
            prec[dt] = {
                "guess_GBps": gb / (gm * 1e-3) / 1e9,
                "ms_per_step_incl_shadow": wall_ * 1e3 / args.precision_steps,
                "methods": {m: {"pcg_iters_per_step": float(np.mean(S["iters"])),
                                "pcg_ms_per_step": S["solve_ms"] / args.precision_steps,
                                "guess_ms_per_step": S["guess_ms"] / args.precision_steps,
                                "guess_rel_err_vs_f64_mean": float(np.mean(S["err"])),
                                "guess_rel_err_vs_f64_max": float(np.max(S["err"])),
                                "max_relres": float(np.max(S["relres"])),
                                "eps_rel": S["history"]["eps_rel"]} for m, S in st_.items()},
            }
        out["precision"] = {"steps": args.precision_steps, "warmup": args.warmup,
                            "reference": "FP64 history fed the same solutions", "dtypes": prec}
    if args.small:
        out["small_sequence"] = small_sequence(args)
    if args.cpu:
        out["cpu_baseline"] = cpu_baseline(args, s)
    op.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
