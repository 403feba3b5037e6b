"""Benchmark: evaluation of F and the full Jacobian of sparse polynomial
systems at complex points, by the reverse mode on each monomial.

Default workload (the largest single-GPU one): 4096 uneven complex
double-double systems, n = N = m drawn uniformly from {32, 64, 128, 256}, every
monomial the product of k = min(16, n/4) distinct variables (uniform without
replacement) with exponents uniform in {1, 2, 3}, unit-circle coefficients and
points (seeded, synthetic), each system evaluated at 8 points.  One step is
one pe_batch_eval call (the persistent launches over every system-point);
inputs are resident in HBM.  Beside it the plain path, one pe_eval launch per
system-point, is timed on the same GPU.

Prints one JSON line: monomial evaluations (value and all partials, summed
into F and J) per second, the roofline of the evaluation kernels by the
method's operation count, and the CPU oracle timed on a bounded sample.
Other workloads (--workload) print the same kind of line for context.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "dd_batch4096"
METRIC = "monomial eval+grad/s and F+J per s (complex D/DD/QD); % of FP64 or HBM roofline"
LEVEL_NAME = {1: "double", 2: "double-double", 4: "quad-double"}
PEAK_FP64_TFLOPS = 78.6  # 256 CUs x 64 FP64 FMA lanes/clk x 2 flops x 2.4 GHz
PEAK_HBM_GBS = 8000.0    # HBM3E
# the machine's CPU share for one GPU: worker pools never exceed it, whatever the
# host's core count
CPU_SHARE = 16

BATCH_COUNT, BATCH_POINTS = 4096, 8

# rocprofv3 counter summaries per workload: HBM bytes (FETCH_SIZE, WRITE_SIZE
# per dispatch, scaled by what the same counters read for a plain device copy
# of known size) and FP64 instruction counts.  They hold for the kernel
# sources they were taken with: the bench reports them only while the
# sources match.  Every counted workload is an evaluation, so the digest
# covers the evaluation kernels' sources, their arithmetic, packing, planning
# and launchers (the least-squares and Gauss-Newton kernels are not among
# them).
COUNTERS_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["eval_kernels.hpp", "mdarith.hpp", "layout.hpp", "polyeval.hip", "packer.cpp", "packer.hpp",
                  "launch.hpp", "instances.hip"]


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1402_2626_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_counters(workload: str):
    """The counter summary of a workload if it matches the current sources."""
    try:
        with open(os.path.join(COUNTERS_DIR, f"counters_{workload}.json")) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("workload") != workload or c.get("source_sha256") != kernel_source_digest():
        return None
    return c


def counter_traffic(c):
    """HBM bytes per step: FETCH and WRITE of the step's kernels, scaled."""
    if not c:
        return None
    return sum((k["fetch_kib_per_dispatch"] * c["fetch_scale"] + k["write_kib_per_dispatch"] * c["write_scale"])
               * 1024.0 * k.get("dispatches_per_step", 1) for k in c["kernels"])


def fp64_issue_fraction(c, step_ms):
    """FP64 VALU instructions per step over what the SIMDs can issue in the
    step's time: a wave64 FP64 instruction occupies a SIMD for 4 cycles, 4
    SIMDs per CU, 256 CUs, 2.4 GHz.  None without counters."""
    if not c or "fp64_wave_insts_per_step" not in c:
        return None
    slots = step_ms * 1e-3 * 2.4e9 * 256 * 4 / 4.0
    return c["fp64_wave_insts_per_step"] / slots


def host_cpu():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def run_oracle_jobs(fn, jobs):
    """Run oracle jobs on min(CPU share, cores) spawned workers; returns
    (results, wall seconds, workers)."""
    import multiprocessing as mp
    workers = max(1, min(CPU_SHARE, os.cpu_count() or 1, len(jobs)))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(fn, jobs)
    return res, time.perf_counter() - t0, workers


def _oracle_rows(args):
    import oracle as O
    sys_, x, rows = args
    O.eval_rows(sys_, x, rows, want_J=True)
    return int(sum(int(sys_.poly_ptr[p + 1] - sys_.poly_ptr[p]) for p in rows))


def cpu_baseline_rows(sys_, x, rows):
    """The exact oracle on the given rows (F and full rows of J) at point x."""
    model, ncpu = host_cpu()
    rows = list(rows)
    per = max(1, (len(rows) + CPU_SHARE - 1) // CPU_SHARE)
    jobs = [(sys_, x, rows[a:a + per]) for a in range(0, len(rows), per)]
    res, dt, workers = run_oracle_jobs(_oracle_rows, jobs)
    return {"value": sum(res) / dt, "unit": "monomials/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(rows)} of {sys_.n_polys} polynomials (F and full J rows, exact arithmetic) at one "
                      f"point, {dt:.1f} s wall", "cpu_model": model, "host_cpus": ncpu}


def _time_steps(fn, K, W, stream):
    """W untimed calls, then K timed calls enqueued back to back.  Returns the
    wall time of the K calls (synchronised on both sides) and the average
    per-call time from HIP events recorded on `stream` around them."""
    import torch
    for _ in range(W):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(K):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, e0.elapsed_time(e1) / K


def line(workload_desc, level, value, K, W, dt, extra_config, roofline, cpu):
    return {"metric": METRIC, "value": value, "unit": "monomials/s", "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64 (%s complex)" % LEVEL_NAME[level], "data": "synthetic",
            "config": dict({"workload": workload_desc}, **extra_config), "roofline": roofline, "cpu_baseline": cpu}


def alu_roofline(flops, ms, counters=None):
    achieved = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": counter_traffic(counters)}


# ------------------------------------------------------------------ the batch

def _oracle_batch(args):
    import oracle as O
    from paper_1402_2626_amd import synth
    i, n, rows = args
    sys_ = synth.batch_system(0, i, n)
    x = synth.unit_circle_points(synth.rng_for((0, 9, i)), 1, n, 2)[0]
    O.eval_rows(sys_, x, rows, want_J=True)
    return int(sum(int(sys_.poly_ptr[p + 1] - sys_.poly_ptr[p]) for p in rows))


def batch_cpu_baseline(ns):
    """The oracle on 64 systems of the batch, 16 of each size, every fourth
    row of each (and the last) at one point: about 10 s on 16 host threads."""
    model, ncpu = host_cpu()
    jobs = []
    for n in (32, 64, 128, 256):
        idx = [i for i in range(len(ns)) if int(ns[i]) == n][:16]
        jobs += [(i, n, sorted(set(range(0, n, 4)) | {n - 1})) for i in idx]
    res, dt, workers = run_oracle_jobs(_oracle_batch, jobs)
    return {"value": sum(res) / dt, "unit": "monomials/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(jobs)} systems of the batch (16 per size n), every fourth row and the last of each "
                      f"(F and full J rows, exact arithmetic) at one point, {dt:.1f} s wall", "cpu_model": model,
            "host_cpus": ncpu}


def bench_batch(args):
    """4096 uneven DD systems at 8 points each in persistent launches, beside
    the plain path (one pe_eval launch per system-point)."""
    import numpy as np
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    S_count, P = BATCH_COUNT, BATCH_POINTS
    ns = synth.batch_sizes(0, S_count)
    cpu = None if args.no_cpu else batch_cpu_baseline(ns)
    t0 = time.perf_counter()
    dev, flops, flops_exec, mons, occ = [], 0.0, 0.0, 0, 0
    for i in range(S_count):
        sy = synth.batch_system(0, i, int(ns[i]))
        dev.append(pe.System.from_sparse(sy))
        flops += W.flops_per_point(sy) * P
        flops_exec += W.executed_flops_per_point(sy) * P
        mons += sy.n_monomials * P
        occ += sy.nnz * P
        del sy
        if i % 512 == 511:
            print(f"# loaded {i + 1} systems, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    B = pe.Batch(dev)
    rng = synth.rng_for((0, 9))
    x = torch.from_numpy(np.concatenate([synth.unit_circle_points(rng, P, int(n), 2).reshape(-1)
                                         for n in ns])).cuda()
    F = torch.empty(int(B.F_off[-1]) * P, dtype=torch.float64, device="cuda")
    J = torch.empty(int(B.J_off[-1]) * P, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    K = max(1, args.steps)
    Wm = max(1, args.warmup)
    print("# timing the batch", file=sys.stderr, flush=True)
    dt, ms = _time_steps(lambda: B.eval(x, P, out=(F, J), stream=st), K, Wm, st)

    # plain path: one pe_eval launch per system-point (and, for context, one
    # per system at its 8 points), into the same outputs; the launch
    # arguments are computed beforehand so the loop is the C calls only
    import ctypes
    lib, sp = pe._lib, ctypes.c_void_p(st.cuda_stream)
    xb, fb, jb = x.data_ptr(), F.data_ptr(), J.data_ptr()
    per_point, per_system = [], []
    for i in range(S_count):
        n = int(ns[i])
        xo, fo, jo = int(B.x_off[i]) * P, int(B.F_off[i]) * P, int(B.J_off[i]) * P
        h = dev[i].handle
        per_system.append((h, P, xb + 8 * xo, fb + 8 * fo, jb + 8 * jo))
        for p in range(P):
            per_point.append((h, 1, xb + 8 * (xo + p * 4 * n), fb + 8 * (fo + p * 4 * n),
                              jb + 8 * (jo + p * 4 * n * n)))

    def plain_points():
        for h, npts, xp, fp, jp in per_point:
            lib.pe_eval(h, npts, xp, fp, jp, sp)

    def plain_systems():
        for h, npts, xp, fp, jp in per_system:
            lib.pe_eval(h, npts, xp, fp, jp, sp)
    print("# timing the plain path", file=sys.stderr, flush=True)
    dt_pts, ms_pts = _time_steps(plain_points, 1, 1, st)
    dt_sys, ms_sys = _time_steps(plain_systems, 1, 1, st)
    info = B.info()
    counters = load_counters("dd_batch4096")
    out = line("batched complex double-double: 4096 systems, n = N = m uniform in {32, 64, 128, 256}, "
               "k = min(16, n/4), exponents {1, 2, 3}, 8 points each", 2, mons * K / dt, K, Wm, dt,
               {"system_points_per_s": S_count * P * K / dt, "F_plus_J_per_s": S_count * P * K / dt,
                "monomials": mons, "occurrences": occ, "kernel_ms": ms,
                "plain_per_system_point_ms": ms_pts, "plain_per_system_point_launches": S_count * P,
                "speedup_vs_plain_per_system_point": ms_pts / ms,
                "plain_per_system_ms": ms_sys, "speedup_vs_plain_per_system": ms_sys / ms,
                "segment": info["segment"], "chunks_per_workgroup": info["chunks_per_workgroup"],
                "flops_method_count": flops, "frac_executed_count": flops_exec / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                "fp64_issue_frac": fp64_issue_fraction(counters, ms)},
               alu_roofline(flops, ms, counters), cpu)
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ single systems

def bench_single(args):
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    sys_, x = synth.workload(args.workload)
    P = x.shape[0]
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_rows(sys_, x[0], range(min(args.cpu_rows, sys_.n_polys)))
    S = pe.System.from_sparse(sys_)
    xd = torch.from_numpy(x).cuda()
    st = torch.cuda.current_stream()
    if args.shapes:
        for seg in (2, 4, 6, 8, 16):
            for G in (1, 2, 4):
                try:
                    S.set_shape(G, segment=seg)
                except pe.PolyevalError:
                    continue
                dt, ms = _time_steps(lambda: S.eval(xd, stream=st), args.steps, args.warmup, st)
                print(json.dumps({"workload": args.workload, "segment": seg, "chunks_per_workgroup": G,
                                  "kernel_ms": ms, "step_ms": dt / args.steps * 1e3,
                                  "lds_bytes": S.info()["lds_bytes"]}), flush=True)
        return
    if args.autotune:
        S.autotune(P)
    F = torch.empty((P, 2, sys_.level, sys_.n_polys), dtype=torch.float64, device="cuda")
    J = torch.empty((P, 2, sys_.level, sys_.n_polys, sys_.n_vars), dtype=torch.float64, device="cuda")
    K = args.steps
    dt, ms = _time_steps(lambda: S.eval(xd, out=(F, J), stream=st), K, args.warmup, st)
    counters = load_counters(args.workload)
    flops = W.flops_per_point(sys_) * P
    w = synth.WORKLOADS[args.workload]
    desc = (f"complex {LEVEL_NAME[sys_.level]}: n = {w['n']}, N = {w['N']}, {w['m']} monomials per polynomial, "
            f"k = {w['k']}, exponents 1..{w['exp_hi']}, {P} point(s)")
    info = S.info()
    out = line(desc, sys_.level, sys_.n_monomials * P * K / dt, K, args.warmup, dt,
               {"name": args.workload, "points": P, "monomials": sys_.n_monomials, "occurrences": sys_.nnz,
                "F_plus_J_per_s": P * K / dt, "kernel_ms": ms, "segment": info["segment"],
                "chunks_per_workgroup": info["chunks_per_workgroup"],
                "frac_executed_count": W.executed_flops_per_point(sys_) * P / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                "fp64_issue_frac": fp64_issue_fraction(counters, ms)},
               alu_roofline(flops, ms, counters), cpu)
    S.close()
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """g = J^H v for the overdetermined DD system (N = 1024, n = 512, k = 24)
    at 64 points; J is never formed."""
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    sys_, x = synth.workload("dd_adjoint_1024x512")
    v = synth.adjoint_vectors(0, x.shape[0], sys_.n_polys, sys_.level)
    P = x.shape[0]
    S = pe.System.from_sparse(sys_)
    xd, vd = torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda()
    g = torch.empty_like(xd)
    st = torch.cuda.current_stream()
    dt, ms = _time_steps(lambda: S.adjoint(xd, vd, out=g, stream=st), args.steps, args.warmup, st)
    flops = W.flops_per_point(sys_) * P
    counters = load_counters("dd_adjoint_1024x512")
    out = line("adjoint J^H v, complex double-double: N = 1024 polynomials in n = 512 variables, 512 monomials "
               "each, k = 24, exponents 1..3, 64 points", 2, sys_.n_monomials * P * args.steps / dt, args.steps,
               args.warmup, dt, {"points": P, "kernel_ms": ms, "fp64_issue_frac": fp64_issue_fraction(counters, ms)},
               alu_roofline(flops, ms, counters), None)
    S.close()
    print(json.dumps(out), flush=True)


# cyclic n-roots (eq. (5)); the paper's Table 5 times on its GPU are context
CYCLIC = {"cyclic_d_n512": (1, 512, 46.43), "cyclic_dd_n512": (2, 512, 267.39)}


def bench_cyclic(args):
    """F and J of the cyclic n-roots system at one point on the unit circle."""
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    L, n, paper_ms = CYCLIC[args.workload]
    sys_ = synth.cyclic_roots_system(n, L)
    x = synth.unit_circle_points(synth.rng_for((0, 1)), 1, n, L)
    S = pe.System.from_sparse(sys_)
    xd = torch.from_numpy(x).cuda()
    F = torch.empty((1, 2, L, n), dtype=torch.float64, device="cuda")
    J = torch.empty((1, 2, L, n, n), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    K = min(args.steps, 50)
    Wm = min(args.warmup, 5)
    dt, ms = _time_steps(lambda: S.eval(xd, out=(F, J), stream=st), K, Wm, st)
    flops = W.flops_per_point(sys_)
    nbytes = W.bytes_per_point(sys_, want_J=True)
    counters = load_counters(args.workload)
    cfg = {"name": args.workload, "kernel_ms": ms, "segment": S.info()["segment"], "monomials": sys_.n_monomials,
           "paper_table5_ms_context": paper_ms, "hbm_frac_algorithmic_bytes": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "fp64_issue_frac": fp64_issue_fraction(counters, ms)}
    out = line(f"cyclic {n}-roots (eq. (5)), complex {LEVEL_NAME[L]}, F and J at one unit-circle point", L,
               sys_.n_monomials * K / dt, K, Wm, dt, cfg, alu_roofline(flops, ms, counters), None)
    S.close()
    print(json.dumps(out), flush=True)


def bench_product(args):
    """The Table-1 shape in complex double: 65,024 one-monomial polynomials,
    each the product of all 1,024 variables; F and the dense 65,024 x 1,024 J
    at one point.  Bound by HBM (the J write dominates)."""
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    sys_, x = synth.product_workload()
    S = pe.System.from_sparse(sys_)
    xd = torch.from_numpy(x).cuda()
    F = torch.empty((1, 2, 1, sys_.n_polys), dtype=torch.float64, device="cuda")
    J = torch.empty((1, 2, 1, sys_.n_polys, sys_.n_vars), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    K = min(args.steps, 50)
    Wm = min(args.warmup, 5)
    dt, ms = _time_steps(lambda: S.eval(xd, out=(F, J), stream=st), K, Wm, st)
    nbytes = W.bytes_per_point(sys_, want_J=True, chunks=sys_.n_polys)
    gbs = nbytes / (ms * 1e-3) / 1e9
    counters = load_counters("d_product_65024x1024")
    out = line("products of variables (the shape of the paper's Table 1), complex double: 65,024 polynomials, "
               "each one monomial of all n = 1,024 variables (exponent 1), 1 point; dense J of 1.07 GB", 1,
               sys_.n_monomials * K / dt, K, Wm, dt,
               {"name": "d_product_65024x1024", "kernel_ms": ms, "algorithmic_bytes": nbytes,
                "flops": W.flops_per_point(sys_)},
               {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                "traffic": counter_traffic(counters)}, None)
    S.close()
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ Newton steps

def bench_newton_single(args):
    """One Gauss-Newton step (evaluation of [J | -F], least-squares solve by
    modified Gram-Schmidt, update) of the 256 x 256 double-double system
    with a planted root, from the perturbed start: the step's time, beside
    the evaluation alone."""
    import torch
    import oracle as O
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth

    sys_, x = synth.workload("dd_n256")
    planted = O.plant_root(sys_, x[0])
    x0 = synth.perturbed_start(1, x[0])[None]
    S = pe.System.from_sparse(planted)
    xd = torch.from_numpy(x0).cuda()
    ws = torch.empty((S.newton_workspace_bytes(1) + 7) // 8, dtype=torch.float64, device="cuda")
    resid = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    K, Wm = min(args.steps, 20), min(args.warmup, 3)
    xs = xd.clone()

    def step():
        xd.copy_(xs)  # every timed step starts from the same point
        S.newton_step(xd, workspace=ws, resid=resid, stream=st)
    dt, ms = _time_steps(step, K, Wm, st)
    # the same step captured once in a HIP graph and replayed (x is reset by
    # a captured copy): what remains of the per-launch cost
    gs = torch.cuda.Stream()
    S.newton_step(xd.clone(), workspace=ws, resid=resid, stream=gs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=gs):
        xd.copy_(xs)
        S.newton_step(xd, workspace=ws, resid=resid, stream=gs)
    torch.cuda.synchronize()
    _, ms_graph = _time_steps(g.replay, K, Wm, torch.cuda.current_stream())
    F = torch.empty((1, 2, 2, 256), dtype=torch.float64, device="cuda")
    J = torch.empty((1, 2, 2, 256, 256), dtype=torch.float64, device="cuda")
    _, ms_eval = _time_steps(lambda: S.eval(xd, out=(F, J), stream=st), K, Wm, st)
    S.close()
    from paper_1402_2626_amd import workmodel as WM
    n = 256
    cmadd = WM.lstsq_multiply_adds(n, n)
    out = line("Gauss-Newton step, complex double-double, 256 x 256 system with a planted root (evaluation, "
               "least squares by modified Gram-Schmidt, update)", 2, sys_.n_monomials * K / dt, K, Wm, dt,
               {"name": "newton_dd_n256", "kernel_ms": ms, "graph_replay_ms": ms_graph, "eval_ms": ms_eval,
                "solve_complex_mult_adds": cmadd}, None, None)
    out["metric"] = "Gauss-Newton steps/s (context)"
    out["value"] = K / dt
    out["unit"] = "steps/s"
    print(json.dumps(out), flush=True)


def bench_newton_batch(args):
    """One batched Gauss-Newton step over the 4096 uneven systems at 8 points
    each (every system-point solved by one workgroup), captured in a HIP
    graph and replayed."""
    import numpy as np
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth

    S_count, P = BATCH_COUNT, BATCH_POINTS
    ns = synth.batch_sizes(0, S_count)
    dev = [pe.System.from_sparse(synth.batch_system(0, i, int(ns[i]))) for i in range(S_count)]
    B = pe.Batch(dev)
    rng = synth.rng_for((0, 9))
    x = torch.from_numpy(np.concatenate([synth.unit_circle_points(rng, P, int(n), 2).reshape(-1)
                                         for n in ns])).cuda()
    ws = torch.empty((B.newton_workspace_bytes(P) + 7) // 8, dtype=torch.float64, device="cuda")
    resid = torch.empty((S_count, P, 2), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    xs = x.clone()
    B.newton_step(x, P, workspace=ws, resid=resid, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        B.newton_step(x, P, workspace=ws, resid=resid, stream=s)
    K, Wm = min(args.steps, 3), 1

    def step():
        x.copy_(xs)
        g.replay()
    dt, ms = _time_steps(step, K, Wm, torch.cuda.current_stream())
    out = line("batched Gauss-Newton step (HIP graph), complex double-double: 4096 systems, n uniform in "
               "{32, 64, 128, 256}, 8 points each", 2, S_count * P * K / dt, K, Wm, dt,
               {"name": "newton_batch4096", "kernel_ms": ms}, None, None)
    out["metric"] = "system-point Gauss-Newton steps/s (context)"
    out["unit"] = "system-point steps/s"
    print(json.dumps(out), flush=True)


def bench_terms_product(args):
    """The computation of the paper's Table 1 in its own output form: the
    value and the full gradient of each of 65,024 products of 1,024
    variables (complex double), written per monomial (pe_eval_terms), not
    summed into F and J."""
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    sys_, x = synth.product_workload()
    S = pe.System.from_sparse(sys_)
    xd = torch.from_numpy(x).cuda()
    V = torch.empty((1, 2, 1, sys_.n_monomials), dtype=torch.float64, device="cuda")
    G = torch.empty((1, 2, 1, sys_.nnz), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    K = min(args.steps, 50)
    Wm = min(args.warmup, 5)
    dt, ms = _time_steps(lambda: S.eval_terms(xd, out=(V, G), stream=st), K, Wm, st)
    nbytes = W.terms_bytes_per_point(sys_)
    gbs = nbytes / (ms * 1e-3) / 1e9
    counters = load_counters("terms_d_product_65024x1024")
    out = line("value and gradient of each of 65,024 products of 1,024 variables (the paper's Table 1), "
               "complex double, per-monomial output", 1, sys_.n_monomials * K / dt, K, Wm, dt,
               {"name": "terms_d_product_65024x1024", "kernel_ms": ms, "algorithmic_bytes": nbytes,
                "paper_table1_ms_context": 9.10},
               {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                "traffic": counter_traffic(counters)}, None)
    S.close()
    print(json.dumps(out), flush=True)


def bench_real_qd_chandrasekhar(args):
    """Newton on Chandrasekhar's H-equation in real quad double at n = 1016
    (the first row of the paper's Table 4: 7 iterations, evaluation on its
    CPU), one step timed (evaluation and least squares on the GPU)."""
    import numpy as np
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth

    n, L = 1016, 4
    sys_ = synth.chandrasekhar_system(n, L)
    S = pe.System(pe.PE_REAL | L, n, sys_.poly_ptr, sys_.mon_ptr, sys_.var_idx, sys_.exps,
                  np.ascontiguousarray(sys_.coef[:1]))
    x0 = np.zeros((1, 1, L, n))
    x0[0, 0, 0] = 1.0
    xd = torch.from_numpy(x0).cuda()
    xs = xd.clone()
    ws = torch.empty((S.newton_workspace_bytes(1) + 7) // 8, dtype=torch.float64, device="cuda")
    resid = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    K, Wm = min(args.steps, 3), 1

    def step():
        xd.copy_(xs)
        S.newton_step(xd, workspace=ws, resid=resid, stream=st)
    dt, ms = _time_steps(step, K, Wm, st)
    S.close()
    out = line("Gauss-Newton step, real quad double, Chandrasekhar H-equation n = 1016 (c = 33/64)", 4,
               K / dt, K, Wm, dt, {"name": "newton_rqd_chandrasekhar1016", "kernel_ms": ms,
                                   "paper_table4_gpu_s_for_7_iterations_context": 59.57}, None, None)
    out["metric"] = "Gauss-Newton steps/s (context)"
    out["unit"] = "steps/s"
    out["dtype"] = "f64 (quad-double real)"
    print(json.dumps(out), flush=True)


# the paper's Newton runs on Chandrasekhar's H-equation: Table 3 (six
# iterations, complex double double) and Table 4 (seven iterations, real quad
# double); its accelerated wall-clock times in seconds, context only
TABLE3_GPU2_S = {1024: 20.083, 2048: 149.770, 3072: 495.565, 4096: 1164.243}
TABLE4_GPU_S = {1016: 59.570, 2032: 402.595, 3048: 1281.047, 4064: 2542.440}


def bench_newton_tables(args, table):
    """All iterations of the paper's Newton runs on the H-equation from
    H = 1, evaluation and least squares on the GPU, one line per dimension."""
    import numpy as np
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth

    from paper_1402_2626_amd import workmodel as WM

    real = table == 4
    L, iters, ref = (4, 7, TABLE4_GPU_S) if real else (2, 6, TABLE3_GPU2_S)
    for n in sorted(ref):
        sys_ = synth.chandrasekhar_system(n, L)
        if real:
            S = pe.System(pe.PE_REAL | L, n, sys_.poly_ptr, sys_.mon_ptr, sys_.var_idx, sys_.exps,
                          np.ascontiguousarray(sys_.coef[:1]))
        else:
            S = pe.System.from_sparse(sys_)
        C = 1 if real else 2
        x = torch.zeros((1, C, L, n), dtype=torch.float64, device="cuda")
        x[0, 0, 0] = 1.0
        ws = torch.empty((S.newton_workspace_bytes(1) + 7) // 8, dtype=torch.float64, device="cuda")
        resid = torch.empty((1, 2), dtype=torch.float64, device="cuda")
        st = torch.cuda.current_stream()
        x0 = x.clone()
        S.newton_step(x, workspace=ws, resid=resid, stream=st)  # warm-up (kernel loading)
        torch.cuda.synchronize()
        x.copy_(x0)
        res = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(st)
        for _ in range(iters):
            S.newton_step(x, workspace=ws, resid=resid, stream=st)
            res.append(resid.clone())
        e1.record(st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        S.close()
        norms = [float(r[0, 0]) for r in res]
        steps = [float(r[0, 1]) for r in res]
        kms = e0.elapsed_time(e1)
        # the solve's flops only (the evaluation is O(n), the solve O(n^3))
        flops = iters * WM.lstsq_flops((pe.PE_REAL | L) if real else L, n, n)
        desc = (f"{iters} Gauss-Newton iterations, {'real quad' if real else 'complex double'} double, "
                f"Chandrasekhar H-equation n = {n} (c = 33/64) from H = 1")
        out = line(desc, L, iters / dt, iters, 1, dt,
                   {"name": f"newton_table{table}_n{n}", "kernel_ms": kms,
                    "F_norm_per_iteration": norms, "step_inf_norm_per_iteration": steps,
                    "solve_flops_per_iteration": flops / iters,
                    f"paper_table{table}_gpu_s_context": ref[n]}, alu_roofline(flops, kms), None)
        out["metric"] = "Gauss-Newton iterations/s (context)"
        out["unit"] = "iterations/s"
        if real:
            out["dtype"] = "f64 (quad-double real)"
        print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-rows", type=int, default=96, help="oracle rows of the single-system workloads")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes (reference for HBM byte counters)")
    ap.add_argument("--shapes", action="store_true",
                    help="time every compiled launch shape of a single-system workload and exit")
    ap.add_argument("--autotune", action="store_true", help="run pe_autotune before timing (single systems)")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="dd_batch4096 (default, the reported line); d_n32, dd_n256, qd_n1024, "
                         "dd_adjoint_1024x512, d_product_65024x1024, cyclic_d_n512, cyclic_dd_n512, "
                         "terms_d_product_65024x1024, newton_dd_n256, newton_batch4096 and "
                         "newton_rqd_chandrasekhar1016 print the same kind of line for context; newton_table3 "
                         "and newton_table4 run the paper's Newton experiments on the H-equation")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path (rows of F and J would shard "
              "across GPUs with no exchange); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_reference:
        import torch
        a = torch.ones(args.copy_reference << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes": a.numel() * 8, "launches": 3}), flush=True)
        return
    if args.workload == "dd_batch4096":
        return bench_batch(args)
    if args.workload == "newton_dd_n256":
        return bench_newton_single(args)
    if args.workload == "newton_batch4096":
        return bench_newton_batch(args)
    if args.workload == "terms_d_product_65024x1024":
        return bench_terms_product(args)
    if args.workload == "newton_rqd_chandrasekhar1016":
        return bench_real_qd_chandrasekhar(args)
    if args.workload == "newton_table3":
        return bench_newton_tables(args, 3)
    if args.workload == "newton_table4":
        return bench_newton_tables(args, 4)
    if args.workload == "dd_adjoint_1024x512":
        return bench_adjoint(args)
    if args.workload == "d_product_65024x1024":
        return bench_product(args)
    if args.workload in CYCLIC:
        return bench_cyclic(args)
    return bench_single(args)


if __name__ == "__main__":
    main()
