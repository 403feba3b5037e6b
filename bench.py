"""Benchmark: evaluation of F and the full Jacobian of a sparse polynomial
system at a complex point, in complex double double.

Workload: n = 256 variables, N = 256 polynomials of 256 monomials each, every
monomial the product of k = 16 distinct variables (uniform without
replacement) with exponents uniform in {1..4}, unit-circle coefficients and
point (seeded, synthetic).  One step is one pe_eval call computing F and the
256 x 256 J at one point; inputs are resident in HBM.

Prints one JSON line: monomial evaluations (value and all partials, summed
into F and J) per second, the roofline of the evaluation kernel, and the CPU
oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "dd_n256"
LEVEL_NAME = {1: "double", 2: "double-double", 4: "quad-double"}


def describe(name):
    from paper_1402_2626_amd import synth
    if name == "dd_batch4096":
        return ("dd_batch4096: 4096 systems, n = N = m uniform in {32,64,128,256}, k = min(16, n/4), "
                "exps {1..3}, 8 points each, one persistent launch")
    w = synth.WORKLOADS[name]
    return (f"{name}: n={w['n']}, N={w['N']}, {w['m']} monomials/poly, k={w['k']}, "
            f"exps {{1..{w['exp_hi']}}}, {w['P']} point(s)")
PEAK_FP64_TFLOPS = 78.6  # 256 CUs x 64 FP64 FMA lanes/clk x 2 flops x 2.4 GHz
PEAK_HBM_GBS = 8000.0    # HBM3E

# HBM bytes of the evaluation kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# passes (KiB per dispatch) scaled by what the same counters read for a plain
# device copy of known size.  The figures hold for the kernel sources they
# were taken with: `traffic` is null when the sources have changed since.
COUNTERS = {"dd_n256": os.path.join(ROOT, "profiles", "eval_rows_dd_n256_counters.json"),
            "d_product_65024x1024": os.path.join(ROOT, "profiles", "eval_rows_d_product_counters.json")}
KERNEL_SOURCES = ["eval_kernels.hpp", "mdarith.hpp", "layout.hpp", "polyeval.hip", "packer.cpp", "packer.hpp"]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1402_2626_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(workload: str):
    """HBM bytes per launch of the evaluation kernel, or None."""
    try:
        with open(COUNTERS[workload]) as fh:
            c = json.load(fh)
    except (KeyError, OSError, ValueError):
        return None
    if c.get("workload") != workload or c.get("source_sha256") != kernel_source_digest():
        return None
    return (c["fetch_kib_per_dispatch"] * c["fetch_scale"] + c["write_kib_per_dispatch"] * c["write_scale"]) * 1024.0


def cpu_baseline(sys_, x, rows: int):
    """The exact oracle on the first `rows` polynomials (F and full rows of
    J) at the same point, spread over the host cores; returns monomials/s,
    the cores used and the wall time."""
    import multiprocessing as mp

    cores = max(1, min(16, os.cpu_count() or 1))
    rr = list(range(rows))
    per = max(1, (rows + cores - 1) // cores)
    jobs = [(sys_, x[0], rr[a:a + per]) for a in range(0, rows, per)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(min(cores, len(jobs))) as pool:
        pool.map(_oracle_rows, jobs)
    dt = time.perf_counter() - t0
    m = int(sys_.poly_ptr[rows] - sys_.poly_ptr[0])
    return m / dt, min(cores, len(jobs)), dt


def _oracle_rows(args):
    import oracle as O
    sys_, x, rows = args
    O.eval_rows(sys_, x, rows, want_J=True)
    return len(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-rows", type=int, default=96)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MB",
                    help="only run a plain device copy of MB megabytes (reference for HBM byte counters)")
    ap.add_argument("--shapes", action="store_true",
                    help="time every compiled launch shape of the workload (one line each) and exit")
    ap.add_argument("--autotune", action="store_true", help="run pe_autotune before timing")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="dd_n256 (default, the reported line); d_n32, qd_n1024, dd_adjoint_1024x512, "
                         "dd_batch4096, d_product_65024x1024, cyclic_d_n512 and cyclic_dd_n512 print the "
                         "same kind of line for context")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rows of F and J would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

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
    if args.workload == "dd_adjoint_1024x512":
        return bench_adjoint(args)
    if args.workload == "d_product_65024x1024":
        return bench_product(args)
    if args.workload in CYCLIC:
        return bench_cyclic(args)
    sys_, x = synth.workload(args.workload)
    P = x.shape[0]

    cpu = None
    if not args.no_cpu:
        v, cores, dt = cpu_baseline(sys_, x, args.cpu_rows)
        cpu = {"value": v, "unit": "monomials/s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_rows} of {sys_.n_polys} polynomials (F and full J rows, "
                         f"exact arithmetic) at the same point, {dt:.1f} s wall"}

    import torch
    from paper_1402_2626_amd import polyeval as pe

    dev = torch.device("cuda:0")
    S = pe.System.from_sparse(sys_)
    if args.shapes:
        xd = torch.from_numpy(x).to(dev)
        st = torch.cuda.current_stream()
        for seg in (2, 4, 8, 16):
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
    xd = torch.from_numpy(x).to(dev)
    F = torch.empty((P, 2, sys_.level, sys_.n_polys), dtype=torch.float64, device=dev)
    J = torch.empty((P, 2, sys_.level, sys_.n_polys, sys_.n_vars), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        S.eval(xd, out=(F, J), stream=stream)
    torch.cuda.synchronize()

    # timed region: K steps, each one pe_eval (one kernel launch), enqueued
    # back to back; HIP events on the launch stream bracket the region, so
    # their interval / K is the average launch duration
    K = args.steps
    dt, kern_ms = _time_steps(lambda: S.eval(xd, out=(F, J), stream=stream), K, 0, stream)

    M = sys_.n_monomials
    flops = W.flops_per_point(sys_) * P
    achieved = flops / (kern_ms * 1e-3) / 1e12
    out = {
        "metric": "monomial eval+grad/s (complex %s, F + full J)" % LEVEL_NAME[sys_.level],
        "value": M * P * K / dt,
        "unit": "monomials/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (%s complex)" % LEVEL_NAME[sys_.level],
        "data": "synthetic",
        "config": {"workload": describe(args.workload),
                   "points": P, "monomials": M, "occurrences": sys_.nnz,
                   "F_plus_J_per_s": P * K / dt, "kernel_ms": kern_ms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": counter_traffic(args.workload)},
        "cpu_baseline": cpu,
    }
    S.close()
    print(json.dumps(out), flush=True)


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
    out = {"metric": "monomial adjoint (J^H v) evals/s (complex double-double)",
           "value": sys_.n_monomials * P * args.steps / dt, "unit": "monomials/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 (double-double complex)",
           "data": "synthetic", "config": {"workload": describe("dd_adjoint_1024x512"), "points": P,
                                           "step_ms_events": ms},
           "roofline": {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, "traffic": None},
           "cpu_baseline": None}
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
    dt, ms = _time_steps(lambda: S.eval(xd, out=(F, J), stream=st), K, min(args.warmup, 5), st)
    flops = W.flops_per_point(sys_)
    out = {"metric": "monomial eval+grad/s (complex %s, F + full J)" % LEVEL_NAME[L],
           "value": sys_.n_monomials * K / dt, "unit": "monomials/s", "n_gpus": 1, "steps": K,
           "warmup": min(args.warmup, 5), "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 (%s complex)" % LEVEL_NAME[L], "data": "synthetic",
           "config": {"workload": "%s: cyclic n-roots, n=%d, %d monomials, 1 point" % (args.workload, n, sys_.n_monomials),
                      "kernel_ms": ms, "segment": S.info()["segment"],
                      "paper_table5_ms_context": paper_ms},
           "roofline": {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, "traffic": None},
           "cpu_baseline": None}
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
    dt, ms = _time_steps(lambda: S.eval(xd, out=(F, J), stream=st), K, min(args.warmup, 5), st)
    chunks = sys_.n_polys  # one chunk per polynomial
    nbytes = W.bytes_per_point(sys_, want_J=True, chunks=chunks)
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"metric": "monomial eval+grad/s (complex double, F + full J)",
           "value": sys_.n_monomials * K / dt, "unit": "monomials/s", "n_gpus": 1, "steps": K,
           "warmup": min(args.warmup, 5), "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 (double complex)", "data": "synthetic",
           "config": {"workload": "d_product_65024x1024: 65,024 polynomials, each one monomial of all "
                                  "n=1,024 variables (exponent 1), 1 point; dense J of 1.07 GB",
                      "kernel_ms": ms, "algorithmic_bytes": nbytes,
                      "flops": W.flops_per_point(sys_)},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": gbs / PEAK_HBM_GBS, "traffic": counter_traffic(args.workload)},
           "cpu_baseline": None}
    S.close()
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """4096 uneven DD systems at 8 points each in one persistent launch,
    beside the plain path (one pe_eval launch per system)."""
    import numpy as np
    import torch
    from paper_1402_2626_amd import polyeval as pe
    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    S_count, P = 4096, 8
    ns = synth.batch_sizes(0, S_count)
    t0 = time.perf_counter()
    systems, dev, flops, mons = [], [], 0.0, 0
    for i in range(S_count):
        sy = synth.batch_system(0, i, int(ns[i]))
        dev.append(pe.System.from_sparse(sy))
        flops += W.flops_per_point(sy) * P
        mons += sy.n_monomials * P
        del sy
        if i % 512 == 0:
            print(f"# loaded {i} systems, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    B = pe.Batch(dev)
    rng = synth.rng_for((0, 9))
    x = torch.from_numpy(np.concatenate([synth.unit_circle_points(rng, P, int(n), 2).reshape(-1)
                                         for n in ns])).cuda()
    F = torch.empty(int(B.F_off[-1]) * P, dtype=torch.float64, device="cuda")
    J = torch.empty(int(B.J_off[-1]) * P, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    K = max(1, min(args.steps, 5))
    dt, ms = _time_steps(lambda: B.eval(x, P, out=(F, J), stream=st), K, 1, st)
    # plain path: one launch per system
    offs = [(int(B.x_off[i]) * P, int(B.F_off[i]) * P, int(B.J_off[i]) * P) for i in range(S_count)]
    views = []
    for i in range(S_count):
        n = int(ns[i])
        xo, fo, jo = offs[i]
        views.append((x[xo:xo + P * 4 * n].view(P, 2, 2, n), F[fo:fo + P * 4 * n].view(P, 2, 2, n),
                      J[jo:jo + P * 4 * n * n].view(P, 2, 2, n, n)))

    def plain():
        for i in range(S_count):
            xv, fv, jv = views[i]
            dev[i].eval(xv, out=(fv, jv), stream=st)
    dt_plain, ms_plain = _time_steps(plain, 1, 1, st)
    out = {"metric": "monomial eval+grad/s (complex double-double, batched uneven systems)",
           "value": mons * K / dt, "unit": "monomials/s", "n_gpus": 1, "steps": K, "warmup": 1,
           "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 (double-double complex)", "data": "synthetic",
           "config": {"workload": describe("dd_batch4096"), "system_points_per_s": S_count * P * K / dt,
                      "plain_path_ms": dt_plain * 1e3, "plain_monomials_per_s": mons / dt_plain,
                      "monomials": mons},
           "roofline": {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, "traffic": None},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
