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
PEAK_FP64_TFLOPS = 78.6  # 256 CUs x 64 FP64 FMA lanes/clk x 2 flops x 2.4 GHz


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
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(rows of F and J shard across GPUs with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    from paper_1402_2626_amd import synth
    from paper_1402_2626_amd import workmodel as W

    sys_, x = synth.workload(WORKLOAD)
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
    xd = torch.from_numpy(x).to(dev)
    F = torch.empty((P, 2, sys_.level, sys_.n_polys), dtype=torch.float64, device=dev)
    J = torch.empty((P, 2, sys_.level, sys_.n_polys, sys_.n_vars), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        S.eval(xd, out=(F, J), stream=stream)
    torch.cuda.synchronize()

    # timed region: K steps, each one pe_eval (one kernel launch)
    K = args.steps
    t0 = time.perf_counter()
    for _ in range(K):
        S.eval(xd, out=(F, J), stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # kernel duration with events on the launch stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for a, b in ev:
        a.record(stream)
        S.eval(xd, out=(F, J), stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    kern_ms = sum(a.elapsed_time(b) for a, b in ev) / K

    M = sys_.n_monomials
    flops = W.flops_per_point(sys_) * P
    achieved = flops / (kern_ms * 1e-3) / 1e12
    out = {
        "metric": "monomial eval+grad/s (complex DD, F + full J)",
        "value": M * P * K / dt,
        "unit": "monomials/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (double-double complex)",
        "data": "synthetic",
        "config": {"workload": "dd_n256: n=256, N=256, 256 monomials/poly, k=16, exps {1..4}, 1 point",
                   "points": P, "monomials": M, "occurrences": sys_.nnz,
                   "F_plus_J_per_s": P * K / dt, "kernel_ms": kern_ms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None},
        "cpu_baseline": cpu,
    }
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
