"""Helpers for the GPU parity tests: run the library, compare with the oracle.

The oracle runs in worker processes started with the ``spawn`` method (fresh
interpreters that never touch the GPU)."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

import oracle as O

TAU = {1: 1e-13, 2: 1e-28, 4: 1e-58}


def tolerance(sys_) -> float:
    """Per-level tolerance scaled by the largest monomial degree."""
    dmax = int(sys_.degrees().max()) if sys_.n_monomials else 0
    return TAU[sys_.level] * max(1.0, dmax / 32.0)


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _rows_job(args):
    sys_, x, F_rows, J_rows, rows = args
    Fx, Jx = O.eval_rows(sys_, x, rows, want_J=J_rows is not None)
    SF, SJ = O.abs_sums_rows(sys_, x, rows)
    eF = eJ = 0.0
    for i, p in enumerate(rows):
        eF = max(eF, O.rel_error(F_rows[0, :, i], F_rows[1, :, i], Fx[p], SF[p]))
        if J_rows is None:
            continue
        for j in range(sys_.n_vars):
            eJ = max(eJ, O.rel_error(J_rows[0, :, i, j], J_rows[1, :, i, j], Jx[p].get(j, O.ZERO),
                                     SJ[p].get(j, 0.0)))
    return eF, eJ


def _cols_job(args):
    sys_, x, J_cols, cols = args
    Jc = O.eval_columns(sys_, x, cols)
    Sc = O.abs_sums_columns(sys_, x, cols)
    e = 0.0
    for i, j in enumerate(cols):
        for p in range(sys_.n_polys):
            e = max(e, O.rel_error(J_cols[0, :, p, i], J_cols[1, :, p, i], Jc[j].get(p, O.ZERO),
                                   Sc[j].get(p, 0.0)))
    return e


def _entries_job(args):
    """F_p and J_{p, cols} of one row p of a system given as its own
    one-row system ``sub`` (plain definition: F by products of powers, each
    partial derivative by its own product)."""
    sub, x, F_got, J_got, cols = args
    X = O.point_from_limbs(x)
    Fx = O.system_value_at(sub, X)[0]
    SF = O.abs_sums_values(sub, x, [0])[0]
    eF = O.rel_error(F_got[0], F_got[1], Fx, SF)
    eJ = 0.0
    if cols:
        Jc = O.eval_columns(sub, x, cols)
        Sc = O.abs_sums_columns(sub, x, cols)
        for i, j in enumerate(cols):
            eJ = max(eJ, O.rel_error(J_got[0, :, i], J_got[1, :, i], Jc[j].get(0, O.ZERO), Sc[j].get(0, 0.0)))
    return eF, eJ


def row_subsystem(sys_, rows):
    """The polynomials `rows` of a system as a system of their own (same
    variables), for oracle checks of sampled rows of a large system."""
    from paper_1402_2626_amd.synth import PolySystem
    mons = [list(range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1]))) for p in rows]
    poly_ptr = np.cumsum([0] + [len(m) for m in mons]).astype(np.int64)
    flat = [t for m in mons for t in m]
    mon_ptr = np.cumsum([0] + [int(sys_.mon_ptr[t + 1] - sys_.mon_ptr[t]) for t in flat]).astype(np.int64)
    occ = (np.concatenate([np.arange(sys_.mon_ptr[t], sys_.mon_ptr[t + 1]) for t in flat]).astype(np.int64)
           if flat else np.zeros(0, np.int64))
    return PolySystem(level=sys_.level, n_vars=sys_.n_vars, poly_ptr=poly_ptr, mon_ptr=mon_ptr,
                      var_idx=np.ascontiguousarray(sys_.var_idx[occ]), exps=np.ascontiguousarray(sys_.exps[occ]),
                      coef=np.ascontiguousarray(sys_.coef[:, :, flat]), name=sys_.name + "_rows")


def max_errors_entries(sys_, x, F, J, picks, parallel: bool = True):
    """Largest metric over sampled entries: ``picks`` maps a row p to the
    columns of J to check there (F_p is always checked).  x: [2, L, n];
    F: [2, L, N]; J: [2, L, N, n] (numpy)."""
    jobs = []
    for p, cols in picks.items():
        cols = list(cols)
        sub = row_subsystem(sys_, [p])
        jobs.append((sub, x, F[:, :, p], J[:, :, p, cols] if cols else None, cols))
    if parallel and len(jobs) > 1:
        with _pool(min(workers(), len(jobs))) as pool:
            res = pool.map(_entries_job, jobs)
    else:
        res = [_entries_job(j) for j in jobs]
    return max(r[0] for r in res), max(r[1] for r in res)


def _value_ratio_job(args):
    sub, x = args
    X = O.point_from_limbs(x)
    F = O.system_value_at(sub, X)
    S = O.abs_sums_values(sub, x, range(sub.n_polys))
    return max(O.cdy_abs_float(F[p]) / S[p] if S[p] else (0.0 if O.cdy_is_zero(F[p]) else float("inf"))
               for p in range(sub.n_polys))


def max_value_ratio(sys_, x, rows):
    """max over rows p of |F_p(x)| / S_F(p), exactly from the limbs of x
    ([2, L, n]): how far x is from a root, relative to the terms' size."""
    rows = list(rows)
    per = max(1, (len(rows) + 4 * workers() - 1) // (4 * workers()))
    jobs = [(row_subsystem(sys_, rows[a:a + per]), x) for a in range(0, len(rows), per)]
    with _pool(min(workers(), len(jobs))) as pool:
        return max(pool.map(_value_ratio_job, jobs))


def _values_job(args):
    sub, x = args
    return O.system_value_at(sub, O.point_from_limbs(x))


def values_at(sys_, x):
    """[2, L, N] limbs of F(x) computed exactly by the oracle (rows in
    parallel) and rounded to the system's level."""
    rows = list(range(sys_.n_polys))
    per = max(1, (len(rows) + 4 * workers() - 1) // (4 * workers()))
    jobs = [(row_subsystem(sys_, rows[a:a + per]), x) for a in range(0, len(rows), per)]
    with _pool(min(workers(), len(jobs))) as pool:
        vals = [v for part in pool.map(_values_job, jobs) for v in part]
    return O.round_point(vals, sys_.level)


def _shift_job(args):
    sub, x, c, t = args
    X = O.point_from_limbs(x)
    F = O.system_value_at(sub, X)
    S = O.abs_sums_values(sub, x, range(sub.n_polys))
    C = O.point_from_limbs(c)
    m, e = O.dy_from_float(t)
    worst = 0.0
    for p in range(sub.n_polys):
        tc = (C[p][0] * m, C[p][1] * m, C[p][2] + e)
        worst = max(worst, O.cdy_abs_float(O.cdy_add(F[p], O.cdy_neg(tc))) / (S[p] + O.cdy_abs_float(tc)))
    return worst


def max_shift_ratio(sys_, x, c, t):
    """max over rows of |f_p(x) - t c_p| / (S_F(p) + |t c_p|), exactly."""
    jobs = [(row_subsystem(sys_, [p]), x, c[:, :, p:p + 1], t) for p in range(sys_.n_polys)]
    with _pool(min(workers(), len(jobs))) as pool:
        return max(pool.map(_shift_job, jobs))


def _pool(n):
    return mp.get_context("spawn").Pool(n)


def max_errors_rows(sys_, x, F, J, rows, parallel: bool = True):
    """Largest metric over F[rows] and J[rows, :] at one point.
    x: [2, L, n]; F: [2, L, N]; J: [2, L, N, n] or None (numpy)."""
    rows = list(rows)
    per = max(1, (len(rows) + 4 * workers() - 1) // (4 * workers()))
    jobs = []
    for a in range(0, len(rows), per):
        rr = rows[a:a + per]
        jobs.append((sys_, x, F[:, :, rr], None if J is None else J[:, :, rr, :], rr))
    if parallel and len(jobs) > 1:
        with _pool(min(workers(), len(jobs))) as pool:
            res = pool.map(_rows_job, jobs)
    else:
        res = [_rows_job(j) for j in jobs]
    return max(r[0] for r in res), max(r[1] for r in res)


def max_error_cols(sys_, x, J, cols, parallel: bool = True):
    cols = list(cols)
    jobs = [(sys_, x, J[:, :, :, [j]], [j]) for j in cols]
    if parallel and len(jobs) > 1:
        with _pool(min(workers(), len(jobs))) as pool:
            res = pool.map(_cols_job, jobs)
    else:
        res = [_cols_job(j) for j in jobs]
    return max(res)


def to_device(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def flush(msg: str):
    print(msg, flush=True)
