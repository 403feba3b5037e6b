"""Exact CPU oracle (test infrastructure only; see the package docstring).

What is computed (Problem Statement and Section 2 of Verschelde & Yu, "GPU
acceleration of Newton's method for large systems of polynomial equations in
double double and quad double arithmetic"):

* a system in sparse distributed form: polynomial p is a list of monomials
  t = (c_t; (i_{t,r}, d_{t,r}) for r = 1..k_t) with distinct variables and
  positive exponents (Section 2.1, eq. (1));
* F_p(x)     = sum over t in p of c_t * prod_r x_{i_r}^{d_r};
* J_{p,j}(x) = sum over t in p containing x_j (as i_r = j) of
               c_t * d_r * x_j^{d_r - 1} * prod_{s != r} x_{i_s}^{d_s},
  which is the product rule applied to eq. (1): the exponent d_r multiplies
  the derivative (Section 2.3) and the common factor x_j^{d_r - 1} divides
  every partial derivative (Section 2.1).

The oracle evaluates these definitions directly, the "straightforward"
method of Section 2.2: every power by repeated multiplication, every partial
derivative as its own product of the other factors, sums left to right.  No
division, no product tree and no shared partial products.  The arithmetic is
exact: a complex dyadic number is a triple (re, im, e) of Python integers
meaning (re + i*im) * 2^e.  Level-L inputs (L doubles per real part) are
converted exactly by summing their limbs.

Also here: the absolute sums that normalise the error metric, rounding of
exact values to level-L limbs, the adjoint J^H v by its definition, and a
Gauss-Newton step (Section 4, Problem Statement) whose least-squares solve is
mpmath's Householder QR factorisation at high precision (not modified
Gram-Schmidt, so it shares no algorithm with the library's solver).
"""
from __future__ import annotations

import math
from typing import Iterable, Sequence

import numpy as np

__all__ = [
    "dy_from_float", "cdy_from_limbs", "cdy_mul", "cdy_add", "cdy_neg", "cdy_conj",
    "cdy_scale", "cdy_is_zero", "cdy_to_complex", "cdy_abs_float", "cdy_to_limbs",
    "dy_to_double", "ONE", "ZERO", "point_from_limbs", "monomial_value_and_partials",
    "eval_rows", "eval_columns", "eval_system", "abs_sums_rows", "rel_error",
    "max_rel_error_rows", "adjoint_exact", "adjoint_columns", "gauss_newton_step_mp",
    "system_value_at", "round_point", "speelpenning_straightforward", "plant_root",
    "abs_sums_columns", "abs_sums_values", "lstsq_limbs", "homotopy_step_mp", "homotopy_track_mp",
    "eval_terms", "abs_terms",
]

# --------------------------------------------------------------------------
# exact complex dyadic arithmetic
# --------------------------------------------------------------------------

ZERO = (0, 0, 0)
ONE = (1, 0, 0)


def dy_from_float(f: float):
    """Exact (mantissa, exponent) of a finite double."""
    if f == 0.0:
        return 0, 0
    num, den = float(f).as_integer_ratio()
    return num, -(den.bit_length() - 1)


def _dy_add(a, b):
    (am, ae), (bm, be) = a, b
    if ae <= be:
        return am + (bm << (be - ae)), ae
    return (am << (ae - be)) + bm, be


def cdy_from_limbs(re_limbs: Iterable[float], im_limbs: Iterable[float]):
    """Exact value of a level-L complex number given by its limbs."""
    r = (0, 0)
    for f in re_limbs:
        r = _dy_add(r, dy_from_float(float(f)))
    i = (0, 0)
    for f in im_limbs:
        i = _dy_add(i, dy_from_float(float(f)))
    e = min(r[1], i[1])
    return (r[0] << (r[1] - e), i[0] << (i[1] - e), e)


def cdy_mul(a, b):
    ar, ai, ae = a
    br, bi, be = b
    return (ar * br - ai * bi, ar * bi + ai * br, ae + be)


def cdy_add(a, b):
    ar, ai, ae = a
    br, bi, be = b
    if ae <= be:
        s = be - ae
        return (ar + (br << s), ai + (bi << s), ae)
    s = ae - be
    return ((ar << s) + br, (ai << s) + bi, be)


def cdy_neg(a):
    return (-a[0], -a[1], a[2])


def cdy_conj(a):
    return (a[0], -a[1], a[2])


def cdy_scale(a, d: int):
    """Multiply by an integer."""
    return (a[0] * d, a[1] * d, a[2])


def cdy_is_zero(a) -> bool:
    return a[0] == 0 and a[1] == 0


def _int_times_pow2_to_float(m: int, e: int) -> float:
    """float(m * 2^e), correctly rounded for moderate sizes (for reporting)."""
    if m == 0:
        return 0.0
    if e >= 0:
        try:
            return float(m << e)
        except OverflowError:
            return math.copysign(math.inf, m)
    return m / (1 << -e)


def cdy_to_complex(a) -> complex:
    return complex(_int_times_pow2_to_float(a[0], a[2]), _int_times_pow2_to_float(a[1], a[2]))


def cdy_abs_float(a) -> float:
    """|a| as a float (for error reporting only)."""
    re, im, e = a
    big = max(abs(re), abs(im)).bit_length()
    if big > 900:  # keep the conversion in range
        sh = big - 900
        re, im, e = re >> sh, im >> sh, e + sh
    return math.hypot(_int_times_pow2_to_float(re, e), _int_times_pow2_to_float(im, e))


def dy_to_double(m: int, e: int) -> float:
    """Round m * 2^e to the nearest double (ties to even).  Python's integer
    true division and int-to-float conversion are correctly rounded."""
    if m == 0:
        return 0.0
    if e >= 0:
        return float(m << e)
    return m / (1 << -e)


def _dy_to_limbs(m: int, e: int, L: int):
    """Level-L expansion of m*2^e: each limb is the nearest double to what the
    limbs above it leave over."""
    out = []
    for _ in range(L):
        f = dy_to_double(m, e)
        out.append(f)
        fm, fe = dy_from_float(f)
        m, e = _dy_add((m, e), (-fm, fe))
    return out


def cdy_to_limbs(a, L: int) -> np.ndarray:
    """``[2, L]`` limbs of the exact complex value ``a``."""
    re, im, e = a
    return np.array([_dy_to_limbs(re, e, L), _dy_to_limbs(im, e, L)], dtype=np.float64)


def point_from_limbs(x: np.ndarray):
    """``x[2, L, n]`` -> list of n exact complex values."""
    n = x.shape[-1]
    return [cdy_from_limbs(x[0, :, j], x[1, :, j]) for j in range(n)]


def round_point(values, L: int) -> np.ndarray:
    """List of exact complex values -> ``[2, L, n]`` limbs."""
    out = np.zeros((2, L, len(values)))
    for j, v in enumerate(values):
        out[:, :, j] = cdy_to_limbs(v, L)
    return out


# --------------------------------------------------------------------------
# the definition of F and J
# --------------------------------------------------------------------------

def _power(v, d: int):
    """v^d by repeated multiplication (v^0 = 1)."""
    r = ONE
    for _ in range(d):
        r = cdy_mul(r, v)
    return r


def monomial_value_and_partials(c, xs: Sequence, ds: Sequence[int]):
    """Value c * prod x_r^{d_r} and every partial derivative
    c * d_r * x_r^{d_r - 1} * prod_{s != r} x_s^{d_s}, each computed directly."""
    k = len(xs)
    pw = [_power(xs[r], ds[r]) for r in range(k)]
    value = c
    for r in range(k):
        value = cdy_mul(value, pw[r])
    partials = []
    for r in range(k):
        g = cdy_scale(c, int(ds[r]))
        g = cdy_mul(g, _power(xs[r], ds[r] - 1))
        for s in range(k):
            if s != r:
                g = cdy_mul(g, pw[s])
        partials.append(g)
    return value, partials


def speelpenning_straightforward(xs: Sequence):
    """Product x_1 ... x_n and its gradient, every component as the product of
    the other n-1 factors (Section 2.2, the n^2 - n - 1 multiplication count)."""
    v, g = monomial_value_and_partials(ONE, xs, [1] * len(xs))
    return v, g


def _coef(sys_, t: int):
    return cdy_from_limbs(sys_.coef[0, :, t], sys_.coef[1, :, t])


def eval_rows(sys_, x: np.ndarray, rows: Iterable[int], want_J: bool = True):
    """Exact F_p and row p of J for every p in ``rows`` at point x[2, L, n].

    Returns ``(F, J)``: F maps p -> value, J maps p -> {j: value} (only the
    columns that receive a term; all others are exactly zero)."""
    X = point_from_limbs(x)
    F, J = {}, {}
    for p in rows:
        f = ZERO
        jrow = {}
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            value, partials = monomial_value_and_partials(_coef(sys_, t), [X[v] for v in vs], ds)
            f = cdy_add(f, value)
            if want_J:
                for r, v in enumerate(vs):
                    v = int(v)
                    jrow[v] = cdy_add(jrow[v], partials[r]) if v in jrow else partials[r]
        F[p] = f
        J[p] = jrow
    return F, J


def eval_terms(sys_, x: np.ndarray, monomials: Iterable[int]):
    """The terms before their sum into F and J (Sec. 2.3), for each input
    monomial t in ``monomials`` at point x[2, L, n]: {t: (value, partials)}
    with value = c_t prod_r x_{i_r}^{d_r} and partials[r] the derivative of
    that term with respect to its r-th variable in the input order (the
    order of var_idx), exactly.  The per-monomial output of products of
    variables and their gradients (Sec. 2.2, Tables 1 and 2)."""
    X = point_from_limbs(x)
    out = {}
    for t in monomials:
        vs, ds = sys_.monomial(int(t))
        out[int(t)] = monomial_value_and_partials(_coef(sys_, int(t)), [X[int(v)] for v in vs], ds)
    return out


def abs_terms(sys_, x: np.ndarray, monomials: Iterable[int]):
    """Normalisers of the terms' error metric (float64): {t: (|c| prod |x|^d,
    [|c| d_r |x_r|^(d_r - 1) prod_{s != r} |x_s|^d_s])}."""
    ax = np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
    out = {}
    for t in monomials:
        vs, ds = sys_.monomial(int(t))
        ac = float(np.hypot(sys_.coef[0, :, int(t)].sum(), sys_.coef[1, :, int(t)].sum()))
        pw = [float(ax[int(v)]) ** int(d) for v, d in zip(vs, ds)]
        val = ac * math.prod(pw)
        parts = []
        for r, (v, d) in enumerate(zip(vs, ds)):
            g = ac * int(d) * float(ax[int(v)]) ** (int(d) - 1)
            for q in range(len(vs)):
                if q != r:
                    g *= pw[q]
            parts.append(g)
        out[int(t)] = (val, parts)
    return out


def eval_columns(sys_, x: np.ndarray, cols: Iterable[int]):
    """Exact J_{p,j} for all p and each j in ``cols``: {j: {p: value}}."""
    X = point_from_limbs(x)
    cols = [int(c) for c in cols]
    out = {j: {} for j in cols}
    want = set(cols)
    for p in range(sys_.n_polys):
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            hit = [r for r, v in enumerate(vs) if int(v) in want]
            if not hit:
                continue
            c = _coef(sys_, t)
            xs = [X[v] for v in vs]
            pw = [_power(xs[s], ds[s]) for s in range(len(vs))]
            for r in hit:
                g = cdy_mul(cdy_scale(c, int(ds[r])), _power(xs[r], ds[r] - 1))
                for s in range(len(vs)):
                    if s != r:
                        g = cdy_mul(g, pw[s])
                j = int(vs[r])
                out[j][p] = cdy_add(out[j][p], g) if p in out[j] else g
    return out


def eval_system(sys_, x: np.ndarray, want_J: bool = True):
    return eval_rows(sys_, x, range(sys_.n_polys), want_J)


def system_value_at(sys_, X_exact) -> list:
    """Exact F at a point given as a list of exact complex values."""
    F = []
    for p in range(sys_.n_polys):
        f = ZERO
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            m = _coef(sys_, t)
            for v, d in zip(vs, ds):
                m = cdy_mul(m, _power(X_exact[int(v)], int(d)))
            f = cdy_add(f, m)
        F.append(f)
    return F


# --------------------------------------------------------------------------
# error metric
# --------------------------------------------------------------------------

def abs_sums_rows(sys_, x: np.ndarray, rows: Iterable[int]):
    """Normalisers of the error metric, in float64:
    S_F(p)   = sum_t |c_t| prod |x|^d
    S_J(p,j) = sum_{t, i_r = j} |c_t| d_r |x_j|^{d_r - 1} prod_{s != r} |x_s|^{d_s}.
    Returns ``(SF: {p: float}, SJ: {p: {j: float}})``."""
    ax = np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
    ac = np.hypot(sys_.coef[0].sum(axis=0), sys_.coef[1].sum(axis=0))
    SF, SJ = {}, {}
    for p in rows:
        sf = 0.0
        sj = {}
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            pw = [float(ax[v]) ** int(d) for v, d in zip(vs, ds)]
            sf += float(ac[t]) * math.prod(pw)
            for r, v in enumerate(vs):
                g = float(ac[t]) * int(ds[r]) * float(ax[v]) ** (int(ds[r]) - 1)
                for s in range(len(vs)):
                    if s != r:
                        g *= pw[s]
                sj[int(v)] = sj.get(int(v), 0.0) + g
        SF[p] = sf
        SJ[p] = sj
    return SF, SJ


def abs_sums_values(sys_, x: np.ndarray, rows: Iterable[int]):
    """S_F(p) = sum_t |c_t| prod |x|^d alone (float64), for rows whose
    Jacobian normalisers are not needed: {p: S}."""
    ax = np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
    ac = np.hypot(sys_.coef[0].sum(axis=0), sys_.coef[1].sum(axis=0))
    SF = {}
    for p in rows:
        sf = 0.0
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            sf += float(ac[t]) * math.prod(float(ax[v]) ** int(d) for v, d in zip(vs, ds))
        SF[p] = sf
    return SF


def rel_error(got_re_limbs, got_im_limbs, exact, S: float) -> float:
    """|got - exact| / S for one entry; entries with S = 0 must be exactly 0
    (returns 0.0 if so, inf otherwise)."""
    g = cdy_from_limbs(got_re_limbs, got_im_limbs)
    d = cdy_add(g, cdy_neg(exact))
    if cdy_is_zero(d):
        return 0.0
    if S == 0.0:
        return math.inf
    return cdy_abs_float(d) / S


def max_rel_error_rows(sys_, x: np.ndarray, F_got: np.ndarray, J_got: np.ndarray | None,
                       rows: Sequence[int]):
    """Largest metric over F[p] and J[p, :] for the given rows.

    ``F_got`` is ``[2, L, N]`` and ``J_got`` is ``[2, L, N, n]`` (or None).
    Returns ``(eF, eJ)``."""
    Fx, Jx = eval_rows(sys_, x, rows, want_J=J_got is not None)
    SF, SJ = abs_sums_rows(sys_, x, rows)
    eF = eJ = 0.0
    for p in rows:
        eF = max(eF, rel_error(F_got[0, :, p], F_got[1, :, p], Fx[p], SF[p]))
        if J_got is None:
            continue
        for j in range(sys_.n_vars):
            ex = Jx[p].get(j, ZERO)
            eJ = max(eJ, rel_error(J_got[0, :, p, j], J_got[1, :, p, j], ex, SJ[p].get(j, 0.0)))
    return eF, eJ


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------

def adjoint_exact(J_rows: dict, v_exact: Sequence, n: int):
    """g_j = sum_p conj(J_{p,j}) * v_p from exact rows {p: {j: value}}."""
    g = [ZERO] * n
    for p in sorted(J_rows):
        for j, jpj in J_rows[p].items():
            g[j] = cdy_add(g[j], cdy_mul(cdy_conj(jpj), v_exact[p]))
    return g


def adjoint_columns(sys_, x: np.ndarray, v: np.ndarray, cols: Iterable[int]):
    """g_j = (J^H v)_j for each j in ``cols`` (v is ``[2, L, N]``), exactly."""
    V = point_from_limbs(v)
    colv = eval_columns(sys_, x, cols)
    out = {}
    for j, col in colv.items():
        g = ZERO
        for p in sorted(col):
            g = cdy_add(g, cdy_mul(cdy_conj(col[p]), V[p]))
        out[j] = g
    return out


# --------------------------------------------------------------------------
# Gauss-Newton (Section 4 with the least-squares solve of the Problem Statement)
# --------------------------------------------------------------------------

def gauss_newton_step_mp(sys_, X_exact, prec: int = 512):
    """One Gauss-Newton step from the exact point ``X_exact``.

    A = J(x), b = -F(x) exactly; the least-squares correction comes from
    mpmath's Householder QR (``mpmath.qr``) at ``prec`` bits, dx = R^-1 Q^H b;
    returns the new point as exact
    dyadic values (each mpmath component converted exactly) and
    ``(|F(x)|_2, |dx|_inf)`` as floats."""
    import mpmath

    n, N = sys_.n_vars, sys_.n_polys
    # exact F and J at X
    F, J = {}, {}
    for p in range(N):
        f = ZERO
        jrow = {}
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            value, partials = monomial_value_and_partials(_coef(sys_, t), [X_exact[v] for v in vs], ds)
            f = cdy_add(f, value)
            for r, v in enumerate(vs):
                v = int(v)
                jrow[v] = cdy_add(jrow[v], partials[r]) if v in jrow else partials[r]
        F[p], J[p] = f, jrow
    with mpmath.workprec(prec):
        def mpc(a):
            return mpmath.mpc(mpmath.ldexp(a[0], a[2]), mpmath.ldexp(a[1], a[2]))
        A = mpmath.matrix(N, n)
        b = mpmath.matrix(N, 1)
        for p in range(N):
            for j, val in J[p].items():
                A[p, j] = mpc(val)
            b[p] = -mpc(F[p])
        dx = _lstsq_householder(A, b)
        fnorm = float(mpmath.norm(b, 2))
        dinf = float(max(abs(dx[j]) for j in range(n))) if n else 0.0
        newX = [_mpc_to_cdy(mpc(X_exact[j]) + dx[j]) for j in range(n)]
    return newX, (fnorm, dinf)


def _exact_F_J(sys_, X_exact):
    """Exact F and rows of J at the exact point X_exact."""
    F, J = {}, {}
    for p in range(sys_.n_polys):
        f = ZERO
        jrow = {}
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            value, partials = monomial_value_and_partials(_coef(sys_, t), [X_exact[v] for v in vs], ds)
            f = cdy_add(f, value)
            for r, v in enumerate(vs):
                v = int(v)
                jrow[v] = cdy_add(jrow[v], partials[r]) if v in jrow else partials[r]
        F[p], J[p] = f, jrow
    return F, J


def homotopy_step_mp(sys_, X_exact, c_exact, wF: float, wc: float, prec: int = 512):
    """One step x += dx of the Newton homotopy f(x) - t c (Sec. 5.3): dx
    solves J(x) dx = wF (-f(x)) + wc c in the least-squares sense (Householder
    QR at ``prec`` bits); wF = 1, wc = t is Newton's method on f(x) - t c = 0
    at fixed t, wF = 0, wc = dt the Euler step along the path.  wF and wc are
    doubles, taken exactly.  Returns the new exact point."""
    import mpmath
    n, N = sys_.n_vars, sys_.n_polys
    F, J = _exact_F_J(sys_, X_exact)
    with mpmath.workprec(prec):
        def mpc(a):
            return mpmath.mpc(mpmath.ldexp(a[0], a[2]), mpmath.ldexp(a[1], a[2]))
        A = mpmath.matrix(N, n)
        b = mpmath.matrix(N, 1)
        mwF, mwc = mpmath.mpf(wF), mpmath.mpf(wc)
        for p in range(N):
            for j, val in J[p].items():
                A[p, j] = mpc(val)
            b[p] = -mwF * mpc(F[p]) + mwc * mpc(c_exact[p])
        dx = _lstsq_householder(A, b)
        return [_mpc_to_cdy(mpc(X_exact[j]) + dx[j]) for j in range(n)]


def homotopy_track_mp(sys_, Z_exact, c_exact, steps: int, corrector_iters: int, prec: int = 512):
    """Follow f(x) - t c = 0 from t = 1 (x = z) to t = 0 in ``steps`` equal
    steps of t (t_k = 1 - k / steps rounded to double, as a caller computes
    it), each an Euler predictor and ``corrector_iters`` Newton steps at the
    new t.  Returns the exact end point."""
    X = list(Z_exact)
    for k in range(1, steps + 1):
        t0 = 1.0 - (k - 1) / steps
        t1 = 0.0 if k == steps else 1.0 - k / steps
        X = homotopy_step_mp(sys_, X, c_exact, 0.0, t1 - t0, prec)
        for _ in range(corrector_iters):
            X = homotopy_step_mp(sys_, X, c_exact, 1.0, t1, prec)
    return X


def _lstsq_householder(A, b):
    """Least-squares solution of A x = b at mpmath's working precision: A = QR
    by Householder reflections (``mpmath.qr``), then R x = Q^H b."""
    import mpmath
    Q, Rm = mpmath.qr(A, mode="skinny")
    return mpmath.lu_solve(Rm, Q.H * b)


def lstsq_limbs(Ab: np.ndarray, prec: int = 400):
    """Least-squares solution of A x = b for level-L limbs Ab[2, L, N, n + 1]
    (column n is b), each entry converted exactly; Householder QR at ``prec``
    bits (the solve of the Gauss-Newton step above).  Returns the n components
    as exact dyadic values."""
    import mpmath
    N, n = Ab.shape[2], Ab.shape[3] - 1
    with mpmath.workprec(prec):
        def mpc(a):
            return mpmath.mpc(mpmath.ldexp(a[0], a[2]), mpmath.ldexp(a[1], a[2]))
        A = mpmath.matrix(N, n)
        b = mpmath.matrix(N, 1)
        for i in range(N):
            for j in range(n + 1):
                v = mpc(cdy_from_limbs(Ab[0, :, i, j], Ab[1, :, i, j]))
                if j < n:
                    A[i, j] = v
                else:
                    b[i] = v
        x = _lstsq_householder(A, b)
        return [_mpc_to_cdy(x[j]) for j in range(n)]


def _mpf_to_dy(v):
    import mpmath
    if v == 0:
        return 0, 0
    man, exp = mpmath.frexp(v)  # v = man * 2^exp, 0.5 <= |man| < 1
    # man has at most the working precision; scale it to an integer exactly
    bits = mpmath.mp.prec + 2
    m = int(mpmath.ldexp(man, bits))
    return m, int(exp) - bits


def _mpc_to_cdy(z):
    r = _mpf_to_dy(z.real)
    i = _mpf_to_dy(z.imag)
    e = min(r[1], i[1])
    return (r[0] << (r[1] - e), i[0] << (i[1] - e), e)


def plant_root(sys_, x_star: np.ndarray):
    """Return a copy of ``sys_`` in which every polynomial gets one more
    monomial, the constant -F_p(x*) rounded to the system's level, so that
    x* is a root up to that rounding.  This is the Newton homotopy
    f(x) - f(z) t of Section 5.3 at t = 1."""
    from paper_1402_2626_amd import synth
    L = sys_.level
    F = system_value_at(sys_, point_from_limbs(x_star))
    polys, coefs = [], []
    for p in range(sys_.n_polys):
        mons = []
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            mons.append((0, list(zip(vs.tolist(), ds.tolist()))))
            coefs.append(sys_.coef[:, :, t])
        mons.append((0, []))
        coefs.append(cdy_to_limbs(cdy_neg(F[p]), L))
        polys.append(mons)
    coef = np.stack(coefs, axis=-1) if coefs else np.zeros((2, L, 0))
    return synth.from_monomial_lists(L, sys_.n_vars, polys, coef_limbs=coef,
                                     name=(sys_.name or "system") + "_planted")


def abs_sums_columns(sys_, x: np.ndarray, cols: Iterable[int]):
    """S_J(p, j) for every p and each j in ``cols`` (float64): {j: {p: S}}."""
    ax = np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
    ac = np.hypot(sys_.coef[0].sum(axis=0), sys_.coef[1].sum(axis=0))
    cols = [int(c) for c in cols]
    want = set(cols)
    out = {j: {} for j in cols}
    for p in range(sys_.n_polys):
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            hit = [r for r, v in enumerate(vs) if int(v) in want]
            if not hit:
                continue
            pw = [float(ax[v]) ** int(d) for v, d in zip(vs, ds)]
            for r in hit:
                g = float(ac[t]) * int(ds[r]) * float(ax[vs[r]]) ** (int(ds[r]) - 1)
                for s in range(len(vs)):
                    if s != r:
                        g *= pw[s]
                j = int(vs[r])
                out[j][p] = out[j].get(p, 0.0) + g
    return out
