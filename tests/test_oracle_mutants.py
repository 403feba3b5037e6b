"""Plant plausible mistakes in the oracle (on the CPU) and check that at least
one pin catches each of them."""
import pytest

import oracle.exact as E
import oracle_pins as pins


def _mut_power_off_by_one(v, d):
    r = E.ONE
    for _ in range(d + 1):
        r = E.cdy_mul(r, v)
    return r


def _mut_mul_sign(a, b):
    ar, ai, ae = a
    br, bi, be = b
    return (ar * br + ai * bi, ar * bi + ai * br, ae + be)


def _mut_mul_swap(a, b):
    ar, ai, ae = a
    br, bi, be = b
    return (ar * br - ai * bi, ar * bi - ai * br, ae + be)


def _mut_add_shift(a, b):
    ar, ai, ae = a
    br, bi, be = b
    if ae <= be:
        s = be - ae
        return (ar + (br << s), ai + (bi << s), ae)
    s = ae - be
    return ((ar << s) + br, (ai << s) + bi, ae)  # wrong exponent kept


def _mut_partials_exponent_e(c, xs, ds):
    k = len(xs)
    pw = [E._power(xs[r], ds[r]) for r in range(k)]
    value = c
    for r in range(k):
        value = E.cdy_mul(value, pw[r])
    partials = []
    for r in range(k):
        g = E.cdy_scale(c, int(ds[r]) - 1)  # e = d - 1 instead of d
        g = E.cdy_mul(g, E._power(xs[r], ds[r] - 1))
        for s in range(k):
            if s != r:
                g = E.cdy_mul(g, pw[s])
        partials.append(g)
    return value, partials


def _mut_partials_no_common_factor(c, xs, ds):
    k = len(xs)
    pw = [E._power(xs[r], ds[r]) for r in range(k)]
    value = c
    for r in range(k):
        value = E.cdy_mul(value, pw[r])
    partials = []
    for r in range(k):
        g = E.cdy_scale(c, int(ds[r]))
        for s in range(k):
            if s != r:
                g = E.cdy_mul(g, pw[s])
        partials.append(g)
    return value, partials


def _mut_partials_include_self(c, xs, ds):
    k = len(xs)
    pw = [E._power(xs[r], ds[r]) for r in range(k)]
    value = c
    for r in range(k):
        value = E.cdy_mul(value, pw[r])
    partials = []
    for r in range(k):
        g = E.cdy_scale(c, int(ds[r]))
        g = E.cdy_mul(g, E._power(xs[r], ds[r] - 1))
        for s in range(k):
            g = E.cdy_mul(g, pw[s])  # forgot s != r
        partials.append(g)
    return value, partials


def _mut_partials_dropped_last_factor(c, xs, ds):
    k = len(xs)
    pw = [E._power(xs[r], ds[r]) for r in range(k)]
    value = c
    for r in range(k):
        value = E.cdy_mul(value, pw[r])
    partials = []
    for r in range(k):
        g = E.cdy_scale(c, int(ds[r]))
        g = E.cdy_mul(g, E._power(xs[r], ds[r] - 1))
        for s in range(k - 1):
            if s != r:
                g = E.cdy_mul(g, pw[s])
        partials.append(g)
    return value, partials


def _mut_conj_noop(a):
    return a


def _mut_from_limbs_drop_last(re_limbs, im_limbs):
    re_limbs = list(re_limbs)[:-1] or [0.0]
    im_limbs = list(im_limbs)[:-1] or [0.0]
    r = (0, 0)
    for f in re_limbs:
        r = E._dy_add(r, E.dy_from_float(float(f)))
    i = (0, 0)
    for f in im_limbs:
        i = E._dy_add(i, E.dy_from_float(float(f)))
    e = min(r[1], i[1])
    return (r[0] << (r[1] - e), i[0] << (i[1] - e), e)


def _make_eval_rows_drop_last_monomial():
    orig = E.eval_rows

    def eval_rows(sys_, x, rows, want_J=True):
        X = E.point_from_limbs(x)
        F, J = {}, {}
        for p in rows:
            f = E.ZERO
            jrow = {}
            for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1]) - 1):
                vs, ds = sys_.monomial(t)
                value, partials = E.monomial_value_and_partials(E._coef(sys_, t), [X[v] for v in vs], ds)
                f = E.cdy_add(f, value)
                for r, v in enumerate(vs):
                    v = int(v)
                    jrow[v] = E.cdy_add(jrow[v], partials[r]) if v in jrow else partials[r]
            F[p] = f
            J[p] = jrow
        return F, J
    del orig
    return eval_rows


def _make_eval_rows_transposed():
    orig = E.eval_rows

    def eval_rows(sys_, x, rows, want_J=True):
        F, J = orig(sys_, x, range(sys_.n_polys), want_J)
        T = {p: {} for p in range(max(sys_.n_polys, sys_.n_vars))}
        for p, row in J.items():
            for j, v in row.items():
                T.setdefault(j, {})[p] = v
        return {p: F[p] for p in rows}, {p: T.get(p, {}) for p in rows}
    return eval_rows


def _make_eval_columns(exp_factor_shift=0, drop_common=False):
    def eval_columns(sys_, x, cols):
        X = E.point_from_limbs(x)
        cols = [int(c) for c in cols]
        out = {j: {} for j in cols}
        want = set(cols)
        for p in range(sys_.n_polys):
            for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
                vs, ds = sys_.monomial(t)
                hit = [r for r, v in enumerate(vs) if int(v) in want]
                if not hit:
                    continue
                c = E._coef(sys_, t)
                xs = [X[v] for v in vs]
                pw = [E._power(xs[s], ds[s]) for s in range(len(vs))]
                for r in hit:
                    g = E.cdy_scale(c, int(ds[r]) - exp_factor_shift)
                    if not drop_common:
                        g = E.cdy_mul(g, E._power(xs[r], ds[r] - 1))
                    for s in range(len(vs)):
                        if s != r:
                            g = E.cdy_mul(g, pw[s])
                    j = int(vs[r])
                    out[j][p] = E.cdy_add(out[j][p], g) if p in out[j] else g
        return out
    return eval_columns


def _make_abs_sums_columns_no_exponent():
    import math as _m
    import numpy as _np

    def abs_sums_columns(sys_, x, cols):
        ax = _np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
        ac = _np.hypot(sys_.coef[0].sum(axis=0), sys_.coef[1].sum(axis=0))
        cols = [int(c) for c in cols]
        want = set(cols)
        out = {j: {} for j in cols}
        for p in range(sys_.n_polys):
            for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
                vs, ds = sys_.monomial(t)
                pw = [float(ax[v]) ** int(d) for v, d in zip(vs, ds)]
                for r, v in enumerate(vs):
                    if int(v) not in want:
                        continue
                    g = float(ac[t]) * float(ax[v]) ** (int(ds[r]) - 1)  # exponent factor dropped
                    g *= _m.prod(pw[s] for s in range(len(vs)) if s != r)
                    out[int(v)][p] = out[int(v)].get(p, 0.0) + g
        return out
    return abs_sums_columns


def _make_abs_sums_rows_no_power():
    orig = E.abs_sums_rows

    def abs_sums_rows(sys_, x, rows):
        import numpy as _np
        ax = _np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
        ac = _np.hypot(sys_.coef[0].sum(axis=0), sys_.coef[1].sum(axis=0))
        SF, SJ = {}, {}
        for p in rows:
            sf, sj = 0.0, {}
            for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
                vs, ds = sys_.monomial(t)
                pw = [float(ax[v]) ** int(d) for v, d in zip(vs, ds)]
                m = float(ac[t])
                for w in pw:
                    m *= w
                sf += m
                for r, v in enumerate(vs):
                    g = float(ac[t]) * int(ds[r])  # |x_j|^(d-1) dropped
                    for s in range(len(vs)):
                        if s != r:
                            g *= pw[s]
                    sj[int(v)] = sj.get(int(v), 0.0) + g
            SF[p], SJ[p] = sf, sj
        return SF, SJ
    del orig
    return abs_sums_rows


def _mut_rel_error_zero_scale_ok(got_re, got_im, exact, S):
    g = E.cdy_from_limbs(got_re, got_im)
    d = E.cdy_add(g, E.cdy_neg(exact))
    if E.cdy_is_zero(d) or S == 0.0:
        return 0.0
    return E.cdy_abs_float(d) / S


def _mut_rel_error_lenient(got_re, got_im, exact, S):
    g = E.cdy_from_limbs(got_re, got_im)
    d = E.cdy_add(g, E.cdy_neg(exact))
    if E.cdy_is_zero(d):
        return 0.0
    if S == 0.0:
        return float("inf")
    return E.cdy_abs_float(d) / (1e6 * S)


def _mut_lstsq_transpose(A, b):
    import mpmath
    Q, Rm = mpmath.qr(A, mode="skinny")
    return mpmath.lu_solve(Rm, Q.T * b)  # Q^T instead of Q^H


def _mut_abs_values_no_power(sys_, x, rows):
    import numpy as _np
    ax = _np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
    ac = _np.hypot(sys_.coef[0].sum(axis=0), sys_.coef[1].sum(axis=0))
    SF = {}
    for p in rows:
        sf = 0.0
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            m = float(ac[t])
            for v in vs:
                m *= float(ax[v])  # exponents dropped
            sf += m
        SF[p] = sf
    return SF


def _make_homotopy_step_sign():
    orig = E.homotopy_step_mp

    def homotopy_step_mp(sys_, X, c, wF, wc, prec=512):
        return orig(sys_, X, c, wF, -wc, prec)  # f(x) + t c instead of f(x) - t c
    return homotopy_step_mp


def _make_terms_sorted_order():
    orig = E.eval_terms

    def eval_terms(sys_, x, monomials):
        # partials in increasing variable order instead of the input order
        out = orig(sys_, x, monomials)
        res = {}
        for t, (v, g) in out.items():
            vs, _ = sys_.monomial(t)
            order = sorted(range(len(vs)), key=lambda r: int(vs[r]))
            res[t] = (v, [g[r] for r in order])
        return res
    return eval_terms


def _make_terms_no_coefficient():
    def eval_terms(sys_, x, monomials):
        X = E.point_from_limbs(x)
        out = {}
        for t in monomials:
            vs, ds = sys_.monomial(int(t))
            out[int(t)] = E.monomial_value_and_partials(E.ONE, [X[int(v)] for v in vs], ds)  # c_t dropped
        return out
    return eval_terms


def _mut_abs_terms_no_exponent(sys_, x, monomials):
    import numpy as np
    ax = np.hypot(x[0].sum(axis=0), x[1].sum(axis=0))
    out = {}
    for t in monomials:
        vs, ds = sys_.monomial(int(t))
        ac = float(np.hypot(sys_.coef[0, :, int(t)].sum(), sys_.coef[1, :, int(t)].sum()))
        pw = [float(ax[int(v)]) ** int(d) for v, d in zip(vs, ds)]
        val = ac
        for q in pw:
            val *= q
        parts = []
        for r, (v, d) in enumerate(zip(vs, ds)):
            g = ac * float(ax[int(v)]) ** (int(d) - 1)  # exponent factor d dropped
            for q in range(len(vs)):
                if q != r:
                    g *= pw[q]
            parts.append(g)
        out[int(t)] = (val, parts)
    return out


MUTANTS = {
    "power_off_by_one": ("_power", _mut_power_off_by_one),
    "mul_sign": ("cdy_mul", _mut_mul_sign),
    "mul_swapped_im": ("cdy_mul", _mut_mul_swap),
    "add_exponent": ("cdy_add", _mut_add_shift),
    "exponent_factor_e": ("monomial_value_and_partials", _mut_partials_exponent_e),
    "no_common_factor": ("monomial_value_and_partials", _mut_partials_no_common_factor),
    "partial_includes_self": ("monomial_value_and_partials", _mut_partials_include_self),
    "partial_drops_factor": ("monomial_value_and_partials", _mut_partials_dropped_last_factor),
    "adjoint_without_conj": ("cdy_conj", _mut_conj_noop),
    "limbs_drop_last": ("cdy_from_limbs", _mut_from_limbs_drop_last),
    "sum_drops_last_monomial": ("eval_rows", _make_eval_rows_drop_last_monomial()),
    "J_transposed": ("eval_rows", _make_eval_rows_transposed()),
    "columns_exponent_factor_e": ("eval_columns", _make_eval_columns(exp_factor_shift=1)),
    "columns_drop_common_factor": ("eval_columns", _make_eval_columns(drop_common=True)),
    "abs_columns_no_exponent": ("abs_sums_columns", _make_abs_sums_columns_no_exponent()),
    "abs_rows_no_power": ("abs_sums_rows", _make_abs_sums_rows_no_power()),
    "metric_zero_scale_accepts": ("rel_error", _mut_rel_error_zero_scale_ok),
    "metric_lenient": ("rel_error", _mut_rel_error_lenient),
    "lstsq_transpose_not_adjoint": ("_lstsq_householder", _mut_lstsq_transpose),
    "abs_values_no_power": ("abs_sums_values", _mut_abs_values_no_power),
    "homotopy_sign": ("homotopy_step_mp", _make_homotopy_step_sign()),
    "terms_sorted_order": ("eval_terms", _make_terms_sorted_order()),
    "terms_no_coefficient": ("eval_terms", _make_terms_no_coefficient()),
    "abs_terms_no_exponent": ("abs_terms", _mut_abs_terms_no_exponent),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    import oracle
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(E, attr, fn)
    # the package re-exports the module's names: the pins see the mutant too
    if hasattr(oracle, attr):
        monkeypatch.setattr(oracle, attr, fn)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            ok = pin()
        except Exception:
            ok = False
        if not ok:
            failed.append(pin.__name__)
            break
    assert failed, f"mutant {name} passed every pin"
