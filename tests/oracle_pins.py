"""Checks that pin the CPU oracle to facts outside itself.

Each ``pin_*`` function returns True when the oracle agrees with a closed form,
an identity of the mathematics, or a library routine on a special case.  The
pins are collected in ``ALL_PINS`` so that the mutation test can plant a
mistake in the oracle and check that some pin fails.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as O
from paper_1402_2626_amd import synth


def _exact_regime_value(re: int, im: int, a: int):
    """(re + i im) * 2^a as an exact complex dyadic, and as a Python complex."""
    return (re, im, a), complex(math.ldexp(re, a), math.ldexp(im, a))


# ---------------------------------------------------------------- Speelpenning

def pin_speelpenning_closed_form() -> bool:
    """(1+i)^k and its gradient (1+i)^(k-1) in every slot, written in closed
    form: (1+i)^2 = 2i, so (1+i)^(2m) = (2i)^m.  Section 2.2."""
    one_plus_i = (1, 1, 0)
    for k in (1, 2, 3, 4, 8, 9, 16):
        v, g = O.speelpenning_straightforward([one_plus_i] * k)
        want_v = (2j) ** (k // 2) * ((1 + 1j) if k % 2 else 1)
        want_g = (2j) ** ((k - 1) // 2) * ((1 + 1j) if (k - 1) % 2 else 1)
        if O.cdy_to_complex(v) != want_v:
            return False
        if any(O.cdy_to_complex(gi) != want_g for gi in g):
            return False
    return True


def pin_speelpenning_figures() -> bool:
    """The circuits of Fig. 1 (n = 4) and Fig. 2 (n = 8) compute the product and
    every partial derivative; with distinct primes as inputs each partial is
    the product divided by its own variable (integer division, exact)."""
    for primes in ((2, 3, 5, 7), (2, 3, 5, 7, 11, 13, 17, 19)):
        xs = [(p, 0, 0) for p in primes]
        v, g = O.speelpenning_straightforward(xs)
        P = math.prod(primes)
        if O.cdy_to_complex(v) != P:
            return False
        if [O.cdy_to_complex(gi) for gi in g] != [P // p for p in primes]:
            return False
    return True


def pin_speelpenning_euler() -> bool:
    """For a product of distinct variables, x_i * dP/dx_i = P for every i:
    checked exactly at a random unit-circle quad-double point."""
    rng = synth.rng_for(11)
    for k in (1, 2, 5, 16):
        x = synth.unit_circle(rng, k, 4)
        xs = O.point_from_limbs(x)
        v, g = O.speelpenning_straightforward(xs)
        for xi, gi in zip(xs, g):
            d = O.cdy_add(O.cdy_mul(xi, gi), O.cdy_neg(v))
            if not O.cdy_is_zero(d):
                return False
    return True


# ---------------------------------------------------------------- linear systems

def _linear_case(seed=3, N=7, n=5, L=2):
    rng = synth.rng_for(seed)
    C = rng.integers(-4, 5, size=(N, n)) + 1j * rng.integers(-4, 5, size=(N, n))
    polys = []
    for p in range(N):
        polys.append([(C[p, j], [(j, 1)]) for j in range(n) if C[p, j] != 0])
    sys_ = synth.from_monomial_lists(L, n, polys)
    xs = synth.exact_regime_points(seed + 1, 1, n, L)[0]
    xc = xs[0, 0] + 1j * xs[1, 0]
    return sys_, xs, C, xc


def pin_linear_system() -> bool:
    """F = C x and J = C for a linear system (k = 1, d = 1), against numpy's
    matrix-vector product on exactly representable data (non-square,
    non-symmetric C, so a transposed index fails)."""
    sys_, xs, C, xc = _linear_case()
    F, J = O.eval_system(sys_, xs)
    Fn = C @ xc
    for p in range(C.shape[0]):
        if O.cdy_to_complex(F[p]) != Fn[p]:
            return False
        for j in range(C.shape[1]):
            got = O.cdy_to_complex(J[p].get(j, O.ZERO))
            if got != C[p, j]:
                return False
    return True


def pin_linear_adjoint() -> bool:
    """J^H v = C^H v for a linear system, against numpy (exact data)."""
    sys_, xs, C, xc = _linear_case(seed=5)
    v = synth.exact_regime_points(9, 1, C.shape[0], sys_.level)[0]
    vc = v[0, 0] + 1j * v[1, 0]
    F, J = O.eval_system(sys_, xs)
    g = O.adjoint_exact(J, O.point_from_limbs(v), sys_.n_vars)
    want = C.conj().T @ vc
    if [O.cdy_to_complex(gi) for gi in g] != list(want):
        return False
    cols = O.adjoint_columns(sys_, xs, v, range(sys_.n_vars))
    return [O.cdy_to_complex(cols[j]) for j in range(sys_.n_vars)] == list(want)


# ---------------------------------------------------------------- univariate

def pin_univariate() -> bool:
    """One variable: F = sum_d c_d x^d and J = sum_d d c_d x^(d-1), against
    numpy.polynomial's polyval/polyder on exactly representable data."""
    from numpy.polynomial import polynomial as npoly
    rng = synth.rng_for(21)
    for trial in range(6):
        deg = int(rng.integers(1, 9))
        coeffs = rng.integers(-5, 6, size=deg + 1) + 1j * rng.integers(-5, 6, size=deg + 1)
        mons = [(coeffs[d], [(0, d)] if d else []) for d in range(deg + 1) if coeffs[d] != 0]
        sys_ = synth.from_monomial_lists(2, 1, [mons])
        x = synth.exact_regime_points(30 + trial, 1, 1, 2)[0]
        xc = complex(x[0, 0, 0], x[1, 0, 0])
        F, J = O.eval_system(sys_, x)
        if O.cdy_to_complex(F[0]) != npoly.polyval(xc, coeffs):
            return False
        if O.cdy_to_complex(J[0].get(0, O.ZERO)) != npoly.polyval(xc, npoly.polyder(coeffs)):
            return False
    return True


def pin_univariate_mpmath() -> bool:
    """One variable at a full quad-double point: mpmath's polyval (with the
    derivative) at 600 bits agrees with the exact oracle to 2^-500."""
    import mpmath
    rng = synth.rng_for(22)
    deg = 7
    coef = synth.unit_circle(rng, deg + 1, 4)
    mons = [(0, [(0, d)] if d else []) for d in range(deg + 1)]
    sys_ = synth.from_monomial_lists(4, 1, [mons], coef_limbs=coef)
    x = synth.unit_circle(rng, 1, 4)
    F, J = O.eval_system(sys_, x)
    with mpmath.workprec(600):
        cs = [mpmath.mpc(sum(mpmath.mpf(float(a)) for a in coef[0, :, d]),
                         sum(mpmath.mpf(float(a)) for a in coef[1, :, d])) for d in range(deg + 1)]
        xm = mpmath.mpc(sum(mpmath.mpf(float(a)) for a in x[0, :, 0]),
                        sum(mpmath.mpf(float(a)) for a in x[1, :, 0]))
        val, der = mpmath.polyval(cs[::-1], xm, derivative=True)
        def close(a, b):
            return abs(mpmath.mpc(mpmath.ldexp(a[0], a[2]), mpmath.ldexp(a[1], a[2])) - b) < mpmath.mpf(2) ** -500
        return close(F[0], val) and close(J[0][0], der)


# ---------------------------------------------------------------- quadratic form

def pin_quadratic_form() -> bool:
    """F = x^T A x (monomials x_i x_j, i < j, with coefficient A_ij + A_ji and
    x_i^2 with A_ii) has J = x^T (A + A^T); against numpy on exact data."""
    rng = synth.rng_for(31)
    n = 6
    A = rng.integers(-3, 4, size=(n, n)) + 1j * rng.integers(-3, 4, size=(n, n))
    mons = []
    for i in range(n):
        if A[i, i] != 0:
            mons.append((A[i, i], [(i, 2)]))
        for j in range(i + 1, n):
            c = A[i, j] + A[j, i]
            if c != 0:
                mons.append((c, [(i, 1), (j, 1)]))
    sys_ = synth.from_monomial_lists(1, n, [mons])
    x = synth.exact_regime_points(32, 1, n, 1)[0]
    xc = x[0, 0] + 1j * x[1, 0]
    F, J = O.eval_system(sys_, x)
    if O.cdy_to_complex(F[0]) != xc @ A @ xc:
        return False
    want = xc @ (A + A.T)
    return all(O.cdy_to_complex(J[0].get(j, O.ZERO)) == want[j] for j in range(n))


# ---------------------------------------------------------------- finite differences

def pin_finite_differences() -> bool:
    """Central differences of the exact F with step h = 2^-80 along the real
    and the imaginary axis of every variable match J to O(h^2); F is a
    polynomial so the difference quotient is computed exactly."""
    sys_ = synth.random_system(41, 4, n_vars=5, n_polys=3, m=4, k=3, exp_lo=1, exp_hi=4)
    x = synth.unit_circle_points(synth.rng_for(42), 1, 5, 4)[0]
    X = O.point_from_limbs(x)
    F, J = O.eval_system(sys_, x)
    h_exp = -80
    for j in range(sys_.n_vars):
        for direction in ((1, 0, h_exp), (0, 1, h_exp)):
            Xp = list(X)
            Xm = list(X)
            Xp[j] = O.cdy_add(X[j], direction)
            Xm[j] = O.cdy_add(X[j], O.cdy_neg(direction))
            Fp = O.system_value_at(sys_, Xp)
            Fm = O.system_value_at(sys_, Xm)
            for p in range(sys_.n_polys):
                diff = O.cdy_add(Fp[p], O.cdy_neg(Fm[p]))
                # divide by 2h (times i for the imaginary step): exact
                if direction[1]:
                    diff = (diff[1], -diff[0], diff[2])
                fd = (diff[0], diff[1], diff[2] - h_exp - 1)
                err = O.cdy_abs_float(O.cdy_add(fd, O.cdy_neg(J[p].get(j, O.ZERO))))
                if err > 1e-40:  # h^2 = 2^-160 ~ 7e-49 times moderate derivatives
                    return False
    return True


# ---------------------------------------------------------------- homogeneity

def _homogeneous_system(seed, L, n, N, m, D):
    """Every monomial of polynomial p has total degree D (no constants)."""
    rng = synth.rng_for(seed)
    polys = []
    for p in range(N):
        mons = []
        for t in range(m):
            k = int(rng.integers(1, min(n, D) + 1))
            vs = np.sort(rng.choice(n, size=k, replace=False))
            ds = np.ones(k, dtype=int)
            for _ in range(D - k):
                ds[int(rng.integers(0, k))] += 1
            mons.append((0, [(int(v), int(d)) for v, d in zip(vs, ds)]))
        polys.append(mons)
    M = N * m
    coef = synth.unit_circle(rng, M, L)
    return synth.from_monomial_lists(L, n, polys, coef_limbs=coef)


def pin_euler_homogeneity() -> bool:
    """Euler's identity for a homogeneous polynomial of degree D:
    sum_j x_j J_pj = D F_p, checked exactly."""
    D = 5
    sys_ = _homogeneous_system(51, 2, n=6, N=3, m=5, D=D)
    x = synth.unit_circle_points(synth.rng_for(52), 1, 6, 2)[0]
    X = O.point_from_limbs(x)
    F, J = O.eval_system(sys_, x)
    for p in range(sys_.n_polys):
        acc = O.ZERO
        for j, v in J[p].items():
            acc = O.cdy_add(acc, O.cdy_mul(X[j], v))
        if not O.cdy_is_zero(O.cdy_add(acc, O.cdy_neg(O.cdy_scale(F[p], D)))):
            return False
    return True


# ---------------------------------------------------------------- cyclic n-roots

def pin_cyclic_at_one() -> bool:
    """Cyclic n-roots (eq. (5)) at x = 1: F_i = n for the first n-1 equations
    and 0 for the last; J_{i,m} = i (1-based i) and the last row is all ones."""
    for n in (3, 4, 7):
        sys_ = synth.cyclic_roots_system(n, 1)
        if sys_.n_monomials != n * n - n + 2:
            return False
        x = np.zeros((2, 1, n))
        x[0, 0] = 1.0
        F, J = O.eval_system(sys_, x)
        for i in range(n - 1):
            if O.cdy_to_complex(F[i]) != n:
                return False
            if any(O.cdy_to_complex(J[i].get(j, O.ZERO)) != i + 1 for j in range(n)):
                return False
        if O.cdy_to_complex(F[n - 1]) != 0:
            return False
        if any(O.cdy_to_complex(J[n - 1].get(j, O.ZERO)) != 1 for j in range(n)):
            return False
    return True


def pin_cyclic_at_roots_of_unity() -> bool:
    """At x_j = w^j (w = e^{2 pi i/n}) the first n-1 equations vanish and the
    last equals (-1)^(n-1) - 1; with x rounded to double double the oracle
    must agree to 1e-28."""
    import mpmath
    for n in (5, 8):
        sys_ = synth.cyclic_roots_system(n, 2)
        x = np.zeros((2, 2, n))
        with mpmath.workprec(300):
            for j in range(n):
                z = mpmath.expjpi(mpmath.mpf(2 * j) / n)
                for part, val in ((0, z.real), (1, z.imag)):
                    hi = float(val)
                    lo = float(val - hi)
                    x[part, 0, j], x[part, 1, j] = hi, lo
        F, _ = O.eval_system(sys_, x, want_J=False)
        for i in range(n - 1):
            if O.cdy_abs_float(F[i]) > 1e-28 * n:
                return False
        want = (-1) ** (n - 1) - 1
        if abs(O.cdy_to_complex(F[n - 1]) - want) > 1e-28 * n:
            return False
    return True


# ---------------------------------------------------------------- limbs and metric

def pin_limb_rounding() -> bool:
    """Rounding exact values to limbs: known expansions, round-to-even ties,
    and agreement with mpmath's own rounding to double of 1/3 and of the
    remainders at 400 bits."""
    import mpmath
    v = O.cdy_add(O.cdy_add((1, 0, 0), (1, 0, -60)), O.cdy_add((1, 0, -120), (1, 0, -180)))
    if list(O.cdy_to_limbs(v, 4)[0]) != [1.0, 2.0 ** -60, 2.0 ** -120, 2.0 ** -180]:
        return False
    tie = O.cdy_add((1, 0, 0), (1, 0, -53))  # halfway between 1 and 1 + 2^-52
    if list(O.cdy_to_limbs(tie, 2)[0]) != [1.0, 2.0 ** -53]:
        return False
    third = ((1 << 400) // 3, 0, -400)
    limbs = O.cdy_to_limbs(third, 4)[0]
    with mpmath.workprec(400):
        r = mpmath.ldexp(third[0], -400)
        for l in range(4):
            f = float(r)  # mpmath rounds to nearest
            if f != limbs[l]:
                return False
            r -= f
    return True


def pin_abs_sums() -> bool:
    """With unit-modulus coefficients and point entries in the exact regime
    (|x| = 1 when a = 0), S_F(p) = number of monomials and S_J(p, j) = sum of
    the exponents of x_j over polynomial p."""
    sys_ = synth.random_system(61, 2, n_vars=6, n_polys=3, m=4, k=3, exp_lo=1, exp_hi=4)
    sys_.coef[:] = 0.0
    sys_.coef[0, 0] = 1.0
    x = np.zeros((2, 2, 6))
    x[1, 0] = 1.0  # x_j = i
    SF, SJ = O.abs_sums_rows(sys_, x, range(3))
    for p in range(3):
        if SF[p] != 4.0:
            return False
        want = {}
        for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
            vs, ds = sys_.monomial(t)
            for v, d in zip(vs, ds):
                want[int(v)] = want.get(int(v), 0) + int(d)
        if {j: int(s) for j, s in SJ[p].items()} != want:
            return False
    return True


# ---------------------------------------------------------------- Gauss-Newton

def pin_gauss_newton_linear() -> bool:
    """For F = C x - b (overdetermined, inconsistent, with zeros on the
    diagonal of C), one Gauss-Newton step from any point lands on the
    least-squares solution; against numpy.linalg.lstsq."""
    rng = synth.rng_for(71)
    for N, n in ((6, 3), (9, 9), (12, 5)):
        C = rng.integers(-4, 5, size=(N, n)) + 1j * rng.integers(-4, 5, size=(N, n))
        for i in range(min(N, n)):
            C[i, i] = 0
        b = rng.integers(-4, 5, size=N) + 1j * rng.integers(-4, 5, size=N)
        polys = [[(C[p, j], [(j, 1)]) for j in range(n) if C[p, j] != 0] + [(-b[p], [])] for p in range(N)]
        sys_ = synth.from_monomial_lists(2, n, polys)
        X0 = [(1, 0, 0)] * n
        X1, _ = O.gauss_newton_step_mp(sys_, X0, prec=256)
        want = np.linalg.lstsq(C, b, rcond=None)[0]
        got = np.array([O.cdy_to_complex(v) for v in X1])
        if not np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want))):
            return False
    return True


def pin_lstsq_limbs() -> bool:
    """The least-squares solve on its own: exactly representable
    overdetermined, inconsistent complex data (with zeros on the diagonal)
    against numpy.linalg.lstsq, and a consistent system whose solution is
    known exactly."""
    import oracle.exact as OE
    rng = synth.rng_for(431)
    for N, n in ((7, 4), (12, 12), (15, 6)):
        C = rng.integers(-4, 5, size=(N, n)) + 1j * rng.integers(-4, 5, size=(N, n))
        for i in range(min(N, n)):
            C[i, i] = 0
        b = rng.integers(-4, 5, size=N) + 1j * rng.integers(-4, 5, size=N)
        Ab = np.zeros((2, 2, N, n + 1))
        Ab[0, 0, :, :n], Ab[1, 0, :, :n] = C.real, C.imag
        Ab[0, 0, :, n], Ab[1, 0, :, n] = b.real, b.imag
        x = np.array([OE.cdy_to_complex(v) for v in OE.lstsq_limbs(Ab, prec=256)])
        want = np.linalg.lstsq(C, b, rcond=None)[0]
        if not np.max(np.abs(x - want)) < 1e-12 * max(1.0, np.max(np.abs(want))):
            return False
    # consistent: b = C x* with x* Gaussian integers, solution exact to 2^-380
    C = rng.integers(-4, 5, size=(9, 5)) + 1j * rng.integers(-4, 5, size=(9, 5))
    xs = rng.integers(-3, 4, size=5) + 1j * rng.integers(-3, 4, size=5)
    b = C @ xs
    Ab = np.zeros((2, 1, 9, 6))
    Ab[0, 0, :, :5], Ab[1, 0, :, :5] = C.real, C.imag
    Ab[0, 0, :, 5], Ab[1, 0, :, 5] = b.real, b.imag
    x = OE.lstsq_limbs(Ab, prec=400)
    return all(OE.cdy_abs_float(OE.cdy_add(x[j], OE.cdy_neg((int(xs[j].real), int(xs[j].imag), 0)))) < 2.0 ** -380
               for j in range(5))


def pin_homotopy_square_root() -> bool:
    """f(x) = x^2 - 4 from z = 3 (c = f(z) = 5): the path of x^2 - 4 - 5t = 0
    is x(t) = sqrt(4 + 5t), so tracking to t = 0 ends at the root 2; a single
    corrector at t = 1/2 from x(1/2) + 1e-3 lands on sqrt(6.5) quadratically."""
    import mpmath
    import oracle.exact as OE
    sys_ = synth.from_monomial_lists(2, 1, [[(1.0, [(0, 2)]), (-4.0, [])]])
    end = OE.homotopy_track_mp(sys_, [(3, 0, 0)], [(5, 0, 0)], steps=8, corrector_iters=6, prec=400)
    if OE.cdy_abs_float(OE.cdy_add(end[0], (-2, 0, 0))) > 1e-100:
        return False
    with mpmath.workprec(400):
        xh = mpmath.sqrt(mpmath.mpf(6.5))
        start = OE._mpc_to_cdy(mpmath.mpc(xh + mpmath.mpf(2) ** -10))
        X = OE.homotopy_step_mp(sys_, [start], [(5, 0, 0)], 1.0, 0.5, prec=400)
        err = abs(mpmath.ldexp(X[0][0], X[0][2]) - xh)
        return 1e-9 < err < 1e-5  # one Newton step: (2^-10)^2 / (2 x) ~ 2e-7


def pin_homotopy_decoupled_squares() -> bool:
    """Decoupled squares x_j^2 - a_j (complex a_j, random start z): each
    path is x_j(t)^2 = a_j + t (z_j^2 - a_j), whose continuous branch from z_j
    is followed here by 4000 small steps of mpmath's square root with the
    sign kept continuous; the tracker's end point matches it."""
    import mpmath
    import oracle.exact as OE
    rng = synth.rng_for(441)
    n = 3
    a = rng.integers(-4, 5, size=n) + 1j * rng.integers(1, 5, size=n)
    z = rng.integers(-3, 4, size=n) + 1j * rng.integers(-3, 4, size=n) + 0.5
    polys = [[(1.0, [(j, 2)]), (-a[j], [])] for j in range(n)]
    sys_ = synth.from_monomial_lists(2, n, polys)
    Z = [OE._mpc_to_cdy(mpmath.mpc(complex(v))) for v in z]
    c = [OE.cdy_add(OE.cdy_mul(Zj, Zj), OE._mpc_to_cdy(mpmath.mpc(-complex(a[j])))) for j, Zj in enumerate(Z)]
    end = OE.homotopy_track_mp(sys_, Z, c, steps=16, corrector_iters=6, prec=300)
    with mpmath.workprec(200):
        for j in range(n):
            x = mpmath.mpc(complex(z[j]))
            w0 = mpmath.mpc(complex(a[j]))
            w1 = mpmath.mpc(complex(z[j])) ** 2 - w0
            for k in range(1, 4001):
                r = mpmath.sqrt(w0 + (1 - mpmath.mpf(k) / 4000) * w1)
                x = r if abs(r - x) < abs(r + x) else -r
            got = mpmath.mpc(mpmath.ldexp(end[j][0], end[j][2]), mpmath.ldexp(end[j][1], end[j][2]))
            if abs(got - x) > mpmath.mpf(10) ** -50:
                return False
    return True


def pin_gauss_newton_quadratic() -> bool:
    """Planted root of a square random system (constant -F_p(x*) rounded to
    quad double appended to each polynomial): from x* + 1e-3 noise the
    distance to x* decays quadratically down to the rounding floor."""
    sys_ = synth.random_system(81, 4, n_vars=4, n_polys=4, m=4, k=2, exp_lo=1, exp_hi=2)
    xs = synth.unit_circle_points(synth.rng_for(82), 1, 4, 4)[0]
    planted = O.plant_root(sys_, xs)
    Xs = O.point_from_limbs(xs)
    X = O.point_from_limbs(synth.perturbed_start(83, xs, 1e-3))
    errs = []
    for _ in range(6):
        X, _ = O.gauss_newton_step_mp(planted, X, prec=512)
        errs.append(max(O.cdy_abs_float(O.cdy_add(X[j], O.cdy_neg(Xs[j]))) for j in range(4)))
    for a, b in zip(errs, errs[1:]):
        if a > 1e-55 and b > 1e3 * a * a:
            return False
    return errs[-1] < 1e-58


# ---------------------------------------------------------------- columns and normalisers

def pin_columns_match_rows() -> bool:
    """The column-wise evaluation (used for sampled columns and the adjoint)
    equals the row-wise one, transposed, exactly: random systems with
    exponents up to 4 at every level; and the adjoint by columns equals
    sum_p conj(J_pj) v_p over the row-wise J."""
    import oracle.exact as OE
    for L, seed in ((1, 401), (2, 402), (4, 403)):
        sys_ = synth.random_system(seed, L, n_vars=9, n_polys=6, m=5, k=4, exp_lo=1, exp_hi=4)
        x = synth.unit_circle_points(synth.rng_for(seed + 10), 1, 9, L)[0]
        _, J = OE.eval_rows(sys_, x, range(6))
        cols = OE.eval_columns(sys_, x, range(9))
        for j in range(9):
            want = {p: J[p][j] for p in range(6) if j in J[p]}
            if set(cols[j]) != set(want):
                return False
            for p, val in want.items():
                if not OE.cdy_is_zero(OE.cdy_add(cols[j][p], OE.cdy_neg(val))):
                    return False
        v = synth.unit_circle_points(synth.rng_for(seed + 20), 1, 6, L)[0]
        g = OE.adjoint_exact(J, OE.point_from_limbs(v), 9)
        gc = OE.adjoint_columns(sys_, x, v, range(9))
        if any(not OE.cdy_is_zero(OE.cdy_add(gc[j], OE.cdy_neg(g[j]))) for j in range(9)):
            return False
    return True


def pin_abs_sums_positive() -> bool:
    """When every coefficient and every variable is a positive real, all
    terms of F_p and of J_pj are positive, so the sum of their absolute
    values equals the absolute value of the exact sum: S_F(p) = |F_p| and
    S_J(p, j) = |J_pj|, by rows and by columns (moduli 2^a, a in -2..2, and
    small integer coefficients, so the float sums are exact)."""
    import oracle.exact as OE
    rng = synth.rng_for(411)
    sys_ = synth.random_system(412, 2, n_vars=7, n_polys=5, m=6, k=3, exp_lo=1, exp_hi=4)
    sys_.coef[:] = 0.0
    sys_.coef[0, 0] = rng.integers(1, 6, size=sys_.n_monomials)
    x = np.zeros((2, 2, 7))
    x[0, 0] = np.ldexp(1.0, rng.integers(-2, 3, size=7))
    F, J = OE.eval_rows(sys_, x, range(5))
    SF, SJ = OE.abs_sums_rows(sys_, x, range(5))
    Sc = OE.abs_sums_columns(sys_, x, range(7))
    Sv = OE.abs_sums_values(sys_, x, range(5))
    for p in range(5):
        if SF[p] != OE.cdy_abs_float(F[p]) or Sv[p] != SF[p]:
            return False
        if set(SJ[p]) != set(J[p]):
            return False
        for j, val in J[p].items():
            if SJ[p][j] != OE.cdy_abs_float(val) or Sc[j].get(p) != SJ[p][j]:
                return False
    return all(set(Sc[j]) == {p for p in range(5) if j in J[p]} for j in range(7))


def pin_error_metric_rejects() -> bool:
    """The checker itself: the exact value rounded to limbs scores at most
    the rounding error; an entry moved by 10 tau S fails a tolerance tau and
    one moved by tau S / 10 passes; a nonzero entry where S = 0 scores inf;
    a wrong entry planted in a whole F/J comparison, or two columns of J
    swapped, are found."""
    import oracle.exact as OE
    tau = 1e-28
    L = 2
    sys_ = synth.random_system(421, L, n_vars=6, n_polys=4, m=5, k=3, exp_lo=1, exp_hi=3)
    x = synth.unit_circle_points(synth.rng_for(422), 1, 6, L)[0]
    F, J = OE.eval_rows(sys_, x, range(4))
    SF, SJ = OE.abs_sums_rows(sys_, x, range(4))
    Fl = np.stack([OE.cdy_to_limbs(F[p], L) for p in range(4)], axis=-1)
    Jl = np.zeros((2, L, 4, 6))
    for p in range(4):
        for j, v in J[p].items():
            Jl[:, :, p, j] = OE.cdy_to_limbs(v, L)
    eF, eJ = OE.max_rel_error_rows(sys_, x, Fl, Jl, range(4))
    if not (eF <= 2.0 ** -104 and eJ <= 2.0 ** -104):
        return False
    p = 2
    for scale, must_fail in ((10.0, True), (0.1, False)):
        # move the real part by scale * tau * S_F(p), exactly (dyadic shift)
        m, e = OE.dy_from_float(scale * tau * SF[p])
        moved = OE.cdy_add(F[p], (m, 0, e))
        lim = OE.cdy_to_limbs(moved, L)
        err = OE.rel_error(lim[0], lim[1], F[p], SF[p])
        if (err > tau) != must_fail:
            return False
    if OE.rel_error([1e-300, 0.0], [0.0, 0.0], OE.ZERO, 0.0) != math.inf:
        return False
    if OE.rel_error([0.0, 0.0], [0.0, 0.0], OE.ZERO, 0.0) != 0.0:
        return False
    bad = Jl.copy()
    j = next(iter(J[1]))
    bad[0, 1, 1, j] += 1e-20 * SJ[1][j]
    if OE.max_rel_error_rows(sys_, x, Fl, bad, range(4))[1] <= tau:
        return False
    cols = sorted(J[3])
    swapped = Jl.copy()
    swapped[:, :, 3, [cols[0], cols[1]]] = Jl[:, :, 3, [cols[1], cols[0]]]
    return OE.max_rel_error_rows(sys_, x, Fl, swapped, range(4))[1] > tau


# ---------------------------------------------------------------- terms

def pin_terms_closed_form() -> bool:
    """Terms in the input order (Sec. 2.2 Tables 1-2 output, Sec. 2.3 factors):
    the monomial 3 x_3^2 x_0 x_1^3 written with its variables out of order, at
    x = (2, 5, 0, -1): value 3 * 1 * 2 * 125 = 750 and the partials in the
    input order d/dx_3 = 3 * 2 x_3 x_0 x_1^3 = -1500, d/dx_0 = 3 x_3^2 x_1^3 =
    375, d/dx_1 = 3 * 3 x_3^2 x_0 x_1^2 = 450; a constant term has no
    partial; complex data: (2i) x_2 at x_2 = 1 + i gives -2 + 2i and 2i."""
    sys_ = synth.from_monomial_lists(1, 4, [[(3.0, [(3, 2), (0, 1), (1, 3)]), (7.0, [])],
                                             [(2j, [(2, 1)])]])
    x = np.zeros((2, 1, 4))
    x[0, 0] = [2.0, 5.0, 1.0, -1.0]
    x[1, 0, 2] = 1.0
    T = O.eval_terms(sys_, x, range(3))
    v0, g0 = T[0]
    if O.cdy_to_complex(v0) != 750 or [O.cdy_to_complex(g) for g in g0] != [-1500, 375, 450]:
        return False
    v1, g1 = T[1]
    if O.cdy_to_complex(v1) != 7 or g1 != []:
        return False
    v2, g2 = T[2]
    return O.cdy_to_complex(v2) == -2 + 2j and [O.cdy_to_complex(g) for g in g2] == [2j]


def pin_terms_euler() -> bool:
    """Euler's identity per term: sum_r x_{i_r} dT/dx_{i_r} = (sum_r d_r) T,
    exactly, for every monomial of a random double-double system with
    exponents up to 4 and variables in shuffled input order."""
    rng = synth.rng_for(71)
    sys_ = synth.random_system(72, 2, n_vars=9, n_polys=4, m=5, k=4, exp_lo=1, exp_hi=4)
    perm = np.concatenate([rng.permutation(np.arange(a, b)) for a, b in zip(sys_.mon_ptr[:-1], sys_.mon_ptr[1:])])
    sys_.var_idx = sys_.var_idx[perm]
    sys_.exps = sys_.exps[perm]
    x = synth.unit_circle_points(synth.rng_for(73), 1, 9, 2)[0]
    X = O.point_from_limbs(x)
    T = O.eval_terms(sys_, x, range(sys_.n_monomials))
    for t, (v, g) in T.items():
        vs, ds = sys_.monomial(t)
        acc = O.ZERO
        for r, j in enumerate(vs):
            acc = O.cdy_add(acc, O.cdy_mul(X[int(j)], g[r]))
        if not O.cdy_is_zero(O.cdy_add(acc, O.cdy_neg(O.cdy_scale(v, int(sum(int(d) for d in ds)))))):
            return False
    return True


def pin_terms_abs() -> bool:
    """The terms' normalisers equal the moduli of the terms when every
    coefficient and every variable is positive (then |term| = term)."""
    sys_ = synth.random_system(74, 1, n_vars=6, n_polys=3, m=4, k=3, exp_lo=1, exp_hi=3)
    c = np.zeros_like(sys_.coef)
    c[0, 0] = np.linspace(0.25, 2.0, sys_.n_monomials)
    sys_.coef = c
    x = np.zeros((2, 1, 6))
    x[0, 0] = [0.5, 1.25, 2.0, 0.75, 1.5, 1.0]
    T = O.eval_terms(sys_, x, range(sys_.n_monomials))
    A = O.abs_terms(sys_, x, range(sys_.n_monomials))
    for t, (v, g) in T.items():
        sv, sg = A[t]
        if abs(O.cdy_to_complex(v).real - sv) > 1e-12 * sv:
            return False
        if any(abs(O.cdy_to_complex(gi).real - s) > 1e-12 * s for gi, s in zip(g, sg)):
            return False
    return True


ALL_PINS = [
    pin_speelpenning_closed_form, pin_speelpenning_figures, pin_speelpenning_euler,
    pin_linear_system, pin_linear_adjoint, pin_univariate, pin_univariate_mpmath,
    pin_quadratic_form, pin_finite_differences, pin_euler_homogeneity,
    pin_cyclic_at_one, pin_cyclic_at_roots_of_unity, pin_limb_rounding, pin_abs_sums,
    pin_gauss_newton_linear, pin_gauss_newton_quadratic, pin_columns_match_rows,
    pin_abs_sums_positive, pin_error_metric_rejects, pin_lstsq_limbs, pin_homotopy_square_root,
    pin_homotopy_decoupled_squares,
    pin_terms_closed_form,
    pin_terms_euler,
    pin_terms_abs,
]
