"""Seeded synthetic inputs: sparse polynomial systems and evaluation points.

This module only draws random structure and random numbers.  It holds none of
the evaluation arithmetic, so both the HIP path and the CPU oracle may use it.

A system is in sparse distributed form (Problem Statement, Section 1): every
polynomial is fully expanded and only monomials with a nonzero coefficient are
stored.  Each monomial is a coefficient plus the list of its variables with
positive exponents, the variables sorted and distinct (Section 2.1, eq. (1)).

Layout conventions shared by the library and the tests:

* ``poly_ptr`` (int64, N+1): monomials of polynomial p are
  ``mon_ptr[poly_ptr[p]] .. poly_ptr[p+1]``.
* ``mon_ptr`` (int64, M+1): occurrences of monomial t are
  ``var_idx[mon_ptr[t]:mon_ptr[t+1]]`` with exponents ``exps[...]``.
* Complex level-L numbers are limb-planar ``[2 (re, im)][L][count]`` float64,
  limbs most significant first, forming a nonoverlapping expansion.
  L = 1 (double), 2 (double double) or 4 (quad double).

Unit-circle numbers at level L: the leading limbs are ``cos t, sin t`` in double
for t ~ U[0, 2 pi); every lower limb is drawn uniformly in (-1/2, 1/2) ulp of
the limb above it, so all limbs are populated and the expansion is
nonoverlapping.  The modulus is 1 to within 2^-53.
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

import numpy as np

LEVELS = (1, 2, 4)


@dataclasses.dataclass
class PolySystem:
    """A sparse polynomial system in the library's input layout."""

    level: int
    n_vars: int
    poly_ptr: np.ndarray  # int64 [N+1]
    mon_ptr: np.ndarray  # int64 [M+1]
    var_idx: np.ndarray  # int32 [nnz]
    exps: np.ndarray  # int32 [nnz]
    coef: np.ndarray  # float64 [2, L, M]
    name: str = ""

    @property
    def n_polys(self) -> int:
        return int(self.poly_ptr.shape[0] - 1)

    @property
    def n_monomials(self) -> int:
        return int(self.mon_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.var_idx.shape[0])

    def monomial(self, t: int):
        a, b = int(self.mon_ptr[t]), int(self.mon_ptr[t + 1])
        return self.var_idx[a:b], self.exps[a:b]

    def degrees(self) -> np.ndarray:
        """Total degree of every monomial (int64 [M])."""
        d = np.zeros(self.n_monomials, dtype=np.int64)
        if self.nnz:
            owner = np.repeat(np.arange(self.n_monomials), np.diff(self.mon_ptr))
            np.add.at(d, owner, self.exps.astype(np.int64))
        return d

    def validate_layout(self) -> None:
        L = self.level
        assert L in LEVELS
        M = self.n_monomials
        assert self.coef.shape == (2, L, M), self.coef.shape
        assert self.poly_ptr[0] == 0 and self.poly_ptr[-1] == M
        assert self.mon_ptr[0] == 0 and self.mon_ptr[-1] == self.nnz
        assert np.all(np.diff(self.poly_ptr) >= 0)
        assert np.all(np.diff(self.mon_ptr) >= 0)


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------

def rng_for(seed: int | Sequence[int]) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def lower_limbs(rng: np.random.Generator, lead: np.ndarray, L: int) -> np.ndarray:
    """Return ``[L, ...]`` limbs whose leading limb is ``lead``.

    Every limb below is uniform in (-1/2, 1/2) ulp of the limb above, which
    keeps the expansion nonoverlapping.  The product of a double in (-1/2, 1/2)
    by a power of two is exact, so no rounding happens here."""
    out = np.empty((L,) + lead.shape, dtype=np.float64)
    out[0] = lead
    for l in range(1, L):
        a = np.abs(out[l - 1])
        # the gap below |limb| (half the gap above when |limb| is a power of 2)
        ulp = a - np.nextafter(a, 0.0)
        out[l] = rng.uniform(-0.5, 0.5, size=lead.shape) * ulp
        # a limb must stay strictly below half a gap of the limb above
        out[l] = np.where(np.abs(out[l]) * 2.0 >= ulp, 0.0, out[l])
    return out


def unit_circle(rng: np.random.Generator, count: int, L: int) -> np.ndarray:
    """``[2, L, count]`` level-L complex numbers of modulus 1 (to 2^-53)."""
    theta = rng.uniform(0.0, 2.0 * np.pi, size=count)
    re = lower_limbs(rng, np.cos(theta), L)
    im = lower_limbs(rng, np.sin(theta), L)
    return np.stack([re, im])


def unit_circle_points(rng: np.random.Generator, P: int, n: int, L: int) -> np.ndarray:
    """``[P, 2, L, n]`` evaluation points with unit-modulus entries."""
    return np.stack([unit_circle(rng, n, L) for _ in range(P)]) if P else np.zeros((0, 2, L, n))


def distinct_sorted_subsets(rng: np.random.Generator, count: int, n: int, k: int) -> np.ndarray:
    """``[count, k]`` int32: each row is a uniform k-subset of range(n), sorted.

    Rows are drawn as uniform k-tuples and redrawn while a tuple repeats an
    index; an accepted tuple is a uniform ordered selection without
    replacement, so its set is a uniform k-subset."""
    if k > n:
        raise ValueError("k > n")
    if k == 0 or count == 0:
        return np.zeros((count, k), dtype=np.int32)
    if 2 * k > n:
        out = np.empty((count, k), dtype=np.int32)
        step = max(1, (1 << 22) // n)
        for a in range(0, count, step):
            b = min(count, a + step)
            keys = rng.random((b - a, n))
            out[a:b] = np.sort(np.argpartition(keys, k - 1, axis=1)[:, :k], axis=1)
        return out
    rows = rng.integers(0, n, size=(count, k), dtype=np.int64)
    rows.sort(axis=1)
    bad = np.nonzero(np.any(rows[:, 1:] == rows[:, :-1], axis=1))[0] if k > 1 else np.zeros(0, np.int64)
    while bad.size:
        redo = rng.integers(0, n, size=(bad.size, k), dtype=np.int64)
        redo.sort(axis=1)
        rows[bad] = redo
        still = np.any(redo[:, 1:] == redo[:, :-1], axis=1)
        bad = bad[still]
    return rows.astype(np.int32)


# --------------------------------------------------------------------------
# system families
# --------------------------------------------------------------------------

def random_system(seed, level: int, n_vars: int, n_polys: int, m: int, k: int,
                  exp_lo: int = 1, exp_hi: int = 3, name: str = "") -> PolySystem:
    """n_polys polynomials with m monomials each; every monomial has k distinct
    variables drawn uniformly without replacement (sorted) and i.i.d. exponents
    uniform in [exp_lo, exp_hi]; unit-circle coefficients.

    Draw order: structure, exponents, coefficients (all from one stream)."""
    rng = rng_for(seed)
    M = n_polys * m
    vars_ = distinct_sorted_subsets(rng, M, n_vars, k)
    exps = rng.integers(exp_lo, exp_hi + 1, size=(M, k)).astype(np.int32)
    coef = unit_circle(rng, M, level)
    return PolySystem(
        level=level, n_vars=n_vars,
        poly_ptr=np.arange(0, M + 1, m, dtype=np.int64) if m else np.zeros(n_polys + 1, np.int64),
        mon_ptr=np.arange(0, M * k + 1, k, dtype=np.int64) if k else np.zeros(M + 1, np.int64),
        var_idx=vars_.reshape(-1), exps=exps.reshape(-1), coef=coef, name=name)


def from_monomial_lists(level: int, n_vars: int, polys, coef_limbs=None, name: str = "") -> PolySystem:
    """Build a system from ``polys[p] = [(coef, [(var, exp), ...]), ...]``.

    ``coef`` is a Python complex (rounded to double, lower limbs zero) unless
    ``coef_limbs`` ([2, L, M]) is given."""
    poly_ptr = [0]
    mon_ptr = [0]
    var_idx, exps, coefs = [], [], []
    for mons in polys:
        for c, occ in mons:
            for v, d in occ:
                var_idx.append(v)
                exps.append(d)
            mon_ptr.append(len(var_idx))
            coefs.append(complex(c))
        poly_ptr.append(len(mon_ptr) - 1)
    M = len(coefs)
    if coef_limbs is None:
        coef_limbs = np.zeros((2, level, M))
        coef_limbs[0, 0] = [c.real for c in coefs]
        coef_limbs[1, 0] = [c.imag for c in coefs]
    return PolySystem(level=level, n_vars=n_vars,
                      poly_ptr=np.asarray(poly_ptr, np.int64), mon_ptr=np.asarray(mon_ptr, np.int64),
                      var_idx=np.asarray(var_idx, np.int32), exps=np.asarray(exps, np.int32),
                      coef=np.asarray(coef_limbs, np.float64), name=name)


def cyclic_roots_system(n: int, level: int) -> PolySystem:
    """The cyclic n-roots system (eq. (5), Section 5.3): for i = 1..n-1 the sum
    over j of the products of i cyclically consecutive variables starting at
    x_j; the last polynomial is x_0 x_1 ... x_{n-1} - 1.  Coefficients are 1
    except the constant -1.  n^2 - n + 2 monomials in total; each monomial's
    variables in increasing order."""
    var_blocks, k_list = [], []
    for i in range(1, n):
        idx = np.sort((np.arange(n)[:, None] + np.arange(i)[None, :]) % n, axis=1)
        var_blocks.append(idx.reshape(-1))
        k_list.append(np.full(n, i, np.int64))
    var_blocks.append(np.arange(n))
    k_list.append(np.array([n, 0], np.int64))
    k = np.concatenate(k_list)
    M = k.size
    var_idx = np.concatenate(var_blocks).astype(np.int32)
    coef = np.zeros((2, level, M))
    coef[0, 0] = 1.0
    coef[0, 0, -1] = -1.0
    poly_ptr = np.concatenate([np.arange(0, n * (n - 1) + 1, n), [M]]).astype(np.int64)
    return PolySystem(level=level, n_vars=n, poly_ptr=poly_ptr,
                      mon_ptr=np.concatenate([[0], np.cumsum(k)]).astype(np.int64),
                      var_idx=var_idx, exps=np.ones(var_idx.size, np.int32), coef=coef, name=f"cyclic{n}")


def product_system(n_monomials: int, n_vars: int, level: int, seed=0) -> PolySystem:
    """One-monomial polynomials, each the product of all n_vars variables with
    exponent 1 (the shape of Table 1, Section 2.2); unit-circle coefficients."""
    rng = rng_for(seed)
    M = n_monomials
    return PolySystem(level=level, n_vars=n_vars,
                      poly_ptr=np.arange(M + 1, dtype=np.int64),
                      mon_ptr=np.arange(0, M * n_vars + 1, n_vars, dtype=np.int64),
                      var_idx=np.tile(np.arange(n_vars, dtype=np.int32), M),
                      exps=np.ones(M * n_vars, np.int32),
                      coef=unit_circle(rng, M, level), name=f"product{M}x{n_vars}")


def chandrasekhar_system(n: int, level: int, c: float = 33.0 / 64.0) -> PolySystem:
    """Chandrasekhar H-equation (Section 5.2) read with j = 1..n:
    f_i = 2n H_i - c H_i sum_j i/(i+j) H_j - 2n.  Coefficients are rounded to
    double (lower limbs zero)."""
    polys = []
    for i in range(1, n + 1):
        mons = [(2.0 * n, [(i - 1, 1)])]
        for j in range(1, n + 1):
            coeff = -c * i / (i + j)
            if j == i:
                mons.append((coeff, [(i - 1, 2)]))
            else:
                a, b = sorted((i - 1, j - 1))
                mons.append((coeff, [(a, 1), (b, 1)]))
        mons.append((-2.0 * n, []))
        polys.append(mons)
    return from_monomial_lists(level, n, polys, name=f"chandra{n}")


def exact_regime_system(seed, level: int, n_vars: int, n_polys: int, m: int, k: int,
                        exp_hi: int = 3) -> PolySystem:
    """Small Gaussian-integer coefficients (real and imaginary parts in
    -3..3, not both zero); structure as in random_system.  Together with
    points from ``exact_regime_points`` every intermediate value of the
    evaluation is a small dyadic number, so all arithmetic is exact."""
    rng = rng_for(seed)
    M = n_polys * m
    vars_ = distinct_sorted_subsets(rng, M, n_vars, k)
    exps = rng.integers(1, exp_hi + 1, size=(M, k)).astype(np.int32)
    re = rng.integers(-3, 4, size=M).astype(np.float64)
    im = rng.integers(-3, 4, size=M).astype(np.float64)
    re = np.where((re == 0) & (im == 0), 1.0, re)
    coef = np.zeros((2, level, M))
    coef[0, 0], coef[1, 0] = re, im
    return PolySystem(level=level, n_vars=n_vars,
                      poly_ptr=np.arange(0, M + 1, m, dtype=np.int64),
                      mon_ptr=np.arange(0, M * k + 1, k, dtype=np.int64),
                      var_idx=vars_.reshape(-1), exps=exps.reshape(-1), coef=coef,
                      name="exact_regime")


def exact_regime_points(seed, P: int, n: int, level: int) -> np.ndarray:
    """Entries in {+1, -1, +i, -i} times 2^a with a uniform in -2..2."""
    rng = rng_for(seed)
    x = np.zeros((P, 2, level, n))
    unit = rng.integers(0, 4, size=(P, n))
    mag = np.ldexp(1.0, rng.integers(-2, 3, size=(P, n)))
    x[:, 0, 0] = np.where(unit == 0, mag, np.where(unit == 1, -mag, 0.0))
    x[:, 1, 0] = np.where(unit == 2, mag, np.where(unit == 3, -mag, 0.0))
    return x


def perturbed_start(seed, x_star: np.ndarray, scale: float = 1e-6) -> np.ndarray:
    """A start point near ``x_star`` ([2, L, n]): leading limbs moved by
    ``scale * e^{i phi}`` (phi ~ U[0, 2 pi)), rounded to double, lower limbs 0."""
    rng = rng_for(seed)
    n = x_star.shape[-1]
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n)
    x0 = np.zeros_like(x_star)
    x0[0, 0] = x_star[0, 0] + scale * np.cos(phi)
    x0[1, 0] = x_star[1, 0] + scale * np.sin(phi)
    return x0


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

WORKLOADS = {
    # plain method, complex double
    "d_n32": dict(level=1, n=32, N=32, m=32, k=8, exp_hi=3, P=1),
    # complex double double, F + 256x256 J, planted root for Gauss-Newton
    "dd_n256": dict(level=2, n=256, N=256, m=256, k=16, exp_hi=4, P=1),
    # complex quad double, compute bound
    "qd_n1024": dict(level=4, n=1024, N=1024, m=1024, k=32, exp_hi=3, P=1),
    # overdetermined DD system for the adjoint, batch of 64 points
    "dd_adjoint_1024x512": dict(level=2, n=512, N=1024, m=512, k=24, exp_hi=3, P=64),
}

# The shape of Table 1 (Section 2.2) in complex double: 65,024 polynomials, each
# one monomial, the product of all 1,024 variables (exponent 1), unit-circle
# coefficients and point; J is dense (65,024 x 1,024), so the evaluation is
# bound by writing it.
PRODUCT_WORKLOAD = dict(name="d_product_65024x1024", level=1, n=1024, N=65024, P=1)


def product_workload(seed: int = 0):
    """``(system, x[1, 2, 1, n])`` for the Table-1-shaped product workload;
    the system uses stream ``seed``, the point stream ``(seed, 1)``."""
    w = PRODUCT_WORKLOAD
    sys_ = product_system(w["N"], w["n"], w["level"], seed=seed)
    x = unit_circle_points(rng_for((seed, 1)), w["P"], w["n"], w["level"])
    return sys_, x


def workload(name: str, seed: int = 0, points: int | None = None):
    """Return ``(system, x[P, 2, L, n])`` for a named workload.

    The system uses stream ``seed``; points use stream ``(seed, 1)``."""
    w = WORKLOADS[name]
    sys_ = random_system(seed, w["level"], w["n"], w["N"], w["m"], w["k"], 1, w["exp_hi"], name=name)
    P = w["P"] if points is None else points
    x = unit_circle_points(rng_for((seed, 1)), P, w["n"], w["level"])
    return sys_, x


def batch_sizes(seed: int, count: int, choices=(32, 64, 128, 256)) -> np.ndarray:
    """Dimensions of the uneven batch: n uniform in ``choices``."""
    return rng_for((seed, 7)).choice(np.asarray(choices), size=count)


def batch_system(seed: int, index: int, n: int, level: int = 2) -> PolySystem:
    """System ``index`` of the uneven batch: N = m = n, k = min(16, n/4),
    exponents in {1, 2, 3}; its own child stream so systems can be drawn one
    at a time."""
    k = min(16, n // 4)
    return random_system((seed, 100, index), level, n, n, n, k, 1, 3, name=f"batch{index}")


def adjoint_vectors(seed: int, P: int, N: int, level: int) -> np.ndarray:
    """``[P, 2, L, N]`` unit-circle cotangent vectors (stream ``(seed, 2)``)."""
    return unit_circle_points(rng_for((seed, 2)), P, N, level)
