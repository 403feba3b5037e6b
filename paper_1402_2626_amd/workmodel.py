"""Algorithmic work of one evaluation: FP64 flops and bytes.

Operation counts per complex level-L operation are those of the arithmetic in
``csrc/mdarith.hpp``, counted from its source: additions, subtractions and
products count 1, an FMA counts 2, and multiplications by +-1 (sign changes)
count 0.

=========  ======  =======  =======
op         L = 1   L = 2    L = 4
=========  ======  =======  =======
cmul       6       50       478
cscal      2       10       92
cadd_J     2       16       170
cadd_F     2       22       170
=========  ======  =======  =======

cmul: D one FMA and one product per component; DD the fused double-word
two-product sum per component; QD the fused order-by-order sum of partial
products per component.  cscal: the product of a partial derivative by its
exponent (DD unnormalised, one product and two FMAs per component).  cadd_J:
one contribution added into a Jacobian entry (DD: TwoSum on the high parts
plus two plain additions per component, the compensated sum of the owners);
cadd_F: one monomial value added into F.

Two counts of complex products per monomial of k variables, l of them with
exponent d >= 2:

* the ALGORITHMIC count of the method (Sec. 2.1-2.3): the product of the k
  variables and all its partial derivatives by the reverse mode, 3k - 5
  products (Sec. 2.2; none for k = 1); the common factor of the l powers
  times the coefficient, max(l - 1, 0) + [l >= 1]; the term formation, one
  product for the value and k for the partial derivatives (Sec. 2.3); l
  scalings by an exponent; k + 1 additions (k into J, one into F).  This is
  the count the roofline fractions use.
* the EXECUTED count of the library's one-lane schedule, which folds the
  coefficient and the common factor into the seed of the reverse sweep
  (l products into the seed, k - 2 prefix products, 2k - 1 in the sweep:
  l + 3k - 3, at least l + 1), plus k exponent scalings.  The butterfly that
  joins the lanes of a monomial spanning several lanes adds products that
  neither count includes.

The table of powers (a few products per variable and point) is not counted.

Bytes: the packed structure that one evaluation must read (8 bytes per
occurrence record, 16L per monomial, 2 (n + 1) per chunk), x, and the
F and J outputs (16L bytes per complex number).
"""
from __future__ import annotations

import numpy as np

FLOPS = {
    1: dict(cmul=6, cscal=2, cadd_J=2, cadd_F=2),
    2: dict(cmul=50, cscal=10, cadd_J=16, cadd_F=22),
    4: dict(cmul=478, cscal=92, cadd_J=170, cadd_F=170),
}


# Real level-L operations, counted the same way: a product (DD with FMA
# two-product, QD order 0..2 partial products exact) and a sum (DD sloppy,
# QD order by order).
RFLOPS = {
    1: dict(mul=1, add=1),
    2: dict(mul=10, add=11),
    4: dict(mul=96, add=85),
}


def lstsq_multiply_adds(N: int, n: int) -> int:
    """Multiply-adds of one least-squares solve of an N x n system by modified
    Gram-Schmidt on the augmented N x (n + 1) matrix (Sec. 3, Fig. 4) and back
    substitution (eq. (4)): each pair of columns c < j takes N for the inner
    product and N for the update, each column N for its squared norm, and the
    back substitution n (n + 1) / 2."""
    return N * n * (n + 1) + N * (n + 1) + n * (n + 1) // 2


def lstsq_flops(level_code: int, N: int, n: int) -> float:
    """FP64 flops of lstsq_multiply_adds at a level code (1, 2, 4 complex;
    8 | L real): a complex multiply-add is a complex product plus a complex
    sum, a real one a product plus a sum."""
    L = level_code & 7
    if level_code & 8:
        f = RFLOPS[L]["mul"] + RFLOPS[L]["add"]
    else:
        f = FLOPS[L]["cmul"] + FLOPS[L]["cadd_F"]
    return float(lstsq_multiply_adds(N, n)) * f


def algorithmic_products(k: int, ell: int) -> int:
    """Complex products of one monomial by the method's own count."""
    if k <= 0:
        return 0
    return max(3 * k - 5, 0) + max(ell - 1, 0) + (1 if ell >= 1 else 0) + 1 + k


def executed_products(k: int, ell: int) -> int:
    """Complex products of the library's one-lane schedule for one monomial."""
    if k <= 0:
        return 0
    return ell + max(3 * k - 3, 1)


def _k_and_ell(sys_):
    k = np.diff(sys_.mon_ptr).astype(np.int64)
    owner = np.repeat(np.arange(sys_.n_monomials), k)
    ell = np.zeros(sys_.n_monomials, np.int64)
    np.add.at(ell, owner, (sys_.exps >= 2).astype(np.int64))
    return k, ell


def algorithmic_counts(sys_):
    """(cmul, cscal, cadd_J, cadd_F) of the method for one point."""
    k, ell = _k_and_ell(sys_)
    pos = k > 0
    kp, lp = k[pos], ell[pos]
    cmul = np.maximum(3 * kp - 5, 0) + np.maximum(lp - 1, 0) + (lp >= 1) + 1 + kp
    return int(cmul.sum()), int(ell.sum()), int(k.sum()), int(sys_.n_monomials)


def executed_counts(sys_):
    """(cmul, cscal, cadd_J, cadd_F) of the library's schedule for one point
    (butterfly products excluded)."""
    k, ell = _k_and_ell(sys_)
    pos = k > 0
    cmul = ell[pos] + np.maximum(3 * k[pos] - 3, 1)
    return int(cmul.sum()), int(k.sum()), int(k.sum()), int(sys_.n_monomials)


def _flops(level, counts) -> float:
    f = FLOPS[level]
    cmul, cscal, cadd_j, cadd_f = counts
    return float(cmul * f["cmul"] + cscal * f["cscal"] + cadd_j * f["cadd_J"] + cadd_f * f["cadd_F"])


def flops_per_point(sys_) -> float:
    """Algorithmic FP64 flops of one evaluation of F and J at one point."""
    return _flops(sys_.level, algorithmic_counts(sys_))


def executed_flops_per_point(sys_) -> float:
    """FP64 flops of the library's schedule at one point."""
    return _flops(sys_.level, executed_counts(sys_))


def terms_bytes_per_point(sys_) -> float:
    """Bytes one per-monomial evaluation (values and partials written in
    input order, nothing summed) must move at one point: the records (8 bytes
    per occurrence), the coefficients and x read; each monomial's value and
    each occurrence's partial derivative written (16L bytes each)."""
    c16 = 16 * sys_.level
    return 8.0 * sys_.nnz + 2.0 * c16 * sys_.n_monomials + c16 * sys_.n_vars + c16 * sys_.nnz


def bytes_per_point(sys_, want_J: bool = True, chunks: int | None = None) -> float:
    L = sys_.level
    c16 = 16 * L
    b = 8.0 * sys_.nnz + c16 * sys_.n_monomials
    if chunks is not None:
        b += 2.0 * (sys_.n_vars + 1) * chunks
    b += c16 * sys_.n_vars + c16 * sys_.n_polys
    if want_J:
        b += c16 * sys_.n_polys * sys_.n_vars
    return b
