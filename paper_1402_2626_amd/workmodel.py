"""Algorithmic work of one evaluation: FP64 flops and bytes.

Operation counts are those of the arithmetic in ``csrc/mdarith.hpp``,
counted from its source: additions, subtractions and products count 1, an
FMA counts 2, and multiplications by +-1 (sign changes) count 0.

Per complex level-L operation (flops):

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
one slot added into a Jacobian column (DD: TwoSum on the high parts plus two
plain additions per component, the compensated sum of the owners); cadd_F:
one monomial value added into F.

The algorithmic work of a monomial with k variables, l of them with exponent
d >= 2, is the work of the reverse mode over its product of variables with
the coefficient and the common factor folded into the seed (Sec. 2.2-2.3):
l products for the common factor, k-1 forward products, k-1 products for the
partial derivatives and k for the backward products (the last one gives the
monomial's value), i.e. l + 3k - 2 complex products; k scalings by the
exponent; k additions into J and one into F.  A constant monomial (k = 0)
costs one addition.  The table of powers costs n (emax - 2) products per point.  The
extra products of the library's lane decomposition (the butterfly across the
lanes of a monomial) are not algorithmic and not counted, so a roofline
fraction from these counts is a lower bound of the FP64 utilisation.

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


def monomial_counts(sys_):
    """(cmul, cscal, cadd_J, cadd_F) totals for one point."""
    k = np.diff(sys_.mon_ptr).astype(np.int64)
    hi = (sys_.exps >= 2).astype(np.int64)
    owner = np.repeat(np.arange(sys_.n_monomials), k)
    ell = np.zeros(sys_.n_monomials, np.int64)
    np.add.at(ell, owner, hi)
    pos = k > 0
    cmul = int(np.sum(ell[pos] + 3 * k[pos] - 2))
    emax = int(sys_.exps.max()) if sys_.nnz else 1
    cmul += sys_.n_vars * max(0, emax - 2)
    cscal = int(np.sum(k))
    return cmul, cscal, int(np.sum(k)), int(sys_.n_monomials)


def flops_per_point(sys_) -> float:
    f = FLOPS[sys_.level]
    cmul, cscal, cadd_j, cadd_f = monomial_counts(sys_)
    return float(cmul * f["cmul"] + cscal * f["cscal"] + cadd_j * f["cadd_J"] + cadd_f * f["cadd_F"])


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
