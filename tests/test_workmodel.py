"""A host model of the kernels' per-lane reverse-mode schedule (Sec. 2.2-2.3).

Each value is a node of a product DAG over symbolic leaves (the coefficient,
the variables, the powers from the table); a product by the constant 1 is no
product.  The model follows the schedule of the monomial phase: lane q of a
monomial's s lanes takes occurrences q, q + s, ... (padding records read the
constant 1), multiplies the common factor of its segment into the seed, forms
prefix products, combines the s segment products by a butterfly and runs the
reverse sweep.  The tests check that every slot receives exactly the partial
derivative of the product rule, and count the products that reach an output:
3k - 5 for a plain product of k variables (Sec. 2.2), and the per-monomial
product count of the work model.
"""
from collections import Counter

import numpy as np
import pytest

from paper_1402_2626_amd import workmodel as W
from paper_1402_2626_amd import synth


class Dag:
    def __init__(self):
        self.nodes = []  # ("leaf", name) or ("mul", a, b)

    def leaf(self, name):
        self.nodes.append(("leaf", name))
        return len(self.nodes) - 1

    def mul(self, a, b):
        if a == ONE:
            return b
        if b == ONE:
            return a
        self.nodes.append(("mul", a, b))
        return len(self.nodes) - 1

    def factors(self, v):
        if v == ONE:
            return Counter()
        node = self.nodes[v]
        if node[0] == "leaf":
            return Counter({node[1]: 1})
        return self.factors(node[1]) + self.factors(node[2])

    def live_products(self, outputs):
        seen, stack = set(), [o for o in outputs if o != ONE]
        while stack:
            v = stack.pop()
            if v in seen:
                continue
            seen.add(v)
            node = self.nodes[v]
            if node[0] == "mul":
                stack += [c for c in node[1:] if c != ONE]
        return sum(1 for v in seen if self.nodes[v][0] == "mul")


ONE = -1


def lanes_for(k, seg):
    need = -(-k // seg)
    s = 1
    while s < need:
        s <<= 1
    return s


def schedule(k, exps, seg, coef_is_one=False):
    """Model of one monomial's lanes; returns (dag, slot values in occurrence
    order, value) with slots before the exponent scaling."""
    dag = Dag()
    s = lanes_for(max(k, 1), seg)
    segc = -(-k // s) if k else 1
    x = [dag.leaf(f"x{r}") for r in range(k)]
    power = {r: dag.leaf(f"x{r}^{exps[r] - 1}") for r in range(k) if exps[r] >= 2}
    c = ONE if coef_is_one else dag.leaf("c")
    lanes = []
    for q in range(s):
        occ = [q + i * s for i in range(segc)]
        occ = [r if r < k else None for r in occ]  # None: padding, the constant 1
        cf = c if q == 0 else ONE
        xv = [x[r] if r is not None else ONE for r in occ]
        pre, A = [], ONE
        for i, r in enumerate(occ):
            if r is not None and r in power:
                cf = dag.mul(cf, power[r])
            A = xv[0] if i == 0 else dag.mul(A, xv[i])
            if i < segc - 1:
                pre.append(A)
        lanes.append(dict(occ=occ, cf=cf, xv=xv, pre=pre, B=dag.mul(A, cf)))
    # butterfly: every lane gets the product of the other lanes' B
    B = [ln["B"] for ln in lanes]
    E = [ONE] * s
    m = 1
    while m < s:
        Bp = [B[q ^ m] for q in range(s)]
        E = [Bp[q] if m == 1 else dag.mul(E[q], Bp[q]) for q in range(s)]
        B = [dag.mul(B[q], Bp[q]) for q in range(s)]
        m <<= 1
    slots, value = {}, None
    for q, ln in enumerate(lanes):
        Sx = dag.mul(ln["cf"], E[q]) if s > 1 else ln["cf"]
        for i in range(segc - 1, 0, -1):
            gi = dag.mul(ln["pre"][i - 1], Sx)
            Sx = dag.mul(Sx, ln["xv"][i])
            if ln["occ"][i] is not None:
                slots[ln["occ"][i]] = gi
        if ln["occ"][0] is not None:
            slots[ln["occ"][0]] = Sx
        Sx = dag.mul(Sx, ln["xv"][0])
        if q == 0:
            value = Sx
    return dag, [slots[r] for r in range(k)], value


@pytest.mark.parametrize("seg", [1, 2, 4, 6, 8, 16])
def test_slots_hold_the_product_rule(seg):
    """Slot r = c x_r^(d_r - 1) prod_{s != r} x_s^(d_s) (before the exponent
    factor), the value = c prod x^d, for ragged, full and multi-lane
    monomials."""
    rng = synth.rng_for(5)
    for k in (1, 2, 3, 5, 8, 13, 16, 31, 32, 50, 64, 100):
        if lanes_for(k, seg) > 64:
            continue
        exps = [int(e) for e in rng.integers(1, 4, size=k)]
        dag, slots, value = schedule(k, exps, seg)

        def term(skip=None):
            f = Counter({"c": 1})
            for r in range(k):
                if r == skip:
                    if exps[r] >= 2:
                        f[f"x{r}^{exps[r] - 1}"] += 1
                    continue
                f[f"x{r}"] += 1
                if exps[r] >= 2:
                    f[f"x{r}^{exps[r] - 1}"] += 1
            return f

        for r in range(k):
            assert dag.factors(slots[r]) == term(skip=r), (k, seg, r)
        assert dag.factors(value) == term(), (k, seg)


@pytest.mark.parametrize("k", list(range(2, 17)) + [24, 32, 64])
def test_plain_product_costs_3k_minus_5(k):
    """One lane over the whole product (segment >= k), coefficient 1 and
    exponents 1: the value and all k partials cost 3k - 5 products, the
    count of Sec. 2.2 (k - 1 for the value, 2k - 4 for the gradient)."""
    dag, slots, value = schedule(k, [1] * k, seg=max(k, 1), coef_is_one=True)
    assert dag.live_products(slots + [value]) == 3 * k - 5


@pytest.mark.parametrize("k", [1, 2, 3, 8, 16, 24, 32])
def test_work_model_counts_the_one_lane_schedule(k):
    """With a coefficient and l variables of exponent >= 2, one lane costs
    l + max(3k - 3, 1) products; the work model counts the same."""
    rng = synth.rng_for((6, k))
    for _ in range(4):
        exps = [int(e) for e in rng.integers(1, 5, size=k)]
        ell = sum(e >= 2 for e in exps)
        dag, slots, value = schedule(k, exps, seg=k)
        live = dag.live_products(slots + [value])
        assert live == ell + max(3 * k - 3, 1)
        assert live == W.executed_products(k, ell)


def test_method_count_bounds_the_schedule():
    """The algorithmic count with a separate term formation (tree 3k - 5,
    common factor and coefficient, value, k partials) is at least what the
    fused schedule executes on one lane."""
    for k in range(1, 40):
        for ell in (0, 1, k // 2, k):
            assert W.algorithmic_products(k, ell) >= W.executed_products(k, ell)


class _Counted:
    """A number that counts the products made with it (a sum follows each
    product in a multiply-add)."""
    products = 0

    def __init__(self, v):
        self.v = v

    def __mul__(self, o):
        _Counted.products += 1
        return _Counted(self.v * (o.v if isinstance(o, _Counted) else o))

    __rmul__ = __mul__

    def __add__(self, o):
        return _Counted(self.v + (o.v if isinstance(o, _Counted) else o))

    __radd__ = __add__

    def __sub__(self, o):
        return _Counted(self.v - (o.v if isinstance(o, _Counted) else o))

    def __truediv__(self, o):
        return _Counted(self.v / (o.v if isinstance(o, _Counted) else o))


@pytest.mark.parametrize("N, n", [(1, 1), (3, 2), (7, 4), (12, 9)])
def test_lstsq_count_matches_a_counted_solve(N, n):
    """Modified Gram-Schmidt on the N x (n + 1) augmented matrix with
    unnormalised pivots (Sec. 3, Fig. 4) and back substitution, written as
    plain loops over counting numbers: the products made equal the work
    model's multiply-adds (with the back substitution's n divisions), and
    the solution is the least-squares one."""
    rng = synth.rng_for((7, N, n))
    A = rng.standard_normal((N, n + 1)) + 3.0 * np.eye(N, n + 1)
    W_ = [[_Counted(float(A[i, j])) for j in range(n + 1)] for i in range(N)]
    _Counted.products = 0
    nrm = []
    R = [[None] * (n + 1) for _ in range(n + 1)]
    for c in range(n + 1):
        s = _Counted(0.0)
        for i in range(N):
            s = s + W_[i][c] * W_[i][c]
        nrm.append(s)
        for j in range(c + 1, n + 1):
            d = _Counted(0.0)
            for i in range(N):
                d = d + W_[i][c] * W_[i][j]
            R[c][j] = d
            f = d / s
            for i in range(N):
                W_[i][j] = W_[i][j] - f * W_[i][c]
    # back substitution on the unnormalised factors: x_j = (y_j - sum_{l > j} r_jl x_l) / |a_j|^2
    x = [None] * n
    for j in range(n - 1, -1, -1):
        t = R[j][n]
        for l in range(j + 1, n):
            t = t - R[j][l] * x[l]
        x[j] = t / nrm[j]
    # the model counts the n divisions of the back substitution with its products
    assert _Counted.products + n == W.lstsq_multiply_adds(N, n)
    if N >= n:
        want = np.linalg.lstsq(A[:, :n], A[:, n], rcond=None)[0]
        assert np.allclose([v.v for v in x], want, rtol=1e-9, atol=1e-9)


def test_real_and_complex_solve_flops():
    """Complex flops are (cmul + cadd_F) per multiply-add, real ones
    (mul + add); a complex multiply-add costs more than twice a real one at
    every level."""
    for L in (1, 2, 4):
        m = W.lstsq_multiply_adds(100, 50)
        assert W.lstsq_flops(L, 100, 50) == m * (W.FLOPS[L]["cmul"] + W.FLOPS[L]["cadd_F"])
        assert W.lstsq_flops(8 | L, 100, 50) == m * (W.RFLOPS[L]["mul"] + W.RFLOPS[L]["add"])
        assert W.lstsq_flops(L, 100, 50) > 2 * W.lstsq_flops(8 | L, 100, 50)


def test_terms_bytes_count_the_outputs_once():
    """Per-monomial output moves each record once (8 bytes), reads the
    coefficients and x, and writes one value per monomial and one partial per
    occurrence (16L bytes each): for the Table-1 shape at L = 1 that is
    8 nnz + 32 M + 16 n + 16 nnz."""
    from paper_1402_2626_amd import synth
    s = synth.product_system(5, 7, 1)
    assert W.terms_bytes_per_point(s) == 8 * 35 + 32 * 5 + 16 * 7 + 16 * 35
    s2 = synth.product_system(5, 7, 2)
    assert W.terms_bytes_per_point(s2) == 8 * 35 + 64 * 5 + 32 * 7 + 32 * 35
