"""Parity of the HIP evaluation path (through the C ABI) with the exact oracle."""
import numpy as np
import pytest

import gpu_util as U
import oracle as O
from paper_1402_2626_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1402_2626_amd import polyeval
    return polyeval


def run_eval(pe, sys_, x, want_J=True):
    import torch
    S = pe.System.from_sparse(sys_)
    F, J = S.eval(U.to_device(x), want_J=want_J)
    torch.cuda.synchronize()
    out = F.cpu().numpy(), (J.cpu().numpy() if J is not None else None)
    S.close()
    return out


# ------------------------------------------------------------------ named workloads

def test_d_n32_full(pe):
    """Plain complex double system: n = N = 32, 32 monomials of k = 8."""
    sys_, x = synth.workload("d_n32")
    U.flush("d_n32: evaluating")
    F, J = run_eval(pe, sys_, x)
    eF, eJ = U.max_errors_rows(sys_, x[0], F[0], J[0], range(sys_.n_polys), parallel=False)
    tol = U.tolerance(sys_)
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


def test_dd_n256_full(pe):
    """Complex double double: n = N = 256, 256 monomials of k = 16, every row."""
    sys_, x = synth.workload("dd_n256")
    U.flush("dd_n256: evaluating")
    F, J = run_eval(pe, sys_, x)
    U.flush("dd_n256: oracle over all rows")
    eF, eJ = U.max_errors_rows(sys_, x[0], F[0], J[0], range(sys_.n_polys))
    tol = U.tolerance(sys_)
    U.flush(f"dd_n256: eF={eF:.3e} eJ={eJ:.3e} tol={tol:.1e}")
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


def test_qd_n1024_sampled(pe):
    """Complex quad double: n = N = 1024, 1024 monomials of k = 32; sampled
    rows (first, last, two inside) and columns against the oracle."""
    sys_, x = synth.workload("qd_n1024")
    U.flush("qd_n1024: evaluating")
    F, J = run_eval(pe, sys_, x)
    tol = U.tolerance(sys_)
    rows = [0, 511, 700, 1023]
    U.flush("qd_n1024: oracle rows")
    eF, eJ = U.max_errors_rows(sys_, x[0], F[0], J[0], rows)
    U.flush(f"qd_n1024: rows eF={eF:.3e} eJ={eJ:.3e} tol={tol:.1e}")
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)
    cols = [0, 17, 500, 1023]
    U.flush("qd_n1024: oracle columns")
    eC = U.max_error_cols(sys_, x[0], J[0], cols)
    assert eC <= tol, (eC, tol)


# ------------------------------------------------------------------ exact regime

@pytest.mark.parametrize("L", [1, 2, 4])
def test_exact_regime_bit_exact(pe, L):
    """x_j in {+-1, +-i} 2^a and Gaussian-integer coefficients: every value is
    exact, so F and J must equal the exact result bit for bit with zero lower
    limbs."""
    sys_ = synth.exact_regime_system(7, L, n_vars=40, n_polys=24, m=12, k=5, exp_hi=3)
    x = synth.exact_regime_points(8, 2, 40, L)
    F, J = run_eval(pe, sys_, x)
    for pt in range(2):
        Fx, Jx = O.eval_system(sys_, x[pt])
        for p in range(sys_.n_polys):
            assert np.array_equal(F[pt, :, :, p], O.cdy_to_limbs(Fx[p], L)), (pt, p)
            for j in range(sys_.n_vars):
                assert np.array_equal(J[pt, :, :, p, j], O.cdy_to_limbs(Jx[p].get(j, O.ZERO), L)), (pt, p, j)


# ------------------------------------------------------------------ edge cases

def _edge_system(L, seed=3):
    """Mixed monomial sizes k in {0,1,2,3,5,31,33,64,100}, an empty
    polynomial, duplicate monomials, exponents up to 9, n = 130."""
    rng = synth.rng_for(seed)
    n = 130
    polys = []
    for p in range(7):
        mons = []
        for k in (0, 1, 2, 3, 5, 31, 33, 64, 100):
            vs = np.sort(rng.choice(n, size=k, replace=False))
            ds = rng.integers(1, 10, size=k)
            mons.append((0, list(zip(vs.tolist(), ds.tolist()))))
        if p == 3:
            mons.append(mons[-2])  # duplicate monomial, kept as given
        if p == 5:
            mons = []  # empty polynomial
        polys.append(mons)
    M = sum(len(m) for m in polys)
    coef = synth.unit_circle(rng, M, L)
    return synth.from_monomial_lists(L, n, polys, coef_limbs=coef, name="edge")


@pytest.mark.parametrize("L", [1, 2, 4])
def test_edge_cases(pe, L):
    sys_ = _edge_system(L)
    x = synth.unit_circle_points(synth.rng_for(4), 2, sys_.n_vars, L)
    x[1, :, :, 5] = 0.0  # a zero variable
    x[1, :, :, 7] = 0.0
    x = x * 0.9  # moduli below one keep degree-100 terms in range
    F, J = run_eval(pe, sys_, x)
    tol = U.tolerance(sys_)
    for pt in range(2):
        eF, eJ = U.max_errors_rows(sys_, x[pt], F[pt], J[pt], range(sys_.n_polys), parallel=False)
        assert eF <= tol and eJ <= tol, (pt, eF, eJ, tol)
    # the empty polynomial's row is exactly zero
    assert np.all(F[:, :, :, 5] == 0.0) and np.all(J[:, :, :, 5, :] == 0.0)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_univariate_large_exponents(pe, L):
    """n = 1 with exponents up to 300: no power table fits the LDS budget
    when... (table up to 299 entries is small, so also forced via n)."""
    rng = synth.rng_for(12)
    polys = [[(0, [(0, int(d))]) for d in (1, 2, 3, 17, 64, 255, 300)], [(0, [])]]
    coef = synth.unit_circle(rng, 8, L)
    sys_ = synth.from_monomial_lists(L, 1, polys, coef_limbs=coef)
    x = synth.unit_circle_points(synth.rng_for(13), 1, 1, L)
    F, J = run_eval(pe, sys_, x)
    eF, eJ = U.max_errors_rows(sys_, x[0], F[0], J[0], range(2), parallel=False)
    tol = U.tolerance(sys_)
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_power_fallback_without_table(pe, L):
    """Many variables with high exponents: the power table would not fit in
    LDS, so powers come from binary powering."""
    n = 1500
    sys_ = synth.random_system(21, L, n_vars=n, n_polys=3, m=40, k=6, exp_lo=1, exp_hi=60)
    x = synth.unit_circle_points(synth.rng_for(22), 1, n, L)
    F, J = run_eval(pe, sys_, x)
    eF, eJ = U.max_errors_rows(sys_, x[0], F[0], J[0], range(3), parallel=False)
    tol = U.tolerance(sys_)
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_F_only_and_points(pe, L):
    """J = NULL evaluates F only; several points at once agree with one point
    at a time bit for bit."""
    sys_ = synth.random_system(31, L, n_vars=50, n_polys=20, m=30, k=7, exp_lo=1, exp_hi=3)
    x = synth.unit_circle_points(synth.rng_for(32), 3, 50, L)
    F3, J3 = run_eval(pe, sys_, x)
    for pt in range(3):
        F1, J1 = run_eval(pe, sys_, x[pt:pt + 1])
        assert np.array_equal(F1[0], F3[pt]) and np.array_equal(J1[0], J3[pt])
    Fo, Jo = run_eval(pe, sys_, x, want_J=False)
    assert Jo is None
    tol = U.tolerance(sys_)
    for pt in range(3):
        eF, _ = U.max_errors_rows(sys_, x[pt], Fo[pt], None, range(20), parallel=False)
        assert eF <= tol


def test_deterministic_and_shapes(pe):
    """Bitwise equal reruns for each launch shape; the one-chunk and
    four-chunk workgroups differ only by rounding."""
    import torch
    sys_, x = synth.workload("dd_n256")
    S = pe.System.from_sparse(sys_)
    assert S.info()["chunks_per_workgroup"] > 1
    xd = U.to_device(x)
    outs = {}
    for G in (S.info()["chunks_per_workgroup"], 1):
        S.set_shape(G)
        assert S.info()["chunks_per_workgroup"] == G
        a = [t.cpu().numpy() for t in S.eval(xd)]
        b = [t.cpu().numpy() for t in S.eval(xd)]
        torch.cuda.synchronize()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), G
        outs[G] = a
    tol = U.tolerance(sys_)
    rows = [0, 100, 255]
    for G in outs:
        eF, eJ = U.max_errors_rows(sys_, x[0], outs[G][0][0], outs[G][1][0], rows, parallel=False)
        assert eF <= tol and eJ <= tol, (G, eF, eJ)
    S.close()


@pytest.mark.parametrize("L", [1, 2, 4])
def test_cyclic_roots_closed_forms(pe, L):
    """Cyclic n-roots (eq. (5)) at x = 1: F_i = n, last 0; J_{i,m} = i (1-based),
    last row ones; exact at every level."""
    n = 64
    sys_ = synth.cyclic_roots_system(n, L)
    x = np.zeros((1, 2, L, n))
    x[0, 0, 0] = 1.0
    F, J = run_eval(pe, sys_, x)
    want_F = np.full(n, float(n))
    want_F[-1] = 0.0
    assert np.array_equal(F[0, 0, 0], want_F) and np.all(F[0, 1] == 0) and np.all(F[0, 0, 1:] == 0)
    want_J = np.repeat(np.arange(1, n + 1, dtype=float)[:, None], n, axis=1)
    want_J[-1] = 1.0
    assert np.array_equal(J[0, 0, 0], want_J) and np.all(J[0, 1] == 0)


def test_shapes_and_autotune(pe, tmp_path):
    """Every compiled launch shape gives results within tolerance; autotune
    keeps one of them and records it in the plan cache, which a new system
    of the same shape picks up."""
    import torch
    sys_ = synth.random_system(41, 2, n_vars=96, n_polys=40, m=96, k=12, exp_lo=1, exp_hi=4)
    x = synth.unit_circle_points(synth.rng_for(42), 2, 96, 2)
    S = pe.System.from_sparse(sys_)
    xd = U.to_device(x)
    tol = U.tolerance(sys_)
    seen = []
    for seg in (4, 6, 8):
        for G in (1, 2, 4):
            try:
                S.set_shape(G, segment=seg)
            except pe.PolyevalError as e:
                assert e.status == pe.PE_EUNSUPPORTED
                continue
            info = S.info()
            assert (info["segment"], info["chunks_per_workgroup"]) == (seg, G)
            F, J = S.eval(xd)
            torch.cuda.synchronize()
            F, J = F.cpu().numpy(), J.cpu().numpy()
            eF, eJ = U.max_errors_rows(sys_, x[1], F[1], J[1], [0, 17, 39], parallel=False)
            assert eF <= tol and eJ <= tol, (seg, G, eF, eJ)
            seen.append((seg, G))
    assert (4, 1) in seen and (8, 1) in seen and len(seen) >= 3
    cache = tmp_path / "plans.txt"
    pe.set_plan_cache(str(cache))
    try:
        S.autotune(P=2)
        chosen = S.info()
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 1 and f"| {chosen['segment']} {chosen['chunks_per_workgroup']} " in lines[0]
        S2 = pe.System.from_sparse(sys_)
        i2 = S2.info()
        assert (i2["segment"], i2["chunks_per_workgroup"]) == (chosen["segment"], chosen["chunks_per_workgroup"])
        F, J = S2.eval(xd)
        torch.cuda.synchronize()
        eF, eJ = U.max_errors_rows(sys_, x[0], F.cpu().numpy()[0], J.cpu().numpy()[0], [5], parallel=False)
        assert eF <= tol and eJ <= tol
        S2.close()
    finally:
        pe.set_plan_cache(None)
    S.close()


@pytest.mark.parametrize("L", [1, 2])
def test_products_without_power_table(pe, L):
    """Exponent-1 systems whose rows use each variable about once: in double
    precision x is gathered from global memory and the LDS holds only the
    slots (double-double keeps its table).  Full rows against the oracle with
    full segments (k = 64), ragged segments (k = 50) and, at a segment of 4,
    rows of two chunks."""
    import torch
    cases = [(512, 6, 8, 64, 0), (512, 6, 6, 50, 0)]
    if L == 2:
        cases.append((2000, 3, 30, 64, 4))
    for n, N, m, k, seg in cases:
        sys_ = synth.random_system((33, n, k), L, n_vars=n, n_polys=N, m=m, k=k, exp_lo=1, exp_hi=1)
        x = synth.unit_circle_points(synth.rng_for((34, n, k)), 1, n, L)
        S = pe.System.from_sparse(sys_)
        if seg:
            S.set_shape(0, seg)
        info = S.info()
        # slots (at most m k + 1 per chunk) and the F partials only: a table
        # of x would add (n + 1) 16 L bytes
        no_table = info["lds_bytes"] <= (m * k + 1 + 16) * 16 * L
        assert no_table == (L == 1), info
        U.flush(f"products without table: L={L} n={n} k={k} segment={info['segment']}")
        F, J = S.eval(U.to_device(x))
        torch.cuda.synchronize()
        S.close()
        F, J = F.cpu().numpy(), J.cpu().numpy()
        eF, eJ = U.max_errors_rows(sys_, x[0], F[0], J[0], range(N), parallel=True)
        tol = U.tolerance(sys_)
        assert eF <= tol and eJ <= tol, (n, k, eF, eJ, tol)


@pytest.mark.parametrize("L", [1, 2])
def test_uneven_rows(pe, L):
    """Rows of very different cost (row p holds 1 + 12p monomials of six
    variables, the longest spanning two chunks) are started in decreasing
    cost; every row must still land in its own place of F and J.  All rows
    against the oracle, at two points."""
    import torch
    rng = synth.rng_for((41, L))
    n, N = 48, 40
    polys = []
    for p in range(N):
        mons = []
        for _ in range(1 + 12 * p):
            vs = np.sort(rng.choice(n, size=6, replace=False))
            ds = rng.integers(1, 4, size=6)
            c = complex(*rng.normal(size=2))
            mons.append((c, [(int(v), int(d)) for v, d in zip(vs, ds)]))
        polys.append(mons)
    sys_ = synth.from_monomial_lists(L, n, polys)
    x = synth.unit_circle_points(synth.rng_for((42, L)), 2, n, L)
    F, J = run_eval(pe, sys_, x)
    tol = U.tolerance(sys_)
    for pt in range(2):
        eF, eJ = U.max_errors_rows(sys_, x[pt], F[pt], J[pt], range(N), parallel=True)
        assert eF <= tol and eJ <= tol, (pt, eF, eJ, tol)


@pytest.mark.gpu
def test_default_segment_follows_monomial_size(pe):
    """The default segment length is the first of the level's preferred
    lengths that the most common monomial size fills exactly."""
    cases = [(2, 16, 8), (2, 24, 6), (2, 12, 6), (2, 4, 4), (2, 20, 8), (4, 32, 4), (4, 6, 2), (1, 16, 8),
             (1, 24, 8)]
    for level, k, want in cases:
        sys_ = synth.random_system(7, level, n_vars=64, n_polys=3, m=8, k=k, exp_lo=1, exp_hi=2)
        S = pe.System.from_sparse(sys_)
        assert S.info()["segment"] == want, (level, k)
        S.close()


def test_product_table1_shape(pe):
    """The Table-1 shape in complex double (65,024 polynomials, each the
    product of all 1,024 variables) at full size: three sampled rows against
    the oracle, and on every row x_j dF/dx_j summed over j = 1024 F (Euler:
    each polynomial is homogeneous of degree 1,024)."""
    import torch
    sys_, x = synth.product_workload()
    S = pe.System.from_sparse(sys_)
    assert S.info()["segment"] == 16
    U.flush("product workload: one launch, J of 1.07 GB")
    F, J = S.eval(U.to_device(x))
    torch.cuda.synchronize()
    S.close()
    tol = U.tolerance(sys_)
    rows = [0, 32511, sys_.n_polys - 1]
    sub = U.row_subsystem(sys_, rows)
    Fs = F[:, :, :, rows].cpu().numpy()[0]
    Js = J[:, :, :, rows, :].cpu().numpy()[0]
    eF, eJ = U.max_errors_rows(sub, x[0], Fs, Js, range(len(rows)), parallel=True)
    assert eF <= tol and eJ <= tol, (eF, eJ)
    # Euler's identity on all rows, in complex128 on the device
    xd = U.to_device(x)
    xc = torch.complex(xd[0, 0, 0], xd[0, 1, 0])
    Jc = torch.complex(J[0, 0, 0], J[0, 1, 0])
    Fc = torch.complex(F[0, 0, 0], F[0, 1, 0])
    lhs = (Jc * xc[None, :]).sum(dim=1)
    err = ((lhs - 1024.0 * Fc).abs() / (1024.0 * Fc.abs())).max().item()
    assert err <= tol, err
    del F, J, Jc


@pytest.mark.parametrize("L", [1, 2])
def test_cyclic_512_closed_forms(pe, L):
    """Cyclic 512-roots (eq. (5)), the largest size of the paper's Table 5 for
    D and DD, at x = 1: F_i = n for i < n, F_n = 0; J_{i,m} = i, last row 1;
    every product and sum is exact."""
    n = 512
    sys_ = synth.cyclic_roots_system(n, L)
    x = np.zeros((1, 2, L, n))
    x[0, 0, 0] = 1.0
    F, J = run_eval(pe, sys_, x)
    want_F = np.full(n, float(n))
    want_F[-1] = 0.0
    assert np.array_equal(F[0, 0, 0], want_F) and np.all(F[0, 1] == 0) and np.all(F[0, 0, 1:] == 0)
    want_J = np.repeat(np.arange(1, n + 1, dtype=float)[:, None], n, axis=1)
    want_J[-1] = 1.0
    assert np.array_equal(J[0, 0, 0], want_J) and np.all(J[0, 1] == 0) and np.all(J[0, 0, 1:] == 0)


def _cyclic_roots_of_unity(n, rows, prec=200):
    """Cyclic n-roots (eq. (5)) at x_k = w^k, w = e^(2 pi i / n), in closed
    form: row r < n - 1 (monomials of d = r + 1 cyclically consecutive
    variables) has F_r = w^(d(d-1)/2) sum_j w^(dj) = 0 and
    J_{r,m} = w^((d-1)m + d(d-1)/2) sum_{t<d} w^(-dt) (a geometric sum); the
    last row x_0 ... x_(n-1) - 1 has F = (-1)^(n-1) - 1 and
    J_{n-1,m} = (-1)^(n-1) w^(-m).  Returns (x limbs helper, {r: F}, {r: [J]})
    as mpmath values."""
    import mpmath
    with mpmath.workprec(prec):
        W = [mpmath.expjpi(mpmath.mpf(2 * k) / n) for k in range(n)]
        Fr, Jr = {}, {}
        for r in rows:
            if r == n - 1:
                sgn = -1 if (n - 1) % 2 else 1
                Fr[r] = mpmath.mpc(sgn - 1)
                Jr[r] = [sgn * W[(-m) % n] for m in range(n)]
                continue
            d = r + 1
            geo = mpmath.fsum(W[(-d * t) % n] for t in range(d))
            Fr[r] = mpmath.mpc(0)
            Jr[r] = [W[((d - 1) * m + d * (d - 1) // 2) % n] * geo for m in range(n)]
    return W, Fr, Jr


@pytest.mark.parametrize("L", [1, 2])
def test_cyclic_512_roots_of_unity(pe, L):
    """Cyclic 512-roots at x_k = w^k rounded to the level: F and sampled full
    rows of J (the shortest, middle, longest and last rows) against the
    closed forms; normaliser S = number of terms (unit moduli)."""
    import mpmath
    import torch
    n = 512
    sys_ = synth.cyclic_roots_system(n, L)
    rows = [0, 1, 2, 7, 63, 127, 255, 256, 383, 449, 500, 507, 508, 509, 510, 511]
    W, Fr, Jr = _cyclic_roots_of_unity(n, rows)
    x = np.zeros((1, 2, L, n))
    with mpmath.workprec(200):
        for k in range(n):
            for part, val in ((0, W[k].real), (1, W[k].imag)):
                rem = val
                for l in range(L):
                    f = float(rem)
                    x[0, part, l, k] = f
                    rem -= f
    S = pe.System.from_sparse(sys_)
    F, J = S.eval(U.to_device(x))
    torch.cuda.synchronize()
    S.close()
    F, J = F.cpu().numpy()[0], J.cpu().numpy()[0]
    tol = U.tolerance(sys_)
    # F of every row: zero up to rounding, normalised by n terms of modulus 1
    with mpmath.workprec(200):
        def val(a):
            return mpmath.mpc(mpmath.fsum(mpmath.mpf(float(v)) for v in a[0]),
                              mpmath.fsum(mpmath.mpf(float(v)) for v in a[1]))
        eF = max(float(abs(val(F[:, :, r]))) / n for r in range(n - 1))
        eF = max(eF, float(abs(val(F[:, :, n - 1]) - Fr[n - 1])) / 2)
        eJ = 0.0
        for r in rows:
            scale = 1.0 if r == n - 1 else float(r + 1)
            for m in range(n):
                eJ = max(eJ, float(abs(val(J[:, :, r, m]) - Jr[r][m])) / scale)
    U.flush(f"cyclic512 roots of unity L={L}: eF={eF:.2e} eJ={eJ:.2e} tol={tol:.1e}")
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


@pytest.mark.parametrize("L", [1, 2])
def test_cyclic_512_random_point(pe, L):
    """Cyclic 512-roots at a random unit-circle point (the bench workload):
    18 sampled rows against the oracle -- full rows of J where the
    monomials are short, F and four columns on the long rows (up to the
    longest, 511 variables, and the last, 512)."""
    import torch
    n = 512
    sys_ = synth.cyclic_roots_system(n, L)
    x = synth.unit_circle_points(synth.rng_for((0, 1)), 1, n, L)
    S = pe.System.from_sparse(sys_)
    F, J = S.eval(U.to_device(x))
    torch.cuda.synchronize()
    S.close()
    F, J = F.cpu().numpy()[0], J.cpu().numpy()[0]
    picks = {r: range(n) for r in (0, 1, 2, 5, 15, 31)}
    for r in (63, 127, 200, 255, 256, 320, 400, 480, 509, 510, 511):
        picks[r] = [0, r // 2, (r + 7) % n, n - 1]
    picks[300] = list(range(0, n, 64))
    U.flush(f"cyclic512 random point L={L}: oracle over {len(picks)} rows")
    eF, eJ = U.max_errors_entries(sys_, x[0], F, J, picks)
    tol = U.tolerance(sys_)
    U.flush(f"cyclic512 random point L={L}: eF={eF:.2e} eJ={eJ:.2e} tol={tol:.1e}")
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


@pytest.mark.parametrize("level, n, k, words", [
    (2, 65536, 3, "65535"),
    (2, 1100, 1025, "more than 1024 variables"),
    (4, 600, 513, "too large for the segment"),
])
def test_size_limits_are_reported(pe, level, n, k, words):
    """The size limits of the header: more than 65535 variables, a monomial
    of more than 1024 variables and a quad-double monomial of 513 are refused
    with PE_EUNSUPPORTED through the C ABI, and nothing is created."""
    import ctypes
    sys_ = synth.random_system(5, level, n_vars=n, n_polys=2, m=2, k=k, exp_lo=1, exp_hi=2)
    h = ctypes.c_void_p()
    arrs = [np.ascontiguousarray(a) for a in (sys_.poly_ptr, sys_.mon_ptr, sys_.var_idx, sys_.exps, sys_.coef)]
    st = pe._lib.pe_system_create(ctypes.byref(h), level, n, sys_.n_polys, *[a.ctypes.data for a in arrs], None)
    assert st == pe.PE_EUNSUPPORTED, st
    assert words in pe._lib.pe_last_error().decode()
    assert not h.value
    # the largest sizes within the limits load and evaluate
    kmax = {1: 1024, 2: 1024, 4: 512}[level]
    ok = synth.random_system(6, level, n_vars=min(n, 4096), n_polys=1, m=1, k=min(k, kmax),
                             exp_lo=1, exp_hi=1)
    S = pe.System.from_sparse(ok)
    S.close()


def test_grid_limit_counts_column_tiles(pe):
    """One workgroup per (point, row, column tile) must stay below 2^31:
    with n = 4500 (three tiles of J) and N = 2, P = 400,000,000 points pass
    the P * N test alone but not with the tiles, so pe_eval refuses them
    before any launch (the buffers are never touched)."""
    import ctypes
    import torch
    sys_ = synth.random_system(7, 2, n_vars=4500, n_polys=2, m=3, k=3, exp_lo=1, exp_hi=2)
    S = pe.System.from_sparse(sys_)
    big = 400_000_000
    buf = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    st = pe._lib.pe_eval(S.handle, big, p, p, p, None)
    assert st == pe.PE_EUNSUPPORTED, st
    assert "column tiles" in pe._lib.pe_last_error().decode()
    S.close()
