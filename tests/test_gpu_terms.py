"""Per-monomial output (pe_eval_terms): every monomial's value and gradient
before the sum reduction (Sec. 2.2 Tables 1-2; Sec. 2.1 and 2.3 for the
coefficient, common factor and exponent), against the exact oracle."""
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


def _shuffled(sys_, seed):
    """The same system with each monomial's variables in a random input
    order (the library packs them sorted; the output must follow the
    input)."""
    rng = synth.rng_for(seed)
    perm = np.concatenate([rng.permutation(np.arange(a, b)) for a, b in zip(sys_.mon_ptr[:-1], sys_.mon_ptr[1:])])
    sys_.var_idx = np.ascontiguousarray(sys_.var_idx[perm])
    sys_.exps = np.ascontiguousarray(sys_.exps[perm])
    return sys_


def _check_terms(sys_, x, V, G, monomials, tol):
    """Every sampled monomial's value and partials against the oracle, in
    the metric |got - exact| / (the term's absolute value)."""
    T = O.eval_terms(sys_, x, monomials)
    A = O.abs_terms(sys_, x, monomials)
    worst = 0.0
    for t in monomials:
        v, g = T[t]
        sv, sg = A[t]
        worst = max(worst, O.rel_error(V[0, :, t], V[1, :, t], v, sv))
        o0 = int(sys_.mon_ptr[t])
        for r, (gr, s) in enumerate(zip(g, sg)):
            worst = max(worst, O.rel_error(G[0, :, o0 + r], G[1, :, o0 + r], gr, s))
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("L", [1, 2, 4])
def test_terms_match_oracle(pe, L):
    """Uneven random systems (monomials of 0 to 9 variables, exponents up to
    4, shuffled variable order, several chunks per row) at three points: all
    values and partials against the oracle; summed, they give pe_eval's F
    and J to the level's tolerance."""
    import torch
    rng = synth.rng_for((601, L))
    polys = []
    for p in range(23):
        mons = []
        for _ in range(int(rng.integers(1, 70))):
            k = int(rng.integers(0, 10))
            vs = rng.choice(40, size=k, replace=False)
            mons.append((complex(np.exp(2j * np.pi * rng.random())), [(int(v), int(rng.integers(1, 5))) for v in vs]))
        polys.append(mons)
    sys_ = synth.from_monomial_lists(L, 40, polys)
    sys_.coef = synth.unit_circle(synth.rng_for((602, L)), sys_.n_monomials, L)
    P = 3
    x = synth.unit_circle_points(synth.rng_for((603, L)), P, 40, L)
    S = pe.System.from_sparse(sys_)
    xd = U.to_device(x)
    V, G = S.eval_terms(xd)
    F, J = S.eval(xd)
    torch.cuda.synchronize()
    V, G, F, J = V.cpu().numpy(), G.cpu().numpy(), F.cpu().numpy(), J.cpu().numpy()
    S.close()
    tol = U.tolerance(sys_)
    for pt in range(P):
        w = _check_terms(sys_, x[pt], V[pt], G[pt], range(sys_.n_monomials), tol)
        U.flush(f"terms L={L} point {pt}: worst {w:.2e} (tolerance {tol:.0e})")
        # the terms summed exactly give F and J within the tolerance
        SF, SJ = O.abs_sums_rows(sys_, x[pt], range(sys_.n_polys))
        for p in range(sys_.n_polys):
            f, jrow = O.ZERO, {}
            for t in range(int(sys_.poly_ptr[p]), int(sys_.poly_ptr[p + 1])):
                f = O.cdy_add(f, O.cdy_from_limbs(V[pt, 0, :, t], V[pt, 1, :, t]))
                for o in range(int(sys_.mon_ptr[t]), int(sys_.mon_ptr[t + 1])):
                    j = int(sys_.var_idx[o])
                    g = O.cdy_from_limbs(G[pt, 0, :, o], G[pt, 1, :, o])
                    jrow[j] = O.cdy_add(jrow[j], g) if j in jrow else g
            assert O.rel_error(F[pt, 0, :, p], F[pt, 1, :, p], f, SF[p]) <= 2 * tol
            for j, g in jrow.items():
                assert O.rel_error(J[pt, 0, :, p, j], J[pt, 1, :, p, j], g, SJ[p][j]) <= 2 * tol


@pytest.mark.parametrize("L", [1, 2])
def test_terms_exact_regime_bit_exact(pe, L):
    """Exactly representable data: every value and partial equals the exact
    result bit for bit (lower limbs zero)."""
    import torch
    sys_ = _shuffled(synth.exact_regime_system(611, L, n_vars=12, n_polys=9, m=7, k=4, exp_hi=3), 612)
    x = synth.exact_regime_points(613, 2, 12, L)
    S = pe.System.from_sparse(sys_)
    V, G = S.eval_terms(U.to_device(x))
    torch.cuda.synchronize()
    V, G = V.cpu().numpy(), G.cpu().numpy()
    S.close()
    for pt in range(2):
        T = O.eval_terms(sys_, x[pt], range(sys_.n_monomials))
        for t, (v, g) in T.items():
            assert np.array_equal(V[pt, :, :, t], O.cdy_to_limbs(v, L)), (pt, t)
            o0 = int(sys_.mon_ptr[t])
            for r, gr in enumerate(g):
                assert np.array_equal(G[pt, :, :, o0 + r], O.cdy_to_limbs(gr, L)), (pt, t, r)


@pytest.mark.parametrize("n, m", [(1024, 1), (256, 4), (32, 32), (4, 256)])
def test_terms_table2_shapes(pe, n, m):
    """The shapes of Table 2 in complex double: blocks of 1,024 variables,
    each holding m products of n = 1024 / m distinct variables with
    coefficient 1 (here 64 blocks, one polynomial each): sampled monomials'
    values and gradients against the oracle, every output finite."""
    import torch
    blocks, nv = 64, 1024
    polys = []
    for b in range(blocks):
        polys.append([(1.0, [(i * n + r, 1) for r in range(n)]) for i in range(m)])
    sys_ = synth.from_monomial_lists(1, nv, polys)
    x = synth.unit_circle_points(synth.rng_for((621, n)), 1, nv, 1)
    S = pe.System.from_sparse(sys_)
    V, G = S.eval_terms(U.to_device(x))
    torch.cuda.synchronize()
    V, G = V.cpu().numpy()[0], G.cpu().numpy()[0]
    S.close()
    tol = U.tolerance(sys_)
    sample = sorted({0, m - 1, (blocks // 2) * m, blocks * m - 1})
    _check_terms(sys_, x[0], V, G, sample, tol)
    assert np.isfinite(V).all() and np.isfinite(G).all()
