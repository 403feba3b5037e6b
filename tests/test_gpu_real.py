"""Real arithmetic (level PE_REAL | L): evaluation, per-monomial terms,
Gauss-Newton and least squares on real data in real double, double double
and quad double (Sec. 2.2 notes real double double; Sec. 5.2 Table 4 runs
Newton in real quad double).  The oracle is the exact complex oracle on the
same data with zero imaginary parts: the exact results are then real."""
import numpy as np
import pytest

import gpu_util as U
import oracle as O
from paper_1402_2626_amd import synth

pytestmark = pytest.mark.gpu

UNIT = {1: 2.0 ** -53, 2: 2.0 ** -104, 4: 2.0 ** -206}


@pytest.fixture(scope="module")
def pe():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1402_2626_amd import polyeval
    return polyeval


def _realify(sys_):
    """The same structure with real coefficients: the real parts of the
    unit-circle ones (values in [-1, 1], every limb populated)."""
    c = np.zeros_like(sys_.coef)
    c[0] = sys_.coef[0]
    sys_.coef = c
    return sys_


def _real_points(seed, P, n, L):
    """[P, 2, L, n] real points (imaginary parts zero), values in [-1, 1]."""
    x = synth.unit_circle_points(synth.rng_for(seed), P, n, L)
    x[:, 1] = 0.0
    return x


def _device_system(pe, sys_):
    """A real device system from a complex PolySystem with zero imaginary
    coefficients."""
    return pe.System(pe.PE_REAL | sys_.level, sys_.n_vars, sys_.poly_ptr, sys_.mon_ptr, sys_.var_idx, sys_.exps,
                     np.ascontiguousarray(sys_.coef[:1]))


def _complexify(a):
    """[P, 1, ...] real outputs -> [P, 2, ...] with zero imaginary parts."""
    return np.concatenate([a, np.zeros_like(a)], axis=1)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_real_eval_matches_oracle(pe, L):
    """F and J of a real random system (exponents up to 4, several chunks per
    row) at three real points, every row against the oracle."""
    import torch
    sys_ = _realify(synth.random_system((701, L), L, n_vars=60, n_polys=45, m=40, k=7, exp_lo=1, exp_hi=4))
    x = _real_points((702, L), 3, 60, L)
    S = _device_system(pe, sys_)
    F, J = S.eval(U.to_device(x[:, :1]))
    torch.cuda.synchronize()
    F, J = _complexify(F.cpu().numpy()), _complexify(J.cpu().numpy())
    S.close()
    tol = U.tolerance(sys_)
    for pt in range(3):
        eF, eJ = U.max_errors_rows(sys_, x[pt], F[pt], J[pt], range(sys_.n_polys))
        U.flush(f"real L={L} point {pt}: F {eF:.2e}, J {eJ:.2e} (tolerance {tol:.0e})")
        assert eF <= tol and eJ <= tol, (pt, eF, eJ)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_real_exact_regime_bit_exact(pe, L):
    """Small integer coefficients and points +-2^a: F, J and the terms equal
    the exact values bit for bit (lower limbs zero)."""
    import torch
    sys_ = synth.exact_regime_system(711, L, n_vars=30, n_polys=20, m=10, k=5, exp_hi=3)
    sys_.coef[1] = 0.0
    sys_.coef[0] = np.where(sys_.coef[0] == 0.0, 1.0, sys_.coef[0])
    x = synth.exact_regime_points(712, 2, 30, L)
    x[:, 0] = np.where(x[:, 0] == 0.0, x[:, 1], x[:, 0])  # +-i 2^a becomes +-2^a
    x[:, 1] = 0.0
    S = _device_system(pe, sys_)
    xd = U.to_device(x[:, :1])
    F, J = S.eval(xd)
    V, G = S.eval_terms(xd)
    torch.cuda.synchronize()
    F, J, V, G = (_complexify(a.cpu().numpy()) for a in (F, J, V, G))
    S.close()
    for pt in range(2):
        Fx, Jx = O.eval_system(sys_, x[pt])
        for p in range(sys_.n_polys):
            assert np.array_equal(F[pt, :, :, p], O.cdy_to_limbs(Fx[p], L)), (pt, p)
            for j in range(sys_.n_vars):
                assert np.array_equal(J[pt, :, :, p, j], O.cdy_to_limbs(Jx[p].get(j, O.ZERO), L)), (pt, p, j)
        T = O.eval_terms(sys_, x[pt], range(sys_.n_monomials))
        for t, (v, g) in T.items():
            assert np.array_equal(V[pt, :, :, t], O.cdy_to_limbs(v, L)), (pt, t)
            o0 = int(sys_.mon_ptr[t])
            for r, gr in enumerate(g):
                assert np.array_equal(G[pt, :, :, o0 + r], O.cdy_to_limbs(gr, L)), (pt, t, r)


@pytest.mark.parametrize("L", [2, 4])
def test_real_terms_match_oracle(pe, L):
    """Per-monomial values and gradients of a real system against the
    oracle, at two real points."""
    import torch
    sys_ = _realify(synth.random_system((721, L), L, n_vars=33, n_polys=12, m=20, k=6, exp_lo=1, exp_hi=3))
    x = _real_points((722, L), 2, 33, L)
    S = _device_system(pe, sys_)
    V, G = S.eval_terms(U.to_device(x[:, :1]))
    torch.cuda.synchronize()
    V, G = _complexify(V.cpu().numpy()), _complexify(G.cpu().numpy())
    S.close()
    tol = U.tolerance(sys_)
    for pt in range(2):
        T = O.eval_terms(sys_, x[pt], range(sys_.n_monomials))
        A = O.abs_terms(sys_, x[pt], range(sys_.n_monomials))
        for t, (v, g) in T.items():
            assert O.rel_error(V[pt, 0, :, t], V[pt, 1, :, t], v, A[t][0]) <= tol
            o0 = int(sys_.mon_ptr[t])
            for r, (gr, sg) in enumerate(zip(g, A[t][1])):
                assert O.rel_error(G[pt, 0, :, o0 + r], G[pt, 1, :, o0 + r], gr, sg) <= tol


@pytest.mark.parametrize("L, n", [(4, 64), (4, 256), (2, 1024), (4, 2600)])
def test_real_newton_chandrasekhar(pe, L, n):
    """Chandrasekhar's H-equation (Sec. 5.2, c = 33/64) in real quad double
    (the setting of Table 4; n = 64 on the one-workgroup solve, n = 256 on
    the column-parallel one, n = 2600 on its 384-thread shape) and real
    double double at n = 1024, from H = 1:
    at n = 64 the first step equals the oracle's Gauss-Newton step
    (Householder at 600 bits) to the level's accuracy, the iterates converge quadratically to the
    level's floor, and at the end F is zero to the tolerance on sampled rows
    (oracle) with H real and above 1."""
    import torch
    sys_ = synth.chandrasekhar_system(n, L)
    x0 = np.zeros((2, L, n))
    x0[0, 0, :] = 1.0
    S = _device_system(pe, sys_)
    xd = U.to_device(x0[None, :1])
    ws = torch.empty((S.newton_workspace_bytes(1) + 7) // 8, dtype=torch.float64, device="cuda")
    iterates, res = [x0], []
    for it in range(6 if L == 2 else 8):
        _, r = S.newton_step(xd, workspace=ws)
        torch.cuda.synchronize()
        iterates.append(_complexify(xd.cpu().numpy())[0])
        res.append(r.cpu().numpy()[0].copy())
        U.flush(f"real chandrasekhar n={n} L={L}: step {it}: |F| = {res[-1][0]:.3e}, |dx| = {res[-1][1]:.3e}")
    S.close()
    u = UNIT[L]
    if n <= 64:
        want, _ = O.gauss_newton_step_mp(sys_, O.point_from_limbs(x0), prec=600)
        d = max(O.cdy_abs_float(O.cdy_add(O.cdy_from_limbs(iterates[1][0, :, j], iterates[1][1, :, j]),
                                          O.cdy_neg(want[j]))) for j in range(n))
        assert d <= 1e4 * n * u, d
    last = O.point_from_limbs(iterates[-1])
    errs = [max(O.cdy_abs_float(O.cdy_add(O.cdy_from_limbs(x[0, :, j], x[1, :, j]), O.cdy_neg(last[j])))
                for j in range(n)) for x in iterates[:-1]]
    for a, b in zip(errs, errs[1:]):
        assert b <= 1e4 * a * a + 1e5 * u, errs
    assert errs[-1] <= 1e5 * u, errs
    rows = [0, 1, n // 2, n - 2, n - 1]
    eF = U.max_value_ratio(U.row_subsystem(sys_, rows), iterates[-1], range(len(rows)))
    assert eF <= U.tolerance(sys_) * 8, eF
    assert np.all(iterates[-1][0, 0] > 1.0)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_real_lstsq_matches_oracle(pe, L):
    """Overdetermined real least squares (N = 50, n = 37, two problems, and
    N = 700, n = 300 on the column-parallel sweep): x against the oracle's
    Householder solve within c N kappa u_L |x|."""
    import torch
    for (N, n, P, seed) in ((50, 37, 2, 731), (700, 300, 1, 732)):
        rng = synth.rng_for((seed, L))
        Ab = np.stack([synth.unit_circle(rng, N * (n + 1), L).reshape(2, L, N, n + 1) for _ in range(P)])
        Ab[:, 1] = 0.0
        x, resid, _, _ = pe.lstsq(U.to_device(Ab[:, :1]))
        torch.cuda.synchronize()
        x, resid = _complexify(x.cpu().numpy()), resid.cpu().numpy()
        for pt in range(P):
            A = Ab[pt, 0, 0, :, :n]
            s = np.linalg.svd(A, compute_uv=False)
            kappa = s[0] / s[-1]
            if n <= 40:
                xs = O.lstsq_limbs(Ab[pt], prec=400)
                xn = max(O.cdy_abs_float(v) for v in xs)
                err = max(O.cdy_abs_float(O.cdy_add(O.cdy_from_limbs(x[pt, 0, :, j], x[pt, 1, :, j]),
                                                    O.cdy_neg(xs[j]))) for j in range(n))
                assert err <= 10 * N * kappa * UNIT[L] * xn, (pt, err, xn, kappa)
            else:
                want = np.linalg.lstsq(A, Ab[pt, 0, 0, :, n], rcond=None)[0]
                got = x[pt, 0, 0]
                assert np.max(np.abs(got - want)) <= 1e3 * kappa * 2.0 ** -53 * np.max(np.abs(want))
            assert resid[pt, 1] > 0.0


def test_real_rejections(pe):
    """Real systems are not batched and have no adjoint: PE_EUNSUPPORTED."""
    import torch
    sys_ = _realify(synth.random_system(741, 2, n_vars=8, n_polys=8, m=3, k=2))
    S = _device_system(pe, sys_)
    x = torch.zeros((1, 1, 2, 8), dtype=torch.float64, device="cuda")
    v = torch.zeros((1, 1, 2, 8), dtype=torch.float64, device="cuda")
    g = torch.zeros_like(x)
    import ctypes
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert pe._lib.pe_eval_adjoint(S.handle, 1, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                   ctypes.c_void_p(g.data_ptr()), st) == pe.PE_EUNSUPPORTED
    with pytest.raises(pe.PolyevalError):
        pe.Batch([S])
    S.close()
