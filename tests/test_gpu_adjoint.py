"""The adjoint J^H v (fused, J never formed) and the autograd Function."""
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


def _jhv_exact(J, v, L):
    """Exact g_j = sum_p conj(J_pj) v_p from limb arrays J[2, L, N, n], v[2, L, N]."""
    N, n = J.shape[2], J.shape[3]
    V = [O.cdy_from_limbs(v[0, :, p], v[1, :, p]) for p in range(N)]
    out = []
    for j in range(n):
        g = O.ZERO
        for p in range(N):
            jp = O.cdy_from_limbs(J[0, :, p, j], J[1, :, p, j])
            g = O.cdy_add(g, O.cdy_mul(O.cdy_conj(jp), V[p]))
        out.append(g)
    return out


def _adjoint_scale(sys_, x, v, cols):
    """Normaliser of the adjoint metric: sum_p S_J(p, j) |v_p|."""
    Sc = O.abs_sums_columns(sys_, x, cols)
    av = np.hypot(v[0].sum(axis=0), v[1].sum(axis=0))
    return {j: sum(s * av[p] for p, s in Sc[j].items()) for j in cols}


@pytest.mark.parametrize("L", [1, 2, 4])
def test_adjoint_matches_explicit_and_oracle(pe, L):
    import torch
    sys_ = synth.random_system(91, L, n_vars=40, n_polys=70, m=20, k=6, exp_lo=1, exp_hi=3)
    P = 3
    x = synth.unit_circle_points(synth.rng_for(92), P, 40, L)
    v = synth.unit_circle_points(synth.rng_for(93), P, 70, L)
    S = pe.System.from_sparse(sys_)
    xd, vd = U.to_device(x), U.to_device(v)
    g = S.adjoint(xd, vd)
    F, J = S.eval(xd)
    torch.cuda.synchronize()
    g, J = g.cpu().numpy(), J.cpu().numpy()
    S.close()
    tol = U.tolerance(sys_)
    cols = list(range(40))
    for pt in range(P):
        scale = _adjoint_scale(sys_, x[pt], v[pt], cols)
        exact = O.adjoint_columns(sys_, x[pt], v[pt], cols)
        for j in cols:
            e = O.rel_error(g[pt, 0, :, j], g[pt, 1, :, j], exact[j], scale[j])
            assert e <= tol, (pt, j, e)
        # the explicit route: J from pe_eval, then J^H v exactly
        ex2 = _jhv_exact(J[pt], v[pt], L)
        for j in cols:
            e = O.rel_error(g[pt, 0, :, j], g[pt, 1, :, j], ex2[j], scale[j])
            assert e <= 4 * tol, (pt, j, e)


def test_adjoint_dd_1024x512_sampled(pe):
    """Overdetermined DD system N = 1024, n = 512, 512 monomials of k = 24,
    64 points: sampled columns at two points against the oracle, and one
    point against J^H v from the explicit Jacobian."""
    import torch
    sys_, x = synth.workload("dd_adjoint_1024x512")
    v = synth.adjoint_vectors(0, x.shape[0], sys_.n_polys, sys_.level)
    S = pe.System.from_sparse(sys_)
    xd, vd = U.to_device(x), U.to_device(v)
    U.flush("adjoint 1024x512: device")
    g = S.adjoint(xd, vd)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    tol = U.tolerance(sys_)
    cols = [0, 129, 511]
    for pt in (0, 63):
        U.flush(f"adjoint 1024x512: oracle columns at point {pt}")
        scale = _adjoint_scale(sys_, x[pt], v[pt], cols)
        exact = O.adjoint_columns(sys_, x[pt], v[pt], cols)
        for j in cols:
            e = O.rel_error(g[pt, 0, :, j], g[pt, 1, :, j], exact[j], scale[j])
            assert e <= tol, (pt, j, e)
    # explicit J at point 5, J^H v in float64 on the leading limbs
    F, J = S.eval(xd[5:6])
    torch.cuda.synchronize()
    J = J.cpu().numpy()[0]
    Jc = J[0, 0] + 1j * J[1, 0]
    vc = v[5, 0, 0] + 1j * v[5, 1, 0]
    want = Jc.conj().T @ vc
    got = g[5, 0, 0] + 1j * g[5, 1, 0]
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))
    S.close()


def test_autograd_function(pe):
    """PolyEval.apply: forward F, backward J^H grad; gradcheck in double and
    the Gauss-Newton gradient of 1/2 |F|^2 in double double."""
    import torch
    from paper_1402_2626_amd.autograd import PolyEval

    sys1 = synth.random_system(95, 1, n_vars=6, n_polys=5, m=4, k=3, exp_lo=1, exp_hi=3)
    S1 = pe.System.from_sparse(sys1)
    x1 = U.to_device(synth.unit_circle_points(synth.rng_for(96), 2, 6, 1)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: PolyEval.apply(t, S1), (x1,), eps=1e-6, atol=1e-7)

    sys2 = synth.random_system(97, 2, n_vars=12, n_polys=16, m=8, k=4, exp_lo=1, exp_hi=3)
    S2 = pe.System.from_sparse(sys2)
    x2 = synth.unit_circle_points(synth.rng_for(98), 1, 12, 2)
    xt = U.to_device(x2).requires_grad_(True)
    F = PolyEval.apply(xt, S2)
    F.backward(F.detach())  # g = F: gradient of 1/2 |F|^2 is J^H F
    got = xt.grad.cpu().numpy()[0]
    Fn = F.detach().cpu().numpy()[0]
    Fx, Jx = O.eval_system(sys2, x2[0])
    Vex = [O.cdy_from_limbs(Fn[0, :, p], Fn[1, :, p]) for p in range(16)]
    want = O.adjoint_exact(Jx, Vex, 12)
    scale = _adjoint_scale(sys2, x2[0], Fn, range(12))
    for j in range(12):
        assert O.rel_error(got[0, :, j], got[1, :, j], want[j], scale[j]) <= 1e-28


def test_adjoint_finite_differences(pe):
    """Re<J^H v, w> equals the derivative of Re<v, F(x + h w)> at h = 0, by
    exact central differences in the oracle (h = 2^-70)."""
    import torch
    L = 4
    sys_ = synth.random_system(99, L, n_vars=10, n_polys=14, m=6, k=4, exp_lo=1, exp_hi=3)
    x = synth.unit_circle_points(synth.rng_for(100), 1, 10, L)
    v = synth.unit_circle_points(synth.rng_for(101), 1, 14, L)
    w = synth.unit_circle_points(synth.rng_for(102), 1, 10, 1)[0, :, 0]  # double direction
    S = pe.System.from_sparse(sys_)
    g = S.adjoint(U.to_device(x), U.to_device(v))
    torch.cuda.synchronize()
    g = g.cpu().numpy()[0]
    S.close()
    X = O.point_from_limbs(x[0])
    V = O.point_from_limbs(v[0])
    W = [O.cdy_from_limbs([w[0, j]], [w[1, j]]) for j in range(10)]
    h = -70

    def re_inner(F):
        acc = O.ZERO
        for p in range(14):
            acc = O.cdy_add(acc, O.cdy_mul(O.cdy_conj(V[p]), F[p]))
        return acc

    Xp = [O.cdy_add(X[j], (W[j][0], W[j][1], W[j][2] + h)) for j in range(10)]
    Xm = [O.cdy_add(X[j], (-W[j][0], -W[j][1], W[j][2] + h)) for j in range(10)]
    d = O.cdy_add(re_inner(O.system_value_at(sys_, Xp)), O.cdy_neg(re_inner(O.system_value_at(sys_, Xm))))
    fd = (d[0], 0, d[2] - h - 1)  # Re of the difference quotient, exact
    G = [O.cdy_from_limbs(g[0, :, j], g[1, :, j]) for j in range(10)]
    acc = O.ZERO
    for j in range(10):
        acc = O.cdy_add(acc, O.cdy_mul(O.cdy_conj(G[j]), W[j]))
    lhs = (acc[0], 0, acc[2])  # Re<J^H v, w>, exact from the GPU limbs
    diff = O.cdy_abs_float(O.cdy_add(lhs, O.cdy_neg(fd)))
    assert diff <= 1e-35 * max(1.0, O.cdy_abs_float(fd)), diff


def test_autograd_dd_1024x512(pe):
    """PolyEval.apply at the adjoint workload's shape (N = 1024, n = 512, 512
    monomials of k = 24, 64 points): forward F on sampled rows and the
    backward J^H v on sampled columns at two points against the oracle."""
    import torch
    from paper_1402_2626_amd.autograd import PolyEval

    sys_, x = synth.workload("dd_adjoint_1024x512")
    P = x.shape[0]
    v = synth.adjoint_vectors(0, P, sys_.n_polys, sys_.level)
    S = pe.System.from_sparse(sys_)
    xt = U.to_device(x).requires_grad_(True)
    U.flush("autograd 1024x512: forward and backward")
    F = PolyEval.apply(xt, S)
    F.backward(U.to_device(v))
    torch.cuda.synchronize()
    g = xt.grad.cpu().numpy()
    Fn = F.detach().cpu().numpy()
    S.close()
    tol = U.tolerance(sys_)
    cols = [3, 256, 510]
    for pt in (1, 62):
        U.flush(f"autograd 1024x512: oracle at point {pt}")
        eF, _ = U.max_errors_entries(sys_, x[pt], Fn[pt], np.zeros((2, 2, sys_.n_polys, 1)),
                                     {0: [], 511: [], 1023: []})
        assert eF <= tol, (pt, eF)
        scale = _adjoint_scale(sys_, x[pt], v[pt], cols)
        exact = O.adjoint_columns(sys_, x[pt], v[pt], cols)
        for j in cols:
            e = O.rel_error(g[pt, 0, :, j], g[pt, 1, :, j], exact[j], scale[j])
            assert e <= tol, (pt, j, e)
