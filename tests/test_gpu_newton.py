"""Gauss-Newton steps on the device (MGS on [A b], back substitution, update)."""
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


def _dist(x, Xs, L):
    """max_j |x_j - x*_j| exactly, x: [2, L, n] limbs, Xs exact values."""
    return max(O.cdy_abs_float(O.cdy_add(O.cdy_from_limbs(x[0, :, j], x[1, :, j]), O.cdy_neg(Xs[j])))
               for j in range(x.shape[-1]))


@pytest.mark.parametrize("L", [2, 4])
def test_newton_small_matches_oracle(pe, L):
    """Square planted system (n = N = 10): each device iterate agrees with
    the oracle's Gauss-Newton iterate (Householder QR at 512 bits) from the
    same start, and the error to x* decays quadratically."""
    import torch
    sys_ = synth.random_system(201, L, n_vars=10, n_polys=10, m=6, k=3, exp_lo=1, exp_hi=3)
    xs = synth.unit_circle_points(synth.rng_for(202), 1, 10, L)[0]
    planted = O.plant_root(sys_, xs)
    x0 = synth.perturbed_start(203, xs, 1e-4)
    S = pe.System.from_sparse(planted)
    xd = U.to_device(x0[None])
    Xo = O.point_from_limbs(x0)
    Xs = O.point_from_limbs(xs)
    u = 2.0 ** (-53 * L)
    errs = []
    for it in range(5):
        _, resid = S.newton_step(xd)
        torch.cuda.synchronize()
        Xo, _ = O.gauss_newton_step_mp(planted, Xo, prec=600)
        xg = xd.cpu().numpy()[0]
        dev = max(O.cdy_abs_float(O.cdy_add(O.cdy_from_limbs(xg[0, :, j], xg[1, :, j]), O.cdy_neg(Xo[j])))
                  for j in range(10))
        errs.append(_dist(xg, Xs, L))
        assert dev <= 1e4 * u + 1e-3 * errs[-1], (it, dev, errs)
        r = resid.cpu().numpy()[0]
        assert r[1] >= 0.0
    for a, b in zip(errs, errs[1:]):
        assert b <= 1e4 * a * a + 1e4 * u, errs  # quadratic down to the floor
    assert errs[-1] <= 1e4 * u, errs
    S.close()


def test_newton_dd_n256_planted(pe):
    """Complex double double, n = N = 256 (256 monomials of k = 16, exponents
    1..4), root planted at the generated point, start x* + 1e-6 noise:
    quadratic convergence to the double-double floor."""
    import torch
    sys_, x = synth.workload("dd_n256")
    U.flush("newton dd_n256: planting the root (oracle)")
    planted = O.plant_root(sys_, x[0])
    x0 = synth.perturbed_start(1, x[0], 1e-6)
    S = pe.System.from_sparse(planted)
    xd = U.to_device(x0[None])
    Xs = O.point_from_limbs(x[0])
    errs, res = [], []
    ws = None
    import torch as _t
    ws = _t.empty((S.newton_workspace_bytes(1) + 7) // 8, dtype=_t.float64, device="cuda")
    for it in range(4):
        U.flush(f"newton dd_n256: step {it}")
        _, r = S.newton_step(xd, workspace=ws)
        torch.cuda.synchronize()
        errs.append(_dist(xd.cpu().numpy()[0], Xs, 2))
        res.append(r.cpu().numpy()[0].copy())
    U.flush(f"newton dd_n256: errors {errs}, residuals {res}")
    # quadratic decay (e1 <= C e0^2) down to the double-double floor
    assert errs[0] <= 1e-8 and errs[1] <= 1e4 * errs[0] ** 2 and errs[-1] <= 1e-29, errs
    assert res[0][0] > res[1][0] > res[2][0]
    S.close()



@pytest.mark.parametrize("L", [1, 2, 4])
def test_newton_chandrasekhar_from_one(pe, L):
    """Chandrasekhar's H-equation (Sec. 5.2, c = 33/64, n = 24, coefficients
    rounded to double) from H = 1, where the paper reports quadratic
    convergence: every device iterate follows the oracle's Gauss-Newton
    iterate (Householder QR at 600 bits) from the same start, the error to the
    oracle's converged solution decays quadratically to the level's floor, and
    the solution is real with every H_i > 1."""
    import torch
    n = 24
    sys_ = synth.chandrasekhar_system(n, L)
    x0 = np.zeros((2, L, n))
    x0[0, 0, :] = 1.0
    Xo = O.point_from_limbs(x0)
    Xs = Xo
    for _ in range(8):  # 8 oracle steps: error below 1e-170
        Xs, _ = O.gauss_newton_step_mp(sys_, Xs, prec=600)
    S = pe.System.from_sparse(sys_)
    xd = U.to_device(x0[None])
    u = 2.0 ** (-53 * L)
    errs = []
    for it in range(7 if L == 4 else 6):
        S.newton_step(xd)
        torch.cuda.synchronize()
        Xo, _ = O.gauss_newton_step_mp(sys_, Xo, prec=600)
        xg = xd.cpu().numpy()[0]
        errs.append(_dist(xg, Xs, L))
        dev = _dist(xg, Xo, L)
        assert dev <= 1e4 * u + 1e-3 * errs[-1], (it, dev, errs)
    for a, b in zip(errs, errs[1:]):
        assert b <= 1e4 * a * a + 1e4 * u, errs
    assert errs[-1] <= 1e4 * u, errs
    xg = xd.cpu().numpy()[0]
    assert np.all(xg[0, 0] > 1.0) and np.all(np.abs(xg[1, 0]) <= 1e4 * u), xg[:, 0]
    S.close()

def test_newton_overdetermined(pe):
    """N = 16 > n = 9, consistent (planted): converges to x*."""
    import torch
    sys_ = synth.random_system(211, 2, n_vars=9, n_polys=16, m=5, k=3, exp_lo=1, exp_hi=2)
    xs = synth.unit_circle_points(synth.rng_for(212), 1, 9, 2)[0]
    planted = O.plant_root(sys_, xs)
    S = pe.System.from_sparse(planted)
    xd = U.to_device(synth.perturbed_start(213, xs, 1e-5)[None])
    for _ in range(4):
        S.newton_step(xd)
    torch.cuda.synchronize()
    assert _dist(xd.cpu().numpy()[0], O.point_from_limbs(xs), 2) <= 1e-28
    S.close()


def test_newton_singular_flags(pe):
    """Two identical linear equations in two variables: J is singular, the
    step is skipped (x unchanged) and the residual slot reports -1."""
    import torch
    polys = [[(1.0, [(0, 1)]), (1.0, [(1, 1)]), (-1.0, [])], [(1.0, [(0, 1)]), (1.0, [(1, 1)]), (-1.0, [])]]
    sys_ = synth.from_monomial_lists(2, 2, polys)
    S = pe.System.from_sparse(sys_)
    x0 = np.zeros((1, 2, 2, 2))
    x0[0, 0, 0] = [0.3, 0.2]
    xd = U.to_device(x0)
    _, r = S.newton_step(xd)
    torch.cuda.synchronize()
    assert r.cpu().numpy()[0, 1] == -1.0
    assert np.array_equal(xd.cpu().numpy(), x0)
    S.close()


def test_newton_graph_replay(pe):
    """A captured HIP graph of one Newton step, replayed several times with
    eager work in between, gives bitwise the same iterates as eager steps."""
    import torch
    sys_ = synth.random_system(221, 2, n_vars=24, n_polys=24, m=10, k=4, exp_lo=1, exp_hi=3)
    xs = synth.unit_circle_points(synth.rng_for(222), 1, 24, 2)[0]
    planted = O.plant_root(sys_, xs)
    S = pe.System.from_sparse(planted)
    x0 = synth.perturbed_start(223, xs, 1e-4)[None]
    P = 1
    ws = torch.empty((S.newton_workspace_bytes(P) + 7) // 8, dtype=torch.float64, device="cuda")
    resid = torch.empty((P, 2), dtype=torch.float64, device="cuda")
    # eager reference
    xe = U.to_device(x0)
    eager = []
    for _ in range(3):
        S.newton_step(xe, workspace=ws, resid=resid)
        torch.cuda.synchronize()
        eager.append(xe.cpu().numpy().copy())
    # graph
    xg = U.to_device(x0)
    s = torch.cuda.Stream()
    S.newton_step(xg.clone(), workspace=ws, resid=resid, stream=s)  # warm up on the side stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        S.newton_step(xg, workspace=ws, resid=resid, stream=s)
    xg.copy_(U.to_device(x0))
    torch.cuda.synchronize()
    for it in range(3):
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk
        assert np.array_equal(xg.cpu().numpy(), eager[it]), it
    S.close()
