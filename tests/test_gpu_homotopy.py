"""The Newton homotopy f(x) - t f(z) (Sec. 5.3) on the device: single
predictor and corrector steps against the oracle's, paths tracked from t = 1
to t = 0 against the oracle's tracker, and the paper's cyclic 512-roots run
(Newton at t just below 1 from a random z, complex double double)."""
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


def _start(sys_, seed, P):
    """Random unit-circle starts z and c = f(z) (exact, rounded to the level)."""
    L = sys_.level
    z = synth.unit_circle_points(synth.rng_for(seed), P, sys_.n_vars, L)
    c = np.stack([O.round_point(O.system_value_at(sys_, O.point_from_limbs(z[p])), L) for p in range(P)])
    return z, c


def _dist(x, Xref):
    return max(O.cdy_abs_float(O.cdy_add(O.cdy_from_limbs(x[0, :, j], x[1, :, j]), O.cdy_neg(Xref[j])))
               for j in range(x.shape[-1]))


@pytest.mark.parametrize("L", [2, 4])
def test_homotopy_steps_match_oracle(pe, L):
    """One Euler predictor (dt = -1/8) and one corrector (t = 7/8) from the
    same device point agree with the oracle's steps (Householder at 600 bits)
    to the level's rounding, at three points."""
    import torch
    sys_ = synth.random_system((901, L), L, n_vars=7, n_polys=7, m=5, k=3, exp_lo=1, exp_hi=2)
    P = 3
    z, c = _start(sys_, (902, L), P)
    S = pe.System.from_sparse(sys_)
    xd, cd = U.to_device(z), U.to_device(c)
    S.homotopy_predict(xd, cd, -0.125)
    torch.cuda.synchronize()
    xp = xd.cpu().numpy()
    S.homotopy_newton_step(xd, cd, 0.875)
    torch.cuda.synchronize()
    xc = xd.cpu().numpy()
    S.close()
    u = UNIT[L]
    for p in range(P):
        C = O.point_from_limbs(c[p])
        want_p = O.homotopy_step_mp(sys_, O.point_from_limbs(z[p]), C, 0.0, -0.125, prec=600)
        assert _dist(xp[p], want_p) <= 1e4 * u, (p, _dist(xp[p], want_p))
        want_c = O.homotopy_step_mp(sys_, O.point_from_limbs(xp[p]), C, 1.0, 0.875, prec=600)
        assert _dist(xc[p], want_c) <= 1e4 * u, (p, _dist(xc[p], want_c))


def _near_decoupled(seed, L, n=6, eps=0.25):
    """f_i = x_i^2 + eps (c1 x_{i+1} x_{i+2} + c2 x_{i+1}) - a_i with
    unit-circle a and c: quadratic, weakly coupled, so the paths of the
    Newton homotopy from unit-circle starts stay away from singular points
    and a fixed-step tracker reaches the roots (a random system's paths may
    not: a fixed-step tracker then ends where the oracle's does, off a
    root)."""
    rng = synth.rng_for(seed)
    a = np.exp(2j * np.pi * rng.random(n))
    cc = np.exp(2j * np.pi * rng.random((n, 2)))
    polys = []
    for i in range(n):
        j, k = (i + 1) % n, (i + 2) % n
        polys.append([(1.0, [(i, 2)]), (eps * cc[i, 0], sorted([(j, 1), (k, 1)])), (eps * cc[i, 1], [(j, 1)]),
                      (-a[i], [])])
    return synth.from_monomial_lists(L, n, polys)


@pytest.mark.parametrize("L", [2, 4])
def test_homotopy_track_matches_oracle(pe, L):
    """Paths of a weakly coupled quadratic system tracked from z (t = 1) to
    t = 0 in 8 steps with 5 correctors each, at four points: every end point
    equals the oracle's tracked end point and is a root of f (|f| / S at the
    rounding level, exactly)."""
    import torch
    sys_ = _near_decoupled((911, L), L)
    P = 4
    z, c = _start(sys_, (912, L), P)
    S = pe.System.from_sparse(sys_)
    xd = U.to_device(z)
    _, r = S.homotopy_track(xd, U.to_device(c), steps=8, corrector_iters=5)
    torch.cuda.synchronize()
    x = xd.cpu().numpy()
    S.close()
    u = UNIT[L]
    for p in range(P):
        end = O.homotopy_track_mp(sys_, O.point_from_limbs(z[p]), O.point_from_limbs(c[p]), 8, 5, prec=600)
        d = _dist(x[p], end)
        U.flush(f"homotopy L={L} path {p}: |x_gpu - x_oracle| = {d:.2e}")
        assert d <= 1e5 * u, (p, d)
        assert U.max_value_ratio(sys_, x[p], range(sys_.n_polys)) <= U.tolerance(sys_) * 64


def test_cyclic_512_newton_homotopy(pe):
    """The paper's run (Sec. 5.3): cyclic 512-roots, random z, Newton on
    f(x) - t f(z) = 0 from x = z in complex double double, for t close
    enough to 1 that Newton converges: at this z, J(z) has condition number
    about 5.5e6 and Newton in double precision diverges at t = 1 - 2^-10 but
    converges quadratically from t = 1 - 2^-18, which is taken here.  The
    right-hand side norm decays to the double-double level within seven
    iterations, and at the end |f(x) - t c| / S is at the tolerance on
    sampled rows, exactly (oracle)."""
    import torch
    n, L = 512, 2
    sys_ = synth.cyclic_roots_system(n, L)
    z = synth.unit_circle_points(synth.rng_for(921), 1, n, L)
    U.flush("cyclic512 homotopy: c = f(z) by the oracle")
    c = U.values_at(sys_, z[0])[None]
    t = 1.0 - 2.0 ** -18
    S = pe.System.from_sparse(sys_)
    xd, cd = U.to_device(z), U.to_device(c)
    ws = torch.empty((S.newton_workspace_bytes(1) + 7) // 8, dtype=torch.float64, device="cuda")
    norms = []
    for it in range(8):
        _, r = S.homotopy_newton_step(xd, cd, t, workspace=ws)
        torch.cuda.synchronize()
        norms.append(float(r.cpu().numpy()[0, 0]))
        U.flush(f"cyclic512 homotopy: iteration {it}: |f(x) - t c| = {norms[-1]:.3e}")
    S.close()
    assert norms[6] <= 1e-24 * norms[0], norms
    x = xd.cpu().numpy()[0]
    rows = [0, 1, 2, 100, 255, 400, 509, 510, 511]
    sub = U.row_subsystem(sys_, rows)
    csub = c[0][:, :, rows]
    e = U.max_shift_ratio(sub, x, csub, t)
    assert e <= U.tolerance(sys_), e
