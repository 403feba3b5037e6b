"""Monomials wider than the default segment allows: double double up to 1024
variables (segment 16) and quad double up to 512 (segment 8), chosen by
default when a system needs them; cyclic n-roots in quad double at n = 448
(the largest QD case of the paper's Table 5)."""
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


def test_cyclic_qd_448(pe):
    """Cyclic 448-roots (eq. (5)) in complex quad double: the default segment
    becomes 8 (monomials of up to 448 variables in 56 lanes); at x = 1 F and
    J equal their closed forms bit for bit (F_i = n for i < n, F_n = 0,
    J_{i,m} = i, last row all ones); at a random unit-circle point sampled
    rows match the oracle (full rows where monomials are short, F and four
    columns on the long rows up to the longest)."""
    import torch
    n, L = 448, 4
    sys_ = synth.cyclic_roots_system(n, L)
    S = pe.System.from_sparse(sys_)
    assert S.info()["segment"] == 8
    one = np.zeros((1, 2, L, n))
    one[0, 0, 0] = 1.0
    F, J = S.eval(U.to_device(one))
    torch.cuda.synchronize()
    F, J = F.cpu().numpy()[0], J.cpu().numpy()[0]
    wantF = np.zeros((2, L, n))
    wantF[0, 0, :n - 1] = n
    assert np.array_equal(F, wantF)
    wantJ = np.zeros((2, L, n, n))
    wantJ[0, 0, :n - 1, :] = np.arange(1, n)[:, None]
    wantJ[0, 0, n - 1, :] = 1.0
    assert np.array_equal(J, wantJ)
    x = synth.unit_circle_points(synth.rng_for((0, 1)), 1, n, L)
    F, J = S.eval(U.to_device(x))
    torch.cuda.synchronize()
    S.close()
    F, J = F.cpu().numpy()[0], J.cpu().numpy()[0]
    picks = {r: range(n) for r in (0, 1, 4, 15)}
    for r in (63, 200, 300, 445, 446, 447):
        picks[r] = [0, r // 2, (r + 7) % n, n - 1]
    U.flush(f"cyclic448 QD random point: oracle over {len(picks)} rows")
    eF, eJ = U.max_errors_entries(sys_, x[0], F, J, picks)
    tol = U.tolerance(sys_)
    U.flush(f"cyclic448 QD: eF={eF:.2e} eJ={eJ:.2e} tol={tol:.1e}")
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


@pytest.mark.parametrize("level, k, seg", [(2, 1024, 16), (2, 700, 16), (4, 512, 8), (4, 300, 8)])
def test_wide_monomials(pe, level, k, seg):
    """Products of k variables (exponent 1) at the level's widest segment,
    three polynomials of two monomials each at a random point: every row
    against the oracle, and Euler's identity sum_j x_j J_pj = k F_p on the
    exact values."""
    import torch
    n = 1024 if k > 512 else 512
    sys_ = synth.random_system((751, level, k), level, n_vars=n, n_polys=3, m=2, k=k, exp_lo=1, exp_hi=1)
    S = pe.System.from_sparse(sys_)
    assert S.info()["segment"] == seg
    x = synth.unit_circle_points(synth.rng_for((752, k)), 1, n, level)
    F, J = S.eval(U.to_device(x))
    torch.cuda.synchronize()
    S.close()
    F, J = F.cpu().numpy()[0], J.cpu().numpy()[0]
    picks = {p: [0, 1, n // 2, n - 1] + list(range(5, n, 97)) for p in range(3)}
    eF, eJ = U.max_errors_entries(sys_, x[0], F, J, picks)
    tol = U.tolerance(sys_)
    assert eF <= tol and eJ <= tol, (eF, eJ, tol)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_wide_rows_in_column_tiles(pe, L):
    """Rows of J wider than 2048 columns (n = 4500: three tiles of 2048
    columns, one workgroup each): every row of F and J at two points against
    the oracle, and F of the F-only evaluation (one workgroup per row, F from
    the forward products) too; the per-monomial output of sampled monomials
    too; the adjoint and batches refuse the system."""
    import torch
    n = 4500
    sys_ = synth.random_system((761, L), L, n_vars=n, n_polys=6, m=150, k=5, exp_lo=1, exp_hi=3)
    x = synth.unit_circle_points(synth.rng_for((762, L)), 2, n, L)
    S = pe.System.from_sparse(sys_)
    xd = U.to_device(x)
    F, J = S.eval(xd)
    F2, _ = S.eval(xd, want_J=False)
    torch.cuda.synchronize()
    F, J, F2 = F.cpu().numpy(), J.cpu().numpy(), F2.cpu().numpy()
    tol = U.tolerance(sys_)
    for pt in range(2):
        eF, eJ = U.max_errors_rows(sys_, x[pt], F[pt], J[pt], range(sys_.n_polys))
        eF2, _ = U.max_errors_rows(sys_, x[pt], F2[pt], J[pt], range(sys_.n_polys))
        U.flush(f"wide rows L={L} point {pt}: eF={eF:.2e} eJ={eJ:.2e} F-only {eF2:.2e} tol={tol:.1e}")
        assert eF <= tol and eJ <= tol and eF2 <= tol, (pt, eF, eJ, eF2)
    # the per-monomial output of the same wide system (no column tiles:
    # every partial goes to its input position), sampled monomials of the
    # first and last rows against the oracle at both points
    V, Gt = S.eval_terms(xd)
    torch.cuda.synchronize()
    V, Gt = V.cpu().numpy(), Gt.cpu().numpy()
    mons = sorted({0, 1, int(sys_.poly_ptr[1]) - 1, sys_.n_monomials - 2, sys_.n_monomials - 1})
    for pt in range(2):
        T = O.eval_terms(sys_, x[pt], mons)
        A = O.abs_terms(sys_, x[pt], mons)
        worst = 0.0
        for t in mons:
            v, g = T[t]
            worst = max(worst, O.rel_error(V[pt, 0, :, t], V[pt, 1, :, t], v, A[t][0]))
            o0 = int(sys_.mon_ptr[t])
            for r, (gr, sg) in enumerate(zip(g, A[t][1])):
                worst = max(worst, O.rel_error(Gt[pt, 0, :, o0 + r], Gt[pt, 1, :, o0 + r], gr, sg))
        U.flush(f"wide rows L={L} point {pt}: terms worst {worst:.2e}")
        assert worst <= tol, (pt, worst)
    if L == 2:
        v = torch.zeros((2, 2, L, sys_.n_polys), dtype=torch.float64, device="cuda")
        with pytest.raises(pe.PolyevalError):
            S.adjoint(xd, v)
        with pytest.raises(pe.PolyevalError):
            pe.Batch([S])
    S.close()


def test_newton_chandrasekhar_4096(pe):
    """The largest case of the paper's Table 3: Chandrasekhar's H-equation at
    n = 4096 in complex double double, six Gauss-Newton iterations from H = 1
    (evaluation in column tiles, least squares by the column-parallel MGS):
    the step sizes decrease quadratically to the level's floor and at the end
    F is zero to the tolerance on sampled rows (oracle), H real and above 1."""
    import torch
    n, L = 4096, 2
    sys_ = synth.chandrasekhar_system(n, L)
    S = pe.System.from_sparse(sys_)
    x = torch.zeros((1, 2, L, n), dtype=torch.float64, device="cuda")
    x[0, 0, 0] = 1.0
    ws = torch.empty((S.newton_workspace_bytes(1) + 7) // 8, dtype=torch.float64, device="cuda")
    steps = []
    for it in range(6):
        _, r = S.newton_step(x, workspace=ws)
        torch.cuda.synchronize()
        steps.append(float(r.cpu().numpy()[0, 1]))
        U.flush(f"chandrasekhar 4096 DD: step {it}: |dx| = {steps[-1]:.3e}")
    S.close()
    for a, b in zip(steps, steps[1:]):
        assert b <= 1e4 * a * a + 1e-27, steps
    xe = x.cpu().numpy()[0]
    rows = [0, 1, 2047, 4094, 4095]
    eF = U.max_value_ratio(U.row_subsystem(sys_, rows), xe, range(len(rows)))
    assert eF <= U.tolerance(sys_) * 8, eF
    assert np.all(xe[0, 0] > 1.0) and np.all(np.abs(xe[1, 0]) <= 1e-25)
