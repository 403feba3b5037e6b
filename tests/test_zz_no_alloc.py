"""pe_eval_adjoint_static: the adjoint with its partial rows in the library's
static device array (no allocation), called through the C ABI and compared
with pe_eval_adjoint and with the exact oracle, on two calls in a row (the
second with a smaller input), plus a call whose groups must shrink to fit
the array and the size refusal."""
import ctypes

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


def _call_static(pe, S, xd, vd, gd):
    import torch
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return pe._lib.pe_eval_adjoint_static(S.handle, int(xd.shape[0]), ctypes.c_void_p(xd.data_ptr()),
                                          ctypes.c_void_p(vd.data_ptr()), ctypes.c_void_p(gd.data_ptr()), st)


def _call_plain(pe, S, xd, vd, gd):
    import torch
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return pe._lib.pe_eval_adjoint(S.handle, int(xd.shape[0]), ctypes.c_void_p(xd.data_ptr()),
                                   ctypes.c_void_p(vd.data_ptr()), ctypes.c_void_p(gd.data_ptr()), st)


def _check_oracle(sys_, x, v, g, cols, tol):
    for pt in range(x.shape[0]):
        Sc = O.abs_sums_columns(sys_, x[pt], cols)
        av = np.hypot(v[pt, 0].sum(axis=0), v[pt, 1].sum(axis=0))
        exact = O.adjoint_columns(sys_, x[pt], v[pt], cols)
        for j in cols:
            scale = sum(s * av[p] for p, s in Sc[j].items())
            e = O.rel_error(g[pt, 0, :, j], g[pt, 1, :, j], exact[j], scale)
            assert e <= tol, (pt, j, e)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_static_adjoint_two_calls(pe, L):
    """Two calls in a row, the second with fewer points and a smaller
    system: bitwise equal to pe_eval_adjoint (same groups) and within the
    level's tolerance of the oracle."""
    import torch
    cases = [(dict(n_vars=48, n_polys=90, m=14, k=6), 5, 301),
             (dict(n_vars=20, n_polys=33, m=9, k=4), 2, 302)]
    for spec, P, seed in cases:
        U.flush(f"static adjoint L={L} n={spec['n_vars']} N={spec['n_polys']} P={P}")
        sys_ = synth.random_system(seed, L, exp_lo=1, exp_hi=3, **spec)
        n, N = spec["n_vars"], spec["n_polys"]
        x = synth.unit_circle_points(synth.rng_for((seed, 1)), P, n, L)
        v = synth.unit_circle_points(synth.rng_for((seed, 2)), P, N, L)
        S = pe.System.from_sparse(sys_)
        xd, vd = U.to_device(x), U.to_device(v)
        gs = torch.full_like(xd, float("nan"))
        gp = torch.full_like(xd, float("nan"))
        assert _call_static(pe, S, xd, vd, gs) == 0, pe._lib.pe_last_error()
        assert _call_plain(pe, S, xd, vd, gp) == 0, pe._lib.pe_last_error()
        torch.cuda.synchronize()
        gs_h, gp_h = gs.cpu().numpy(), gp.cpu().numpy()
        S.close()
        assert np.array_equal(gs_h, gp_h)
        _check_oracle(sys_, x, v, gs_h, list(range(n)), U.tolerance(sys_))


def test_static_adjoint_shrinks_groups_to_fit(pe):
    """A call whose default groups would need more partial rows than the
    array holds (P * NG * 16 L n bytes > 32 MiB): fewer, larger groups,
    within the tolerance of pe_eval_adjoint's values and the oracle."""
    import torch
    L, n, N, P = 2, 1024, 600, 64
    # default groups: gsize = ceil(600 * 64 / 4096) = 10, NG = 60 -> 64 * 60
    # partial rows of 32 KiB = 120 MiB; the array holds 1024 such rows, 16
    # groups at 64 points
    U.flush("static adjoint: shrinking groups, n=1024 N=600 P=64")
    sys_ = synth.random_system(303, L, n_vars=n, n_polys=N, m=8, k=5, exp_lo=1, exp_hi=2)
    x = synth.unit_circle_points(synth.rng_for((303, 1)), P, n, L)
    v = synth.unit_circle_points(synth.rng_for((303, 2)), P, N, L)
    S = pe.System.from_sparse(sys_)
    xd, vd = U.to_device(x), U.to_device(v)
    gs, gp = torch.empty_like(xd), torch.empty_like(xd)
    assert _call_static(pe, S, xd, vd, gs) == 0, pe._lib.pe_last_error()
    assert _call_plain(pe, S, xd, vd, gp) == 0, pe._lib.pe_last_error()
    torch.cuda.synchronize()
    gs_h, gp_h = gs.cpu().numpy(), gp.cpu().numpy()
    tol = U.tolerance(sys_)
    # against the exact oracle at every column of four points; against
    # pe_eval_adjoint at every point within the same metric (the two differ
    # only in the order of the group sums)
    cols = list(range(n))
    pts = [0, 1, P // 2, P - 1]
    _check_oracle(sys_, x[pts], v[pts], gs_h[pts], cols, tol)
    for pt in range(0, P, 8):
        Sc = O.abs_sums_columns(sys_, x[pt], cols)
        av = np.hypot(v[pt, 0].sum(axis=0), v[pt, 1].sum(axis=0))
        for j in cols:
            scale = sum(s * av[p] for p, s in Sc[j].items())
            ref = O.cdy_from_limbs(gp_h[pt, 0, :, j], gp_h[pt, 1, :, j])
            e = O.rel_error(gs_h[pt, 0, :, j], gs_h[pt, 1, :, j], ref, scale)
            assert e <= 2 * tol, (pt, j, e)
    # the refusal: one partial row per point must fit
    P2 = 1100  # 1100 rows of 32 KiB > 32 MiB
    x2 = torch.zeros((P2, 2, L, n), dtype=torch.float64, device="cuda")
    v2 = torch.zeros((P2, 2, L, N), dtype=torch.float64, device="cuda")
    g2 = torch.zeros_like(x2)
    st = _call_static(pe, S, x2, v2, g2)
    assert st == pe.PE_EUNSUPPORTED
    assert b"static scratch" in pe._lib.pe_last_error()
    S.close()
