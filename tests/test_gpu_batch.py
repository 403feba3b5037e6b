"""Batched evaluation of uneven systems in one persistent launch, and the
batched Gauss-Newton step (also captured in a HIP graph)."""
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


def _pack_points(batch, xs, P):
    """Per-system points xs[s] of shape [P, 2, L, n_s] -> flat packed array."""
    out = np.zeros(int(batch.x_off[-1]) * P)
    for s, x in enumerate(xs):
        a = int(batch.x_off[s]) * P
        out[a:a + x.size] = x.reshape(-1)
    return out


def _unpack(flat, off, s, shape, P):
    a = int(off[s]) * P
    size = int(np.prod(shape))
    return flat[a:a + size].reshape(shape)


def test_batch_uneven_matches_single_and_oracle(pe):
    """Systems shaped like the uneven DD batch (n = N = m in {32, 64, 128,
    256}, k = min(16, n/4), exponents 1..3) at 8 points each: the persistent
    launch equals one-system launches bit for bit; sampled rows match the
    oracle."""
    import torch
    S_count, P = 24, 8
    ns = synth.batch_sizes(0, S_count)
    systems = [synth.batch_system(0, i, int(ns[i])) for i in range(S_count)]
    dev = [pe.System.from_sparse(s) for s in systems]
    B = pe.Batch(dev)
    xs = [synth.unit_circle_points(synth.rng_for((0, 300, i)), P, int(ns[i]), 2) for i in range(S_count)]
    xflat = U.to_device(_pack_points(B, xs, P))
    U.flush("batch: persistent launch")
    G = B.info()["chunks_per_workgroup"]
    assert B.info()["systems"] == S_count and G in (1, 2)
    F, J = B.eval(xflat, P)
    torch.cuda.synchronize()
    F, J = F.cpu().numpy(), J.cpu().numpy()
    # F only
    Fo, Jo = B.eval(xflat, P, want_J=False)
    torch.cuda.synchronize()
    assert Jo is None
    Fo = Fo.cpu().numpy()
    B.close()  # the systems may be repacked once no batch holds them
    for i in range(S_count):
        n = int(ns[i])
        Fi = _unpack(F, B.F_off, i, (P, 2, 2, n), P)
        Ji = _unpack(J, B.J_off, i, (P, 2, 2, n, n), P)
        dev[i].set_shape(G)  # the batch's chunks per workgroup
        F1, J1 = dev[i].eval(U.to_device(xs[i]))
        torch.cuda.synchronize()
        assert np.array_equal(F1.cpu().numpy(), Fi) and np.array_equal(J1.cpu().numpy(), Ji), i
        dev[i].set_shape(0)
    for i in (0, 5, 17):
        n = int(ns[i])
        Fi = _unpack(F, B.F_off, i, (P, 2, 2, n), P)
        Ji = _unpack(J, B.J_off, i, (P, 2, 2, n, n), P)
        tol = U.tolerance(systems[i])
        for pt in (0, 7):
            eF, eJ = U.max_errors_rows(systems[i], xs[i][pt], Fi[pt], Ji[pt], [0, n - 1], parallel=False)
            assert eF <= tol and eJ <= tol, (i, pt, eF, eJ)
    for i in (2, 9):
        n = int(ns[i])
        eF, _ = U.max_errors_rows(systems[i], xs[i][3], _unpack(Fo, B.F_off, i, (P, 2, 2, n), P)[3], None,
                                  [0, 1], parallel=False)
        assert eF <= U.tolerance(systems[i])
    for d in dev:
        d.close()


def test_batch_refuses_repack_while_alive(pe):
    """A system held by a live batch cannot be repacked, tuned or destroyed
    (the batch keeps its device arrays); after the batch is destroyed it can."""
    sys_ = synth.batch_system(0, 3, 64)
    S = pe.System.from_sparse(sys_)
    B = pe.Batch([S, S])
    for call in (lambda: S.set_shape(1, segment=4), lambda: S.autotune(1)):
        with pytest.raises(pe.PolyevalError) as e:
            call()
        assert e.value.status == pe.PE_EINVAL and "live batch" in str(e.value)
    assert pe._lib.pe_system_destroy(S.handle) == pe.PE_EINVAL
    B.close()
    S.set_shape(1, segment=4)
    S.close()


def test_batch_wide_rows_of_small_monomials(pe):
    """A dense linear system of 1,024 variables (monomials of one variable,
    four chunks per row, slot regions of 257 slots) batched with a system of
    multi-chunk rows: the batch must not take two chunks per workgroup for
    rows too wide for the slot regions; rows against the oracle and equal to
    pe_eval."""
    import torch
    rng = synth.rng_for(601)
    n = 1024
    polys = [[(0, [(j, 1)]) for j in range(n)] for _ in range(5)]
    wide = synth.from_monomial_lists(2, n, polys, coef_limbs=synth.unit_circle(rng, 5 * n, 2), name="dense_linear")
    other = synth.batch_system(0, 11, 128)
    systems = [wide, other]
    dev = [pe.System.from_sparse(s) for s in systems]
    dev[1].set_shape(0, segment=dev[0].info()["segment"])
    B = pe.Batch(dev)
    P = 2
    xs = [synth.unit_circle_points(synth.rng_for((602, i)), P, s.n_vars, 2) for i, s in enumerate(systems)]
    F, J = B.eval(U.to_device(_pack_points(B, xs, P)), P)
    torch.cuda.synchronize()
    F, J = F.cpu().numpy(), J.cpu().numpy()
    G = B.info()["chunks_per_workgroup"]
    B.close()
    for i, s in enumerate(systems):
        Fi = _unpack(F, B.F_off, i, (P, 2, 2, s.n_polys), P)
        Ji = _unpack(J, B.J_off, i, (P, 2, 2, s.n_polys, s.n_vars), P)
        tol = U.tolerance(s)
        for pt in range(P):
            eF, eJ = U.max_errors_rows(s, xs[i][pt], Fi[pt], Ji[pt], [0, s.n_polys - 1], parallel=False)
            assert eF <= tol and eJ <= tol, (i, pt, eF, eJ, G)
        if i == 0:
            F1, J1 = dev[i].eval(U.to_device(xs[i]))
            torch.cuda.synchronize()
            assert np.array_equal(F1.cpu().numpy(), Fi) and np.array_equal(J1.cpu().numpy(), Ji)
    for d in dev:
        d.close()


def test_batch_4096_full_size(pe):
    """The uneven DD batch at full size: 4,096 systems (n = N = m uniform in
    {32, 64, 128, 256}, k = min(16, n/4), exponents 1..3) at 8 points each,
    one call.  Two systems of each size: first and last rows at the first and
    last point against the oracle; 64 systems (16 of each size) equal to
    pe_eval on their own, bit for bit, on the device."""
    import torch
    S_count, P = 4096, 8
    ns = synth.batch_sizes(0, S_count)
    U.flush("batch 4096: loading systems")
    dev = [pe.System.from_sparse(synth.batch_system(0, i, int(ns[i]))) for i in range(S_count)]
    B = pe.Batch(dev)
    rng = synth.rng_for((0, 9))
    xs_host = [synth.unit_circle_points(rng, P, int(n), 2) for n in ns]
    x = U.to_device(np.concatenate([a.reshape(-1) for a in xs_host]))
    U.flush("batch 4096: persistent launch")
    F, J = B.eval(x, P)
    torch.cuda.synchronize()
    G = B.info()["chunks_per_workgroup"]
    by_n = {int(n): [i for i in range(S_count) if int(ns[i]) == int(n)] for n in (32, 64, 128, 256)}
    checked = 0
    for n, idx in by_n.items():
        for i in (idx[0], idx[-1]):
            sys_ = synth.batch_system(0, i, n)
            a, b = int(B.F_off[i]) * P, int(B.J_off[i]) * P
            Fi = F[a:a + P * 4 * n].view(P, 2, 2, n).cpu().numpy()
            Ji = J[b:b + P * 4 * n * n].view(P, 2, 2, n, n).cpu().numpy()
            tol = U.tolerance(sys_)
            for pt in (0, P - 1):
                U.flush(f"batch 4096: oracle system {i} (n = {n}) point {pt}")
                eF, eJ = U.max_errors_rows(sys_, xs_host[i][pt], Fi[pt], Ji[pt], [0, n - 1], parallel=True)
                assert eF <= tol and eJ <= tol, (i, n, pt, eF, eJ)
                checked += 1
        for i in idx[:: max(1, len(idx) // 16)][:16]:
            info = dev[i].info()
            assert info["chunks_per_workgroup"] in (1, G), (i, info, G)
            a, f, b = int(B.x_off[i]) * P, int(B.F_off[i]) * P, int(B.J_off[i]) * P
            F1, J1 = dev[i].eval(x[a:a + P * 4 * n].view(P, 2, 2, n))
            assert torch.equal(F1.reshape(-1), F[f:f + P * 4 * n]), i
            assert torch.equal(J1.reshape(-1), J[b:b + P * 4 * n * n]), i
    assert checked == 16
    del F, J
    B.close()
    for d in dev:
        d.close()


def _planted_batch(L, sizes, seed):
    systems, stars = [], []
    for i, n in enumerate(sizes):
        s = synth.random_system((seed, i), L, n_vars=n, n_polys=n + (i % 2) * 3, m=6, k=3, exp_lo=1, exp_hi=3)
        xs = synth.unit_circle_points(synth.rng_for((seed, 50 + i)), 1, n, L)[0]
        systems.append(O.plant_root(s, xs))
        stars.append(xs)
    return systems, stars


@pytest.mark.parametrize("L", [2, 4])
def test_batch_newton_matches_single(pe, L):
    """Batched Gauss-Newton over systems of different sizes (some
    overdetermined) equals the one-system step bit for bit and converges."""
    import torch
    sizes = [8, 20, 13, 32, 5]
    P = 2
    systems, stars = _planted_batch(L, sizes, 401)
    dev = [pe.System.from_sparse(s) for s in systems]
    B = pe.Batch(dev)
    x0 = [np.stack([synth.perturbed_start((402, i, pt), stars[i], 1e-5) for pt in range(P)])
          for i in range(len(sizes))]
    xb = U.to_device(_pack_points(B, x0, P))
    singles = [U.to_device(x0[i]) for i in range(len(sizes))]
    for it in range(4):
        _, rb = B.newton_step(xb, P)
        for i in range(len(sizes)):
            dev[i].newton_step(singles[i])
        torch.cuda.synchronize()
        xbn = xb.cpu().numpy()
        for i in range(len(sizes)):
            got = _unpack(xbn, B.x_off, i, (P, 2, L, sizes[i]), P)
            assert np.array_equal(got, singles[i].cpu().numpy()), (it, i)
    u = 2.0 ** (-53 * L)
    for i in range(len(sizes)):
        got = _unpack(xb.cpu().numpy(), B.x_off, i, (P, 2, L, sizes[i]), P)
        Xs = O.point_from_limbs(stars[i])
        for pt in range(P):
            d = max(O.cdy_abs_float(O.cdy_add(O.cdy_from_limbs(got[pt, 0, :, j], got[pt, 1, :, j]), O.cdy_neg(Xs[j])))
                    for j in range(sizes[i]))
            assert d <= 1e6 * u, (i, pt, d)
    B.close()
    for d in dev:
        d.close()


def test_batch_newton_graph(pe):
    """The batched Newton step captured once in a HIP graph and replayed with
    eager work in between reproduces the eager iterates bit for bit."""
    import torch
    sizes = [12, 7, 24]
    P = 3
    systems, stars = _planted_batch(2, sizes, 501)
    dev = [pe.System.from_sparse(s) for s in systems]
    B = pe.Batch(dev)
    x0 = [np.stack([synth.perturbed_start((502, i, pt), stars[i], 1e-5) for pt in range(P)])
          for i in range(len(sizes))]
    flat0 = _pack_points(B, x0, P)
    ws = torch.empty((B.newton_workspace_bytes(P) + 7) // 8, dtype=torch.float64, device="cuda")
    resid = torch.empty((len(sizes), P, 2), dtype=torch.float64, device="cuda")
    xe = U.to_device(flat0)
    eager = []
    for _ in range(3):
        B.newton_step(xe, P, workspace=ws, resid=resid)
        torch.cuda.synchronize()
        eager.append(xe.cpu().numpy().copy())
    s = torch.cuda.Stream()
    xg = U.to_device(flat0)
    B.newton_step(xg.clone(), P, workspace=ws, resid=resid, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        B.newton_step(xg, P, workspace=ws, resid=resid, stream=s)
    xg.copy_(U.to_device(flat0))
    torch.cuda.synchronize()
    for it in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (torch.randn(4096, device="cuda") * 2).sum().item()
        assert np.array_equal(xg.cpu().numpy(), eager[it]), it
    B.close()
    for d in dev:
        d.close()
