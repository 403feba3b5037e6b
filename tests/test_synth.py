"""The seeded input generator: determinism, structure and value laws."""
import numpy as np

from paper_1402_2626_amd import synth


def test_deterministic():
    a, xa = synth.workload("d_n32")
    b, xb = synth.workload("d_n32")
    for f in ("poly_ptr", "mon_ptr", "var_idx", "exps", "coef"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert np.array_equal(xa, xb)


def test_structure_laws():
    s, x = synth.workload("dd_n256")
    s.validate_layout()
    assert s.n_polys == 256 and s.n_monomials == 256 * 256 and s.nnz == 256 * 256 * 16
    v = s.var_idx.reshape(-1, 16)
    assert np.all(np.diff(v, axis=1) > 0), "variables must be sorted and distinct"
    assert v.min() >= 0 and v.max() < 256
    assert set(np.unique(s.exps)) == {1, 2, 3, 4}
    # uniform without replacement: every variable about equally often
    counts = np.bincount(s.var_idx, minlength=256)
    assert abs(counts.mean() - 4096) < 1 and counts.std() < 4 * np.sqrt(4096)
    assert x.shape == (1, 2, 2, 256)


def test_limbs_nonoverlapping_and_unit_modulus():
    rng = synth.rng_for(5)
    for L in (1, 2, 4):
        z = synth.unit_circle(rng, 5000, L)
        mod = np.hypot(z[0, 0], z[1, 0])
        assert np.all(np.abs(mod - 1.0) < 4e-16)
        for l in range(1, L):
            for part in (0, 1):
                hi, lo = z[part, l - 1], z[part, l]
                # RN(hi + lo) == hi: lo is below half a gap of hi
                assert np.all(hi + lo == hi)
                assert np.count_nonzero(lo) > 4900


def test_subsets_uniform_dense_branch():
    rng = synth.rng_for(9)
    rows = synth.distinct_sorted_subsets(rng, 20000, 8, 6)  # 2k > n path
    assert np.all(np.diff(rows, axis=1) > 0)
    counts = np.bincount(rows.reshape(-1), minlength=8)
    assert np.allclose(counts / counts.sum(), 1 / 8, atol=0.01)


def test_cyclic_shape():
    s = synth.cyclic_roots_system(6, 2)
    assert s.n_monomials == 6 * 6 - 6 + 2
    assert s.n_polys == 6
    k = np.diff(s.mon_ptr)
    # row i (0-based) has monomials of i+1 variables; last row: full product and constant
    for i in range(5):
        assert set(k[s.poly_ptr[i]:s.poly_ptr[i + 1]]) == {i + 1}
    assert list(k[s.poly_ptr[5]:]) == [6, 0]


def test_batch_sizes():
    n = synth.batch_sizes(0, 4096)
    assert set(np.unique(n)) == {32, 64, 128, 256}
    s = synth.batch_system(0, 3, int(n[3]))
    assert s.n_polys == n[3] and s.n_monomials == n[3] * n[3]
    assert np.all(np.diff(s.mon_ptr) == min(16, n[3] // 4))
