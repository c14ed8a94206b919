"""The seeded input generator: shape, ranges, determinism, and the Zipf law."""
import numpy as np

import synth


def _check_csr(m, lo, hi):
    lens = np.diff(m.indptr)
    assert lens.min() >= lo and lens.max() <= hi
    for i in range(0, m.n_rows, max(1, m.n_rows // 200)):
        d, w = m.row(i)
        assert np.all(np.diff(d) > 0)
        assert d.min() >= 0 and d.max() < m.n_dims
        assert np.all(w > 0)


def test_tiny_shapes_and_ranges():
    S = synth.make("tiny", "S")
    R = synth.make("tiny", "R")
    assert S.n_rows == 10_000 and R.n_rows == 1_000 and S.n_dims == 10_000
    _check_csr(S, 20, 100)
    _check_csr(R, 20, 100)
    assert S.values.dtype == np.uint8 and S.values.min() >= 1 and S.values.max() == 255
    assert abs(np.diff(S.indptr).mean() - 60) < 1.0


def test_determinism_and_row_independence():
    a = synth.make("medium", "S", n_rows=3000)
    b = synth.make("medium", "S", n_rows=1000)
    np.testing.assert_array_equal(a.indptr[:1001], b.indptr)
    np.testing.assert_array_equal(a.indices[:b.nnz], b.indices)
    np.testing.assert_array_equal(a.values[:b.nnz], b.values)


def test_zipf_head_frequencies():
    """Rank-1..5 dimensions appear with the probability successive sampling predicts."""
    S = synth.make("medium", "S", n_rows=20_000)
    perm = synth.workload_perm("medium")
    _check_csr(S, 50, 200)
    cnt = np.bincount(S.indices, minlength=S.n_dims)
    # the most frequent dimensions are the first entries of the permutation
    assert set(np.argsort(-cnt)[:3]) <= set(perm[:6].tolist())
    # rank-1 dimension: p1 = 1/H(10000,1.1) ~ 0.152 per draw; a vector with >= 50 distinct
    # draws contains it with probability > 0.99
    assert cnt[perm[0]] / S.n_rows > 0.99
    # a deep-tail rank is rare
    assert cnt[perm[9000]] / S.n_rows < 0.02


def test_lognormal_nnz_and_f32_norm():
    R = synth.make("batched", "R", n_rows=20_000)
    lens = np.diff(R.indptr)
    assert lens.min() >= 10 and lens.max() <= 1000
    assert 80 < np.median(lens) < 120          # median of lognormal(ln 100, .8) is 100
    F = synth.make("fp32", "R", n_rows=500)
    _check_csr(F, 30, 300)
    norms = np.sqrt(np.add.reduceat(F.values.astype(np.float64) ** 2, F.indptr[:-1]))
    np.testing.assert_allclose(norms, 1.0, rtol=1e-6)
