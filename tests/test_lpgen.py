"""The seeded input generators: published hash vectors, determinism and the stated laws."""
import numpy as np

import lpgen


def test_splitmix64_published_vectors():
    # First three outputs of SplitMix64 started from state 0 (Steele, Lea & Flood 2014).
    g = 0x9E3779B97F4A7C15
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = [lpgen._mix_int((k * g) % 2**64) for k in range(3)]
    assert got == want
    arr = lpgen._mix_arr(np.array([(k * g) % 2**64 for k in range(3)], dtype=np.uint64))
    assert [int(v) for v in arr] == want


def test_scalar_and_vector_hash_agree():
    idx = np.arange(0, 5000, 7, dtype=np.uint64)
    v = lpgen.hash_array(12345, 3, idx)
    for k in (0, 1, 100, len(idx) - 1):
        assert int(v[k]) == lpgen.hash_scalar(12345, 3, int(idx[k]))


def test_dense_law():
    A, b, c = lpgen.dense_lp(9, 37, 53)
    assert A.flags.f_contiguous and A.shape == (37, 53)
    assert A.min() >= 0 and A.max() < 1 and b.min() >= 1 and b.max() < 10 and c.min() >= 1 and c.max() < 10
    A2, b2, c2 = lpgen.dense_lp(9, 37, 53)
    assert np.array_equal(A, A2) and np.array_equal(b, b2) and np.array_equal(c, c2)
    # entry (i, j) is u(seed, A, j*m+i): regenerable one by one
    i, j = 5, 17
    assert A[i, j] == lpgen.uniform(9, lpgen.S_A, np.array([j * 37 + i], dtype=np.uint64), 0.0, 1.0)[0]
    A3, _, _ = lpgen.dense_lp(10, 37, 53)
    assert not np.array_equal(A, A3)


def test_degenerate_law_structure():
    m, n = 200, 400
    A, b, c = lpgen.degenerate_lp(3, m, n)
    k = round(0.02 * m)
    nnz = (A != 0).sum(axis=0)
    assert np.all(nnz == k + 1)
    assert np.all(A.max(axis=0) >= 0.5)  # the extra positive entry
    assert np.sum(b == 0) == round(0.3 * m)
    assert np.all((b == 0) | (b >= 1))
    assert c.min() >= 0 and c.max() < 1
    Ab, bb, cb = lpgen.degenerate_lp(3, m, n, budget_row=True)
    assert Ab.shape == (m + 1, n) and np.array_equal(Ab[:m], A) and np.all(Ab[m] == 1) and bb[m] == m


def test_batch_sizes_law():
    ms, ns = lpgen.batch_sizes(0, 4096)
    assert ms.min() >= 16 and ms.max() <= 256 and np.all(ns == 2 * ms)
    assert len(np.unique(ms)) > 200


def test_general_law_is_feasible_by_construction():
    """x0 (regenerated from its stream) satisfies every row of the general law, in the
    given row types and signs; the law has >= rows, = rows and negative b."""
    m, n = 200, 400
    A, b, c, rt = lpgen.general_lp(3, m, n, ge_frac=0.2, eq_frac=0.1, neg_frac=0.1)
    x0 = lpgen.uniform(3, lpgen.S_EXTRA, np.arange(n, dtype=np.uint64), 0.0, 2.0 / n)
    Ax = A @ x0
    tol = 1e-12 * (1 + np.abs(b).max())
    assert np.all(Ax[rt == lpgen.ROW_LE] <= b[rt == lpgen.ROW_LE] + tol)
    assert np.all(Ax[rt == lpgen.ROW_GE] >= b[rt == lpgen.ROW_GE] - tol)
    assert np.allclose(Ax[rt == lpgen.ROW_EQ], b[rt == lpgen.ROW_EQ], rtol=0, atol=tol)
    assert (rt == lpgen.ROW_GE).any() and (rt == lpgen.ROW_EQ).any() and (b < 0).any()
    assert A.flags.f_contiguous and (c >= 1).all() and (c < 10).all()
    A2, b2, c2, rt2 = lpgen.general_lp(3, m, n, ge_frac=0.2, eq_frac=0.1, neg_frac=0.1)
    assert np.array_equal(A, A2) and np.array_equal(b, b2) and np.array_equal(rt, rt2)
