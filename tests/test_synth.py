"""Shapes and structure of the seeded synthetic inputs."""
import numpy as np
import pytest

import synth as S


def test_laplacian_sizes():
    A = S.laplacian_2d(64)
    assert A.n == 4096 and A.col.size == 5 * 4096 - 4 * 64 == 20224
    A = S.laplacian_3d(20)
    assert A.n == 8000 and A.col.size == 7 * 20 ** 3 - 6 * 20 ** 2


@pytest.mark.slow
def test_laplacian_3d_160_size():
    A = S.laplacian_3d(160)
    assert A.n == 4_096_000 and A.col.size == 28_518_400
    assert A.rowptr.dtype == np.int32 and A.col.dtype == np.int32


def test_csr_conventions():
    for A in [S.laplacian_2d(7, 5), S.laplacian_3d(4, 3, 5), S.random_pattern(100, 4, 1),
              S.knn_graph_laplacian(500, k=6, seed=2)]:
        rp, c = A.rowptr.astype(np.int64), A.col.astype(np.int64)
        assert rp[0] == 0 and rp[-1] == c.size and np.all(np.diff(rp) >= 0)
        for i in range(A.n):
            seg = c[rp[i]:rp[i + 1]]
            assert np.all(np.diff(seg) > 0) and (seg.size == 0 or (seg[0] >= 0 and seg[-1] < A.n))


def test_knn_laplacian_structure():
    A = S.knn_graph_laplacian(2000, k=26, seed=0)
    n, rp, c, v = A.n, A.rowptr.astype(np.int64), A.col.astype(np.int64), A.val
    assert n == 2000
    counts = np.diff(rp)
    assert counts.min() >= 27  # k neighbours + diagonal
    rows = np.repeat(np.arange(n), counts)
    key = set(zip(rows.tolist(), c.tolist()))
    assert all((j, i) in key for i, j in key)  # symmetric pattern
    # L 1 = shift * 1 (rows of D - W sum to zero)
    rs = np.bincount(rows, weights=v, minlength=n)
    assert np.allclose(rs, 0.1, atol=1e-12)
    # Morton order keeps neighbours close in index on average
    off = np.abs(rows - c)[rows != c]
    assert np.median(off) < n / 10


def test_vectors_seeded():
    assert np.array_equal(S.uniform_vector(10, 3), S.uniform_vector(10, 3))
    x = S.integer_vector(1000, 1)
    assert np.all(x == np.round(x)) and np.abs(x).max() <= 1 << 20
