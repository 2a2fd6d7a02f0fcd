"""Pins of the oracle's GS2-preconditioned MPK (Sec. 5.1, Alg. 4a; reading R21) against
facts that do not come from the oracle: the Neumann series of the strictly lower part
built densely, exact forward substitution once gamma >= n - 1 (D^{-1} L is nilpotent),
SciPy's triangular solve, the Jacobi special case gamma = 0 built by column scaling, and
an integer-exact case.  Each test names the plausible mistake it would catch."""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

import oracle as O
import synth as S


def dense(A):
    n, rp, c, v = A
    M = np.zeros((n, n))
    for i in range(n):
        M[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return M


def dominant(n, seed, symmetric=False):
    A = S.random_pattern(n, 5, seed, symmetric=symmetric)
    M = dense(A)
    M[np.arange(n), np.arange(n)] = 1.0 + np.abs(M).sum(axis=1)
    return S.from_dense(M), M


@pytest.mark.parametrize("gamma", [0, 1, 2, 3])
@pytest.mark.parametrize("seed", range(3))
def test_neumann_series_built_densely(gamma, seed):
    # P^{-1} = sum_{i<=gamma} (-D^{-1} L)^i D^{-1}, then A P^{-1} applied p times
    # catches: U instead of L, a missing D^{-1} on the sweep term, an extra or missing sweep
    A, M = dominant(40, seed)
    D = np.diag(np.diag(M))
    L = np.tril(M, -1)
    N = -np.linalg.solve(D, L)
    P = sum(np.linalg.matrix_power(N, i) for i in range(gamma + 1)) @ np.linalg.inv(D)
    x = S.uniform_vector(40, seed + 5)
    W = O.gs2_mpk(A, x, 3, gamma)
    w = x
    for j in range(3):
        w = M @ (P @ w)
        np.testing.assert_allclose(W[j], w, rtol=1e-12, atol=1e-12 * np.abs(w).max())


def test_enough_sweeps_are_the_exact_forward_substitution():
    # D^{-1} L is strictly lower triangular, so gamma >= n - 1 sweeps give (D + L)^{-1} v
    # exactly in exact arithmetic; compare with SciPy's triangular solve
    A, M = dominant(30, 7)
    v = S.uniform_vector(30, 1)
    z = O.gs2_precondition(A, v, 29)
    np.testing.assert_allclose(z, solve_triangular(np.tril(M), v, lower=True), rtol=1e-12, atol=1e-13)
    # for a lower triangular A the preconditioner is exact: A P^{-1} = I
    T = S.from_dense(np.tril(M))
    np.testing.assert_allclose(O.gs2_mpk(T, v, 2, 29), np.tile(v, (2, 1)), rtol=1e-11, atol=1e-12)


def test_gamma_zero_is_the_diagonal_scaling():
    A, M = dominant(35, 3)
    x = S.uniform_vector(35, 2)
    B = M / np.diag(M)[None, :]
    w = x
    W = O.gs2_mpk(A, x, 4, 0)
    for j in range(4):
        w = B @ w
        np.testing.assert_allclose(W[j], w, rtol=1e-12, atol=1e-12 * np.abs(w).max())


def test_lower_part_uses_the_original_numbering():
    # a 3 x 3 case by hand: L holds only a_10, a_20, a_21
    M = np.array([[2.0, 5.0, 7.0], [3.0, 4.0, 11.0], [13.0, 17.0, 8.0]])
    A = S.from_dense(M)
    x = np.array([1.0, 2.0, 3.0])
    assert np.array_equal(O.spmv_lower(A, x), np.array([0.0, 3.0, 13.0 + 34.0]))
    # one sweep: g0 = x / d = (1/2, 1/2, 3/8); g1 = g0 - L g0 / d
    g0 = np.array([0.5, 0.5, 0.375])
    g1 = g0 - np.array([0.0, 1.5, 6.5 + 8.5]) / np.array([2.0, 4.0, 8.0])
    assert np.array_equal(O.gs2_precondition(A, x, 1), g1)


def test_integer_exact_with_power_of_two_diagonal():
    # 2D Laplacian, D = 4 I: one sweep on x a multiple of 4^6 stays integer
    A = S.laplacian_2d(5, 4)
    Mi = dense(A).astype(np.int64)
    Li = np.tril(Mi, -1)
    x = S.integer_vector(A.n, 4, bound=1 << 8).astype(np.int64) * 4 ** 6
    W = O.gs2_mpk(A, x.astype(np.float64), 2, 1)
    w = x
    for j in range(2):
        assert np.all(w % 16 == 0)
        g0 = w // 4
        g1 = g0 - (Li @ g0) // 4
        w = Mi @ g1
        assert np.array_equal(W[j], w.astype(np.float64))
