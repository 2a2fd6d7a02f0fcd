"""Pins of the oracle's fused pre-smoother and residual (Sec. 5.3 with the GS2 smoother of
Sec. 5.1; reading R23) against facts that do not come from the oracle: the error
propagation matrix of the stationary iteration built densely, exact Gauss-Seidel sweeps
once gamma >= n - 1 (SciPy's triangular solve), the Jacobi smoother's closed form on
Laplacian eigenvectors, one-sweep convergence on a diagonal matrix, SciPy's sparse direct
solve after many sweeps, and an integer-exact case.  Planted mistakes (the compact listing
taken literally, U for L, the residual taken before the last sweep, one inner sweep too
many) each fail the dense check."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
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


def dense_smoother(M, b, x0, sweeps, gamma):
    # x^nu = x* + E^nu (x0 - x*) with E = I - P^{-1} A and P^{-1} the truncated Neumann
    # series sum_{i<=gamma} (-D^{-1} L)^i D^{-1}; r = b - A x^nu
    n = M.shape[0]
    D = np.diag(np.diag(M))
    N = -np.linalg.solve(D, np.tril(M, -1))
    P = sum(np.linalg.matrix_power(N, i) for i in range(gamma + 1)) @ np.linalg.inv(D)
    E = np.eye(n) - P @ M
    xs = np.linalg.solve(M, b)
    x = xs + np.linalg.matrix_power(E, sweeps) @ (x0 - xs)
    return x, b - M @ x


@pytest.mark.parametrize("gamma", [0, 1, 2, 3])
@pytest.mark.parametrize("sweeps", [0, 1, 2, 4])
def test_error_propagation_built_densely(gamma, sweeps):
    A, M = dominant(40, gamma + 7 * sweeps)
    b = S.uniform_vector(40, 3)
    x0 = S.uniform_vector(40, 4)
    x, r = O.gs2_smooth_residual(A, b, x0, sweeps, gamma)
    xe, re = dense_smoother(M, b, x0, sweeps, gamma)
    np.testing.assert_allclose(x, xe, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(r, re, rtol=1e-10, atol=1e-11 * np.abs(b).max())


def test_enough_inner_sweeps_are_gauss_seidel():
    # gamma >= n - 1: each outer sweep solves (D + L) x^{k+1} = b - U x^k exactly
    A, M = dominant(25, 11)
    b = S.uniform_vector(25, 5)
    x0 = S.uniform_vector(25, 6)
    x = x0
    for _ in range(3):
        x = solve_triangular(np.tril(M), b - np.triu(M, 1) @ x, lower=True)
    got, r = O.gs2_smooth_residual(A, b, x0, 3, 24)
    np.testing.assert_allclose(got, x, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(r, b - M @ x, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("sweeps", [1, 2, 5])
def test_jacobi_smoother_on_laplacian_eigenvectors(sweeps):
    # gamma = 0 is the Jacobi smoother; with b = 0 the error x0 = v_m (a sine mode of the
    # 1D Dirichlet Laplacian, eigenvalue lambda_m = 2 - 2 cos(m pi / (n + 1))) is damped by
    # (1 - lambda_m / 2) per sweep, and r = -A x = -lambda_m x
    n, m = 31, 5
    A = S.laplacian_1d(n)
    lam = 2.0 - 2.0 * np.cos(m * np.pi / (n + 1))
    v = np.sin(m * np.pi * np.arange(1, n + 1) / (n + 1))
    x, r = O.gs2_smooth_residual(A, np.zeros(n), v, sweeps, 0)
    np.testing.assert_allclose(x, (1 - lam / 2) ** sweeps * v, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r, -lam * (1 - lam / 2) ** sweeps * v, rtol=1e-11, atol=1e-14)


def test_diagonal_matrix_converges_in_one_sweep():
    d = np.array([2.0, 4.0, 0.5, 8.0, 1.0])
    A = S.from_dense(np.diag(d))
    b = np.array([1.0, -3.0, 0.25, 6.0, 7.0])
    for gamma in (0, 2):
        x, r = O.gs2_smooth_residual(A, b, np.ones(5), 1, gamma)
        assert np.array_equal(x, b / d)
        assert np.array_equal(r, np.zeros(5))


def test_no_sweep_is_the_residual_and_one_sweep_from_zero_is_the_preconditioner():
    A, M = dominant(30, 2)
    b = S.uniform_vector(30, 1)
    x0 = S.uniform_vector(30, 2)
    x, r = O.gs2_smooth_residual(A, b, x0, 0, 2)
    assert np.array_equal(x, x0)
    np.testing.assert_allclose(r, b - M @ x0, rtol=1e-13, atol=1e-13)
    # x^0 = 0, one sweep: b - A 0 = b exactly, so x^1 is R21's P^{-1} b
    x, _ = O.gs2_smooth_residual(A, b, np.zeros(30), 1, 2)
    assert np.array_equal(x, O.gs2_precondition(A, b, 2))


def test_many_sweeps_solve_the_system():
    A, M = dominant(200, 9, symmetric=True)
    b = S.uniform_vector(200, 8)
    n, rp, c, v = A
    xs = spla.spsolve(sp.csr_matrix((v, c, rp), shape=(n, n)).tocsc(), b)
    x, r = O.gs2_smooth_residual(A, b, np.zeros(200), 80, 1)
    np.testing.assert_allclose(x, xs, rtol=1e-10, atol=1e-12)
    assert np.abs(r).max() < 1e-10 * np.abs(b).max()


def test_integer_exact_with_power_of_two_diagonal():
    # 2D Laplacian, D = 4 I, gamma = 1, two sweeps: with b and x0 multiples of 4^5 every
    # division by 4 is exact, so int64 arithmetic gives the result exactly
    A = S.laplacian_2d(5, 4)
    Mi = dense(A).astype(np.int64)
    Li = np.tril(Mi, -1)
    b = S.integer_vector(A.n, 1, bound=1 << 8).astype(np.int64) * 4 ** 5
    x0 = S.integer_vector(A.n, 2, bound=1 << 8).astype(np.int64) * 4 ** 5
    x = x0
    for _ in range(2):
        res = b - Mi @ x
        assert np.all(res % 16 == 0)
        g0 = res // 4
        g1 = g0 - (Li @ g0) // 4
        x = x + g1
    got, r = O.gs2_smooth_residual(A, b.astype(np.float64), x0.astype(np.float64), 2, 1)
    assert np.array_equal(got, x.astype(np.float64))
    assert np.array_equal(r, (b - Mi @ x).astype(np.float64))


# ---- planted mistakes: each must fail the dense check ----------------------------------
def _compact_literal(A, b, x0, sweeps, gamma):
    # the listing taken literally: g_0 = D^{-1}(b - U x), x = x + g_gamma
    M = dense(A)
    d = np.diag(M)
    U = np.triu(M, 1)
    x = np.array(x0, dtype=float)
    for _ in range(sweeps):
        g0 = (b - U @ x) / d
        g = g0
        for _ in range(gamma):
            g = g0 - np.tril(M, -1) @ g / d
        x = x + g
    return x, b - M @ x


def _upper_for_lower(A, b, x0, sweeps, gamma):
    M = dense(A)
    d = np.diag(M)
    x = np.array(x0, dtype=float)
    for _ in range(sweeps):
        g0 = (b - M @ x) / d
        g = g0
        for _ in range(gamma):
            g = g0 - np.triu(M, 1) @ g / d
        x = x + g
    return x, b - M @ x


def _residual_before_last_sweep(A, b, x0, sweeps, gamma):
    M = dense(A)
    x_prev = np.array(x0, dtype=float)
    x, _ = O.gs2_smooth_residual(A, b, x0, sweeps, gamma)
    if sweeps:
        x_prev, _ = O.gs2_smooth_residual(A, b, x0, sweeps - 1, gamma)
    return x, b - M @ x_prev


def _extra_inner_sweep(A, b, x0, sweeps, gamma):
    return O.gs2_smooth_residual(A, b, x0, sweeps, gamma + 1)


@pytest.mark.parametrize("mutant", [_compact_literal, _upper_for_lower, _residual_before_last_sweep,
                                    _extra_inner_sweep])
def test_planted_mistakes_fail(mutant):
    A, M = dominant(40, 21)
    b = S.uniform_vector(40, 3)
    x0 = S.uniform_vector(40, 4)
    x, r = mutant(A, b, x0, 2, 1)
    xe, re = dense_smoother(M, b, x0, 2, 1)
    assert not (np.allclose(x, xe, rtol=1e-11, atol=1e-12) and np.allclose(r, re, rtol=1e-10, atol=1e-11))
