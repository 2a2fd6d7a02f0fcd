"""Pins of the oracle's Jacobi-preconditioned MPK (Sec. 5.1; reading R20) against
closed forms and special cases that do not come from the oracle: Dirichlet
Laplacian eigenpairs, exact Jacobi on diagonal matrices, the fused A D^{-1} form
built densely, convergence of many sweeps to A^{-1}, and exact integer arithmetic.
Each test names the plausible mistake it would catch."""
import math

import numpy as np
import pytest

import oracle as O
import synth as S


def dense(A):
    n, rp, c, v = A
    M = np.zeros((n, n))
    for i in range(n):
        M[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return M


@pytest.mark.parametrize("k", [1, 2, 3, 6])
@pytest.mark.parametrize("j", [1, 7, 13])
def test_laplacian_eigenvector_closed_form(k, j):
    # 1D Dirichlet Laplacian: D = 2 I, so one sweep multiplies an eigenvector by 1/2 and
    # the Jacobi iteration matrix I - A/2 has eigenvalue 1 - lam/2; k sweeps from zero give
    # P^{-1} v = (1 - (1 - lam/2)^k) / lam v, hence A P^{-1} v = (1 - (1 - lam/2)^k) v
    # catches: a wrong sign of (L + U), a missing D^{-1} on v, an extra or missing sweep
    n = 15
    A = S.laplacian_1d(n)
    lam = 2 - 2 * math.cos(j * math.pi / (n + 1))
    v = np.sin(j * math.pi * np.arange(1, n + 1) / (n + 1))
    mu = 1 - (1 - lam / 2) ** k
    W = O.jacobi_mpk(A, v, 4, k)
    for p in range(4):
        np.testing.assert_allclose(W[p], mu ** (p + 1) * v, atol=1e-13)
    np.testing.assert_allclose(O.jacobi_precondition(A, v, k), (mu / lam) * v, atol=1e-13)


def test_diagonal_matrix_jacobi_is_exact():
    # for diagonal A the Jacobi iteration solves exactly after one sweep: A P^{-1} = I
    d = np.array([3.0, -0.5, 7.25, 2.0, 11.0])
    A = S.diagonal(d)
    x = S.uniform_vector(5, 2)
    for k in (1, 2, 5):
        assert np.array_equal(O.jacobi_mpk(A, x, 3, k), np.tile(x, (3, 1)))


@pytest.mark.parametrize("seed", range(3))
def test_one_sweep_is_the_fused_column_scaling(seed):
    # k = 1: P^{-1} = D^{-1}, so w_j = (A D^{-1})^j x; built densely with column scaling
    A = S.random_pattern(40, 6, seed, symmetric=False)
    Ad = dense(A)
    B = Ad / np.diag(Ad)[None, :]
    x = S.uniform_vector(40, seed + 1)
    W = O.jacobi_mpk(A, x, 5, 1)
    w = x
    for p in range(5):
        w = B @ w
        np.testing.assert_allclose(W[p], w, rtol=1e-12, atol=1e-12 * np.abs(w).max())


def test_many_sweeps_invert_a_diagonally_dominant_matrix():
    # Jacobi converges for strictly diagonally dominant A: P^{-1} -> A^{-1}, A P^{-1} -> I
    A = S.random_pattern(60, 5, 4, symmetric=False)
    Ad = dense(A) + 12 * np.eye(60)
    A = S.from_dense(Ad)
    v = S.uniform_vector(60, 3)
    np.testing.assert_allclose(O.jacobi_precondition(A, v, 200), np.linalg.solve(Ad, v), atol=1e-12)
    np.testing.assert_allclose(O.jacobi_mpk(A, v, 2, 200)[1], v, atol=1e-12)


def test_integer_exact_with_power_of_two_diagonal():
    # 2D 5-point Laplacian: D = 4 I; x a multiple of 4^p with integers keeps every
    # intermediate an exact integer; compare with integer arithmetic
    A = S.laplacian_2d(6, 5)
    M = dense(A).astype(np.int64)
    x = S.integer_vector(A.n, 3, bound=1 << 10).astype(np.int64) * 4 ** 3
    W = O.jacobi_mpk(A, x.astype(np.float64), 3, 1)
    w = x
    for p in range(3):
        assert np.all(w % 4 == 0)
        w = M @ (w // 4)
        assert np.array_equal(W[p], w.astype(np.float64))


def test_missing_or_zero_diagonal_is_refused():
    with pytest.raises(ValueError):
        O.diagonal(S.cyclic_shift(5))
    with pytest.raises(ValueError):
        O.diagonal(S.from_dense(np.array([[0.0, 1.0], [1.0, 2.0]]), keep_zeros=True))
