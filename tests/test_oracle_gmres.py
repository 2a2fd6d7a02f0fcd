"""Pins of the oracle's s-step GMRES (Sec. 4, Alg. 3a/3c; readings R17-R19) against
facts that do not come from the oracle itself: textbook GMRES (Alg. 3b, modified
Gram-Schmidt Arnoldi written here), closed forms of the Chebyshev shift polynomial,
finite termination on matrices with few distinct eigenvalues, SciPy's direct solve
and hand-worked small cases.  Each test names the plausible mistake it would catch."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.sparse import csr_matrix

import oracle as O
import synth as S


def dense(A):
    n, rp, c, v = A
    M = np.zeros((n, n))
    for i in range(n):
        M[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return M


def lap_bounds(dims):
    return (sum(2 - 2 * math.cos(math.pi / (m + 1)) for m in dims),
            sum(2 + 2 * math.cos(math.pi / (m + 1)) for m in dims))


def cheb_T(d, u):
    """T_d(u) from the trigonometric / hyperbolic closed forms."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    inside = np.abs(u) <= 1
    out[inside] = np.cos(d * np.arccos(u[inside]))
    big = ~inside
    out[big] = np.sign(u[big]) ** d * np.cosh(d * np.arccosh(np.abs(u[big])))
    return out


def dense_preconditioned(A, d, lmin, lmax):
    """S = s(A) and M = A S for symmetric A from its eigendecomposition and the closed
    form lam s(lam) = 1 - T_d((theta - lam)/delta) / T_d(theta/delta)."""
    Ad = dense(A)
    lam, V = np.linalg.eigh(Ad)
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    ms = 1 - cheb_T(d, (theta - lam) / delta) / cheb_T(d, np.array([theta / delta]))[0]
    return (V * (ms / lam)) @ V.T, (V * ms) @ V.T


def textbook_gmres_cycle(M, r, m):
    """Alg. 3b: Arnoldi with modified Gram-Schmidt, then the small least-squares problem.
    Returns the correction u = V_m y (to be mapped through S)."""
    n = r.size
    beta = np.linalg.norm(r)
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    V[0] = r / beta
    for j in range(m):
        w = M @ V[j]
        for i in range(j + 1):
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
    e0 = np.zeros(m + 1)
    e0[0] = beta
    y = np.linalg.lstsq(H, e0, rcond=None)[0]
    return V[:m].T @ y


# ------------------------------------------------------------------ shifts (R18)
def test_leja_order_hand_worked():
    # The three Chebyshev points of [0, 2]: 1 + cos(pi/6), 1, 1 - cos(pi/6).
    # First the largest modulus: 1.866.  Distances to it: 0.134 -> 1.732, 1 -> 0.866,
    # so 0.134 comes next; 1 is last.
    # catches: taking the points in their natural order, or maximising the sum of distances
    pts = [1 + math.cos(math.pi / 6), 1.0, 1 - math.cos(math.pi / 6)]
    assert np.array_equal(O.leja_order(pts), np.array([pts[0], pts[2], pts[1]]))
    # product rule, not the sum: from {4}, the candidates 0 (dist 4) and 3.9 (0.1);
    # then 1 has product 3 * 1 = 3 against 2 (2 * 2 = 4): 2 wins.
    assert list(O.leja_order([4.0, 3.9, 0.0, 1.0, 2.0])[:3]) == [4.0, 0.0, 2.0]
    # ties go to the lowest index
    assert list(O.leja_order([-1.0, 1.0])) == [-1.0, 1.0]


@pytest.mark.parametrize("s", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("d", [2, 8, 17])
def test_shift_polynomial_is_a_scaled_chebyshev_polynomial(s, d):
    # prod_k (mu - lambda_k) / sigma^s = 2^(1-s) (eps/2)^-s eps^s T_s((mu - 1)/eps) =
    # 2 T_s((mu - 1)/eps) on the interval of M's spectrum
    # catches: wrong interval centre or half-width, wrong sigma, a missing point
    lmin, lmax = 0.05, 7.3
    lam, sig = O.newton_shifts(s, d, lmin, lmax)
    eps = 1.0 / O.chebyshev_scale(d, lmin, lmax)
    mu = 1.0 + eps * np.linspace(-1, 1, 41)
    prod = np.ones_like(mu)
    for k in range(s):
        prod *= (mu - lam[k]) / sig[k]
    np.testing.assert_allclose(prod, 2.0 * cheb_T(s, (mu - 1.0) / eps), atol=1e-9)
    # Leja prefix: the first s' shifts of a longer sequence are not the Chebyshev
    # points of s', but they are distinct and inside the interval
    assert np.all(np.abs(lam - 1.0) < eps) and len(set(lam.tolist())) == s


@pytest.mark.parametrize("d", [1, 2, 5, 8, 12])
def test_spectrum_of_preconditioned_operator_hits_interval_ends(d):
    # lam = lmin gives M = 1 - T_d(1)/T_d(theta/delta) = 1 - eps; lam = lmax gives
    # 1 - (-1)^d eps; in between M stays inside [1 - eps, 1 + eps]
    # catches: a wrong sign of the residual polynomial, or T_d(theta/delta) miscomputed
    lmin, lmax = 0.3, 9.0
    eps = 1.0 / O.chebyshev_scale(d, lmin, lmax)
    diag = np.concatenate([[lmin, lmax], np.linspace(lmin, lmax, 30)])
    A = S.diagonal(diag)
    c, theta, delta = O.chebyshev_inverse_coeffs(d, lmin, lmax)
    Mx = O.spmv(A, O.poly_chebyshev(A, np.ones(diag.size), c, theta, delta))
    assert abs(Mx[0] - (1 - eps)) < 1e-12
    assert abs(Mx[1] - (1 - (-1) ** d * eps)) < 1e-12
    assert np.all(np.abs(Mx - 1.0) <= eps * (1 + 1e-12))


# ------------------------------------------------------------- Cholesky QR (R17)
def test_cholqr_truncated_hand_worked():
    # G = [[4, 2], [2, 2]] = R^T R with R = [[2, 1], [0, 1]]
    R, kk = O.cholqr_truncated(np.array([[4.0, 2.0], [2.0, 2.0]]), np.array([4.0, 2.0]))
    assert kk == 2 and np.array_equal(R, np.array([[2.0, 1.0], [0.0, 1.0]]))
    # rank one: the second pivot is 1 - 1 = 0 -> dependent, R[0, 1] still filled
    R, kk = O.cholqr_truncated(np.array([[4.0, 2.0], [2.0, 1.0]]), np.array([4.0, 1.0]))
    assert kk == 1 and R[0, 0] == 2.0 and R[0, 1] == 1.0 and R[1, 1] == 0.0
    # a pivot below 2^-24 of the column's length is dependent, one above is kept
    small = 2.0 ** -25
    G = np.array([[1.0, 0.0], [0.0, small ** 2]])
    assert O.cholqr_truncated(G, np.array([1.0, 1.0]))[1] == 1
    assert O.cholqr_truncated(G, np.array([1.0, small ** 2]))[1] == 2


@pytest.mark.parametrize("seed", range(4))
def test_cholqr_matches_library_cholesky(seed):
    # catches: index slips in the column-by-column factorisation
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((40, 6))
    G = X.T @ X
    R, kk = O.cholqr_truncated(G, np.diag(G))
    assert kk == 6
    np.testing.assert_allclose(R, np.linalg.cholesky(G).T, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------- the cycle (Alg. 3c)
@pytest.mark.parametrize("s,m", [(1, 6), (3, 6), (4, 12), (8, 16)])
def test_hessenberg_relation_full_basis(s, m):
    # M Q_{0..m-1} = Q_{0..m} H with Q orthonormal, M applied densely (no oracle code)
    # catches: a transposed change of basis, wrong B entries, a dropped H_old term
    A = S.random_pattern(50, 4, 5, symmetric=False)
    M = dense(A) + 5.0 * np.eye(50)
    lam = O.leja_order(5.0 + 1.5 * np.cos(np.pi * (2 * np.arange(s) + 1) / (2 * s)))
    sig = np.full(s, 1.0)
    r = S.uniform_vector(50, 4)
    beta = np.linalg.norm(r)
    # the cycle returns Q_{0..c-1}; rebuild Q_c from the last Hessenberg column
    Q, H, y, rho = O.sstep_cycle(lambda v: M @ v, r / beta, m, s, lam, sig, beta, 0.0)
    Qm = np.array(Q)
    assert Qm.shape == (m, 50) and H.shape == (m + 1, m)
    np.testing.assert_allclose(Qm @ Qm.T, np.eye(m), atol=1e-10)
    lhs = M @ Qm.T                                  # (n, m)
    resid = lhs - Qm.T @ H[:m]                      # equals Q_m H[m, :] (rank one)
    qm = resid[:, -1] / H[m, m - 1]
    np.testing.assert_allclose(np.outer(qm, H[m]), resid, atol=1e-9)
    assert abs(np.linalg.norm(qm) - 1.0) < 1e-9 and np.abs(Qm @ qm).max() < 1e-9
    # upper Hessenberg: nothing below the subdiagonal
    assert np.abs(np.tril(H, -2)).max() < 1e-9


@pytest.mark.parametrize("s,m", [(1, 12), (2, 12), (4, 12), (6, 12), (4, 10)])
def test_sstep_cycle_equals_textbook_gmres(s, m):
    # in exact arithmetic s-step GMRES and standard GMRES (Alg. 3b) give the same
    # iterate; on a well-conditioned operator they agree to rounding
    # catches: any error in BOrtho, TSQR, the Hessenberg reconstruction or the
    # least-squares step
    dims = (7, 8)
    A = S.laplacian_2d(*dims)
    lmin, lmax = lap_bounds(dims)
    d = 3
    Sd, Md = dense_preconditioned(A, d, lmin, lmax)
    b = S.uniform_vector(A.n, 9)
    x1, hist, iters = O.sstep_gmres(A, b, np.zeros(A.n), s, m, d, lmin, lmax, 0.0, 1)
    u = textbook_gmres_cycle(Md, b, m)
    x_ref = Sd @ u
    assert iters == m
    np.testing.assert_allclose(x1, x_ref, rtol=0, atol=1e-10 * np.abs(x_ref).max())


def test_nonsymmetric_cycle_equals_textbook_gmres():
    # nonsymmetric, diagonally dominant A (spectrum in a disc around 8); d = 1 makes
    # s(A) the constant 1/theta, so M = A / theta is known densely without the oracle
    A = S.random_pattern(70, 5, 21, symmetric=False, value_range=1.0)
    Ad = dense(A) + 8.0 * np.eye(70)
    A = S.from_dense(Ad)
    lmin, lmax = 2.0, 14.0
    theta = 0.5 * (lmin + lmax)
    b = S.uniform_vector(70, 2)
    for s in (1, 3, 5):
        x1, hist, iters = O.sstep_gmres(A, b, np.zeros(70), s, 15, 1, lmin, lmax, 0.0, 1)
        x_ref = textbook_gmres_cycle(Ad / theta, b, 15) / theta
        np.testing.assert_allclose(x1, x_ref, rtol=0, atol=1e-10 * np.abs(x_ref).max())


def test_finite_termination_with_three_distinct_eigenvalues():
    # with d = 3 the eigenvalues 1, 2.5, 4 of A map to 1 - eps, 1, 1 + eps in M (with
    # d = 2, 1 and 4 would both map to 1 - eps), so the Krylov space stops growing after 3
    # vectors: the block of 4 finds its 4th column dependent, the Hessenberg matrix is
    # square and the solve is exact after one cycle
    # catches: a wrong dependent-column rule or a wrong square-H branch
    diag = np.repeat([1.0, 2.5, 4.0], 20)
    A = S.diagonal(diag)
    b = S.uniform_vector(60, 1)
    lam, sig = O.newton_shifts(4, 3, 1.0, 4.0)
    c, theta, delta = O.chebyshev_inverse_coeffs(3, 1.0, 4.0)
    beta = np.linalg.norm(b)

    def apply_M(v):
        return O.spmv(A, O.poly_chebyshev(A, v, c, theta, delta))

    Q, H, y, rho = O.sstep_cycle(apply_M, b / beta, 8, 4, lam, sig, beta, 0.0)
    assert H.shape == (3, 3) and len(Q) == 3 and rho < 1e-12 * beta
    x, hist, iters = O.sstep_gmres(A, b, np.zeros(60), 4, 8, 3, 1.0, 4.0, 1e-13, 2)
    np.testing.assert_allclose(x, b / diag, rtol=1e-12)
    assert iters == 3 and hist[-1] < 1e-13


def test_eigenvector_right_hand_side_is_solved_in_one_column():
    # b an eigenvector of A: W_1 is parallel to q_0, the first column is dependent and
    # H is 1 x 1; x = b / lambda exactly
    n = 15
    A = S.laplacian_1d(n)
    j = 11
    lam = 2 - 2 * math.cos(j * math.pi / (n + 1))
    b = np.sin(j * math.pi * np.arange(1, n + 1) / (n + 1))
    lmin, lmax = lap_bounds((n,))
    x, hist, iters = O.sstep_gmres(A, b, np.zeros(n), 4, 8, 4, lmin, lmax, 1e-12, 2)
    assert iters == 1
    np.testing.assert_allclose(x, b / lam, atol=1e-13)


@pytest.mark.parametrize("values", [None, np.float32])
def test_solve_matches_direct_solver(values):
    # the converged iterate equals SciPy's sparse direct solution within
    # cond(A) * tol; the reported history is the true residual
    # catches: a wrong final map x = x0 + s(A) Q y (for instance without s(A))
    A = S.knn_graph_laplacian(1500, seed=2)
    n, rp, c, v = A
    lmin, lmax = 0.1, 2.0 * float(np.max(np.diff(rp))) + 0.1
    b = S.uniform_vector(n, 5)
    x, hist, iters = O.sstep_gmres(A, b, np.zeros(n), 8, 32, 8, lmin, lmax, 1e-10, 40, values=values)
    ref = spla.spsolve(csr_matrix((v, c, rp), shape=(n, n)).tocsc(), b)
    true = np.linalg.norm(b - O.spmv(A, x)) / np.linalg.norm(b)
    assert hist[-1] <= 1e-10 and abs(true - hist[-1]) <= 1e-14
    cond = lmax / lmin
    assert np.linalg.norm(x - ref) <= 2 * cond * 1e-10 * np.linalg.norm(ref)
    if values is not None:       # the 0.1 shift is not representable: several cycles
        assert len(hist) > 2


def test_max_cycles_zero_returns_the_initial_guess():
    A = S.laplacian_2d(6)
    b = S.uniform_vector(36, 1)
    x0 = S.uniform_vector(36, 2)
    x, hist, iters = O.sstep_gmres(A, b, x0, 4, 8, 4, *lap_bounds((6, 6)), 1e-12, 0)
    assert np.array_equal(x, x0) and iters == 0 and len(hist) == 1


# ------------------------------------------- without / with the Jacobi preconditioner (R22)
def test_interval_shifts_polynomial_bounded():
    # the shift polynomial over [lo, hi] is 2 T_s((mu - c)/h) with the column scaling h/2
    lo, hi = 0.3, 7.9
    c, h = 0.5 * (hi + lo), 0.5 * (hi - lo)
    for s in (1, 3, 8):
        lam, sig = O.interval_shifts(s, lo, hi)
        mu = np.linspace(lo, hi, 33)
        prod = np.ones_like(mu)
        for k in range(s):
            prod *= (mu - lam[k]) / sig[k]
        np.testing.assert_allclose(prod, 2.0 * cheb_T(s, (mu - c) / h), atol=1e-9)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("s,m", [(1, 10), (3, 12), (4, 12), (5, 10)])
def test_preconditioned_cycle_equals_textbook_gmres(precond, s, m):
    # one cycle equals textbook GMRES (Alg. 3b) on the dense operator M = A or A D^{-1},
    # mapped back by x = Q y or D^{-1} Q y
    # catches: a missing D^{-1} in the final map, the operator without the column scaling
    A = S.random_pattern(60, 5, 13, symmetric=False)
    Ad = dense(A)
    Ad[np.arange(60), np.arange(60)] = 2.0 + np.abs(Ad).sum(axis=1) * np.linspace(1, 3, 60)
    A = S.from_dense(Ad)
    dg = np.diag(Ad)
    M = Ad / dg[None, :] if precond == "jacobi" else Ad
    b = S.uniform_vector(60, 4)
    ev = np.linalg.eigvals(M)
    lo, hi = float(ev.real.min()) * 0.9, float(ev.real.max()) * 1.1
    x1, hist, iters = O.sstep_gmres_precond(A, b, np.zeros(60), s, m, precond, lo, hi, 0.0, 1)
    u = textbook_gmres_cycle(M, b, m)
    x_ref = u / dg if precond == "jacobi" else u
    assert iters == m
    np.testing.assert_allclose(x1, x_ref, rtol=0, atol=1e-9 * np.abs(x_ref).max())


@pytest.mark.parametrize("values", [None, np.float32])
def test_jacobi_gmres_solves_knn_laplacian(values):
    # converged solution against SciPy's direct solve; Jacobi bounds: B = A D^{-1} is similar
    # to D^{-1/2} A D^{-1/2}, whose spectrum lies in (0, 2) by Gershgorin for this Laplacian
    A = S.knn_graph_laplacian(1500, seed=2)
    n, rp, c, v = A
    b = S.uniform_vector(n, 5)
    x, hist, iters = O.sstep_gmres_precond(A, b, np.zeros(n), 8, 48, "jacobi", 0.002, 2.0, 1e-10, 60,
                                           values=values)
    ref = spla.spsolve(csr_matrix((v, c, rp), shape=(n, n)).tocsc(), b)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(x - ref) <= 2e-10 * 2000 * np.linalg.norm(ref)


@pytest.mark.parametrize("gamma", [0, 1, 2])
@pytest.mark.parametrize("s,m", [(1, 9), (3, 12), (4, 12)])
def test_gs2_cycle_equals_textbook_gmres(gamma, s, m):
    # M = A P^{-1} with P^{-1} = sum_{i<=gamma} (-D^{-1} L)^i D^{-1} built densely; one
    # cycle equals textbook GMRES on M, mapped back by x = P^{-1} Q y
    # catches: the final map without P^{-1}, the operator without the preconditioner
    A = S.random_pattern(50, 5, 17, symmetric=False)
    Ad = dense(A)
    Ad[np.arange(50), np.arange(50)] = 1.0 + np.abs(Ad).sum(axis=1)
    A = S.from_dense(Ad)
    D = np.diag(np.diag(Ad))
    N = -np.linalg.solve(D, np.tril(Ad, -1))
    P = sum(np.linalg.matrix_power(N, i) for i in range(gamma + 1)) @ np.linalg.inv(D)
    M = Ad @ P
    b = S.uniform_vector(50, 8)
    ev = np.linalg.eigvals(M)
    lo, hi = float(ev.real.min()) * 0.9, float(ev.real.max()) * 1.1
    x1, hist, iters = O.sstep_gmres_precond(A, b, np.zeros(50), s, m, "gs2", lo, hi, 0.0, 1, gamma=gamma)
    x_ref = P @ textbook_gmres_cycle(M, b, m)
    assert iters == m
    np.testing.assert_allclose(x1, x_ref, rtol=0, atol=1e-9 * np.abs(x_ref).max())


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("s,m", [(1, 9), (4, 12)])
def test_jacobi_k_sweeps_cycle_equals_textbook_gmres(k, s, m):
    # P^{-1} = sum_{i<k} (I - D^{-1} A)^i D^{-1} built densely (the paper's Jacobi iteration
    # from zero); one cycle equals textbook GMRES on M = A P^{-1}, mapped back by P^{-1}
    A = S.random_pattern(50, 5, 23, symmetric=False)
    Ad = dense(A)
    Ad[np.arange(50), np.arange(50)] = 1.0 + np.abs(Ad).sum(axis=1)
    A = S.from_dense(Ad)
    Dinv = np.diag(1.0 / np.diag(Ad))
    N = np.eye(50) - Dinv @ Ad
    P = sum(np.linalg.matrix_power(N, i) for i in range(k)) @ Dinv
    M = Ad @ P
    b = S.uniform_vector(50, 6)
    ev = np.linalg.eigvals(M)
    lo, hi = float(ev.real.min()) * 0.9, float(ev.real.max()) * 1.1
    x1, hist, iters = O.sstep_gmres_precond(A, b, np.zeros(50), s, m, "jacobi", lo, hi, 0.0, 1, ksweeps=k)
    x_ref = P @ textbook_gmres_cycle(M, b, m)
    assert iters == m
    np.testing.assert_allclose(x1, x_ref, rtol=0, atol=1e-9 * np.abs(x_ref).max())


# ---- Newton shifts from Ritz values (reading R24) ---------------------------------------
def test_arnoldi_relation_and_orthonormal_basis():
    # M Q[:k] = Q H with Q orthonormal, on a nonsymmetric dense operator
    A = S.random_pattern(40, 5, 3, symmetric=False)
    M = dense(A)
    q0 = S.uniform_vector(40, 1)
    q0 = q0 / np.linalg.norm(q0)
    Q, H = O.arnoldi(lambda v: M @ v, q0, 8)
    assert Q.shape == (9, 40) and H.shape == (9, 8)
    np.testing.assert_allclose(Q @ Q.T, np.eye(9), atol=1e-12)
    np.testing.assert_allclose(M @ Q[:8].T, Q.T @ H, atol=1e-11)
    assert np.all(np.tril(H, -2) == 0.0)


@pytest.mark.parametrize("k", [3, 6])
def test_ritz_values_are_eigenvalues_of_the_projected_operator(k):
    # independent construction: an orthonormal basis of the Krylov space from numpy's QR
    # of [q0, M q0, ..., M^{k-1} q0]; the Ritz values are the eigenvalues of V^T M V
    # catches: eigenvalues of a rectangular or shifted block of H, a transposed H
    A = S.random_pattern(30, 4, 5, symmetric=False)
    M = dense(A)
    M[np.arange(30), np.arange(30)] += 3.0
    q0 = S.uniform_vector(30, 2)
    q0 = q0 / np.linalg.norm(q0)
    K = np.empty((30, k))
    K[:, 0] = q0
    for j in range(1, k):
        K[:, j] = M @ K[:, j - 1]
    V, _ = np.linalg.qr(K)
    ref = np.linalg.eigvals(V.T @ M @ V)
    lam, sig = O.ritz_shifts(lambda v: M @ v, q0, k)
    np.testing.assert_allclose(np.sort(lam), np.sort(ref.real), rtol=1e-9, atol=1e-10)
    assert np.allclose(sig, (lam.max() - lam.min()) / 4)


def test_ritz_shifts_on_a_diagonal_operator_are_its_entries_in_leja_order():
    # s = n distinct entries: the Krylov space is everything, the Ritz values are exact
    d = np.array([0.5, 3.0, 1.25, 2.0, 4.5, 0.75])
    q0 = np.ones(6) / math.sqrt(6)
    lam, sig = O.ritz_shifts(lambda v: d * v, q0, 6)
    np.testing.assert_allclose(lam, O.leja_order(d), rtol=1e-10)
    assert lam[0] == pytest.approx(4.5) and sig[0] == pytest.approx((4.5 - 0.5) / 4)


def test_ritz_shifts_stop_on_an_invariant_subspace_and_repeat():
    # three distinct eigenvalues: Arnoldi stops after three steps with the exact values,
    # and the shifts repeat them cyclically
    d = np.array([1.0, 1.0, 2.0, 2.0, 5.0, 5.0])
    q0 = np.ones(6) / math.sqrt(6)
    Q, H = O.arnoldi(lambda v: d * v, q0, 5)
    assert H.shape == (3, 3)
    lam, _ = O.ritz_shifts(lambda v: d * v, q0, 5)
    np.testing.assert_allclose(lam, [5.0, 1.0, 2.0, 5.0, 1.0], rtol=1e-10)


def test_symmetric_operator_gives_a_tridiagonal_hessenberg():
    A = S.laplacian_2d(7, 6)
    M = dense(A)
    q0 = S.uniform_vector(42, 3)
    q0 = q0 / np.linalg.norm(q0)
    _, H = O.arnoldi(lambda v: M @ v, q0, 8)
    assert np.abs(np.triu(H, 2)).max() < 1e-12


def test_complex_pairs_give_their_real_part():
    # a rotation block [[1, -2], [2, 1]] and a real eigenvalue 4: Ritz values 1 +- 2i, 4
    M = np.array([[1.0, -2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 4.0]])
    q0 = np.array([1.0, 1.0, 1.0]) / math.sqrt(3)
    lam, sig = O.ritz_shifts(lambda v: M @ v, q0, 3)
    np.testing.assert_allclose(lam, [4.0, 1.0, 1.0], rtol=1e-10)
    assert sig[0] == pytest.approx(0.75)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_gmres_with_ritz_shifts_solves_knn_laplacian(precond):
    # no spectrum interval given: the shifts come from the first cycle's Arnoldi steps;
    # the converged solution against SciPy's direct solve
    A = S.knn_graph_laplacian(1500, seed=2)
    n, rp, c, v = A
    b = S.uniform_vector(n, 5)
    x, hist, iters = O.sstep_gmres_precond(A, b, np.zeros(n), 8, 48, precond, None, None, 1e-10, 80)
    ref = spla.spsolve(csr_matrix((v, c, rp), shape=(n, n)).tocsc(), b)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(x - ref) <= 2e-10 * 2000 * np.linalg.norm(ref)


def test_one_cycle_with_ritz_shifts_equals_textbook_gmres():
    # GMRES's iterate depends on the Krylov space only, not on the shifts of its basis
    A = S.random_pattern(60, 5, 11, symmetric=False)
    Ad = dense(A)
    Ad[np.arange(60), np.arange(60)] = 1.0 + np.abs(Ad).sum(axis=1)
    A = S.from_dense(Ad)
    b = S.uniform_vector(60, 4)
    x1, hist, iters = O.sstep_gmres_precond(A, b, np.zeros(60), 4, 12, "none", None, None, 0.0, 1)
    u = textbook_gmres_cycle(Ad, b, 12)
    assert iters == 12
    np.testing.assert_allclose(x1, u, rtol=0, atol=1e-9 * np.abs(u).max())
