"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
exact integer arithmetic, closed-form Laplacian eigenpairs and grid levels,
SciPy's shortest paths, hand-worked fixtures, brute force and special cases.
Each test names the plausible oracle mistake it would catch."""
import math
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle as O
import synth as S

EPS = np.finfo(np.float64).eps


def dense(A):
    n, rp, c, v = A
    M = np.zeros((n, n))
    for i in range(n):
        M[i, c[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return M


def int_dense(A):
    n, rp, c, v = A
    M = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        M[i, c[rp[i]:rp[i + 1]]] = np.asarray(v[rp[i]:rp[i + 1]]).astype(np.int64)
    return M


# ----------------------------------------------------------------- SpMV / MPK
def test_spmv_sums_each_row_in_stored_order_from_zero():
    # catches: a summation order other than the stored (ascending-column) order,
    # or a fused multiply-add.  Row 0 holds 1e16, 1, -1e16 against x = 1: left to
    # right, 1e16 + 1 rounds back to 1e16 (the spacing there is 2), so the row
    # sums to exactly 0; any order that pairs 1e16 with -1e16 first gives 1.
    # Row 1: 0.1 * 3 is rounded before the addition of -0.3, leaving 2^-54
    # (an FMA would return 0.1 * 3 - 0.3 exactly, about 1.67e-17).
    A = (2, np.array([0, 3, 5]), np.array([0, 1, 2, 0, 1]),
         np.array([1e16, 1.0, -1e16, 0.1, -0.3]))
    y = O.spmv(A, np.array([1.0, 1.0, 1.0]))
    assert y[0] == 0.0
    A1 = (2, np.array([0, 0, 2]), np.array([0, 1]), np.array([0.1, -0.3]))
    y1 = O.spmv(A1, np.array([3.0, 1.0]))
    assert y1[1] == 2.0 ** -54 and y1[0] == 0.0


@pytest.mark.parametrize("seed", range(5))
def test_spmv_within_rounding_of_exact_row_sums(seed):
    # catches: dropped or duplicated entries, a wrong column, a transposed
    # operand: every row must agree with its exactly rounded sum (math.fsum over
    # the exact products, computed here from the dense matrix) within the
    # recursive-summation bound (row length) * eps * sum |a_ij x_j|
    A = S.random_pattern(40, 6, seed)
    x = S.uniform_vector(40, seed + 100)
    M = dense(A)
    y = O.spmv(A, x)
    for i in range(A.n):
        terms = [M[i, j] * x[j] for j in range(A.n) if M[i, j] != 0.0]
        bound = (len(terms) + 1) * EPS * sum(abs(t) for t in terms)
        assert abs(y[i] - math.fsum(terms)) <= bound


@pytest.mark.parametrize("mk", [lambda: S.laplacian_2d(5, 7), lambda: S.laplacian_3d(3, 4, 2),
                                lambda: S.random_pattern(50, 5, 3, integer=True)])
@pytest.mark.parametrize("p", [1, 2, 5, 8])
def test_mpk_exact_against_integer_dense_powers(mk, p):
    # catches: dropped/duplicated powers, wrong operand (A^T), index slips
    A = mk()
    x = S.integer_vector(A.n, 7, bound=1 << 16)
    M = int_dense(A)
    y = x.astype(np.int64)
    Y = O.mpk(A, x, p)
    for k in range(p):
        y = M @ y
        assert np.array_equal(Y[k], y.astype(np.float64)), k


# ------------------------------------------- reduced-precision values (R11)
def test_round_values_known_constants():
    # catches: rounding to the wrong precision, truncation instead of nearest,
    # or values that are not widened back exactly
    from fractions import Fraction
    A = S.from_dense([[0.1, 1.0 / 3.0], [2.0 ** -30, -6.0]])
    got = [Fraction(float(v)) for v in O.round_values(A).val]
    # 0.1 = 1.6 * 2^-4 and 1.6 * 2^23 = 13421772.8, so the nearest FP32 is 13421773 * 2^-27
    assert got[0] == Fraction(13421773, 2 ** 27)
    # 1/3 lies in [2^-2, 2^-1), where FP32 spacing is 2^-25: 2^25 / 3 = 11184810.67
    # rounds up to 11184811
    assert got[1] == Fraction(11184811, 2 ** 25)
    assert got[2] == Fraction(1, 2 ** 30) and got[3] == -6
    assert O.round_values(A).col is A.col and O.round_values(A).rowptr is A.rowptr


def test_reduced_precision_mpk_exact_for_representable_values():
    # catches: a reduced-precision path that changes anything but the values
    A = S.laplacian_3d(6, 5, 4)
    x = S.integer_vector(A.n, 3, bound=1 << 16)
    assert np.array_equal(O.mpk(O.round_values(A), x, 6), O.mpk(A, x, 6))


@pytest.mark.parametrize("p", [1, 4, 8])
def test_reduced_precision_mpk_within_perturbation_bound(p):
    # |A~ - A| <= u |A| elementwise with u = 2^-24 gives, in exact arithmetic,
    # |A~^p x - A^p x| <= ((1 + u)^p - 1) |A|^p |x|; FP64 rounding adds far less
    # than the 1e-12 slack.  catches: errors beyond single rounding of A, e.g. a
    # rounded vector or FP32 accumulation
    A = S.knn_graph_laplacian(2000, k=26, seed=4)
    x = S.uniform_vector(A.n, 5)
    u = 2.0 ** -24
    absA = A._replace(val=np.abs(A.val))
    bound = O.mpk(absA, np.abs(x), p)
    err = np.abs(O.mpk(O.round_values(A), x, p) - O.mpk(A, x, p))
    for k in range(p):
        assert np.all(err[k] <= ((1 + u) ** (k + 1) - 1) * bound[k] * (1 + 1e-12) + 1e-300), k
    assert err.max() > 0  # the 0.1 shift is not representable: rounding did happen


# ------------------------------- Chebyshev preconditioner and refinement (R12, R13)
def _cheb_T(d, u):
    """T_d(u) in closed form: cos(d arccos u) inside [-1, 1], cosh outside."""
    u = np.asarray(u, dtype=np.float64)
    inside = np.abs(u) <= 1
    out = np.empty_like(u)
    out[inside] = np.cos(d * np.arccos(u[inside]))
    uo = u[~inside]
    out[~inside] = np.sign(uo) ** d * np.cosh(d * np.arccosh(np.abs(uo)))
    return out


@pytest.mark.parametrize("d", [1, 2, 5, 8, 16])
def test_chebyshev_inverse_residual_polynomial(d):
    # 1 - lam s(lam) must equal T_d((theta - lam)/delta) / T_d(theta/delta) everywhere.
    # catches: wrong nodes, a missing halving of c_0, a sign flip of the argument
    lmin, lmax = 0.1, 24.0
    c, theta, delta = O.chebyshev_inverse_coeffs(d, lmin, lmax)
    lam = np.concatenate([np.random.default_rng(d).uniform(lmin, lmax, 50), [lmin, lmax, 0.05, 30.0]])
    u = (lam - theta) / delta
    s_val = sum(ck * _cheb_T(k, u) for k, ck in enumerate(c))
    want = _cheb_T(d, (theta - lam) / delta) / _cheb_T(d, np.array([theta / delta]))[0]
    assert np.allclose(1 - lam * s_val, want, rtol=0, atol=1e-12 * np.maximum(1, np.abs(want)))


def test_refinement_step_on_diagonal_contracts_by_residual_polynomial():
    # with A = diag(lam) (FP32-exact values), e_{i+1} = (1 - lam s(lam)) e_i componentwise.
    # catches: a wrong sign in the update, residuals taken with the rounded matrix
    lam = np.array([0.25, 0.5, 1.0, 3.0, 7.5, 12.0])
    A = S.diagonal(lam)
    xs = np.array([1.0, -2.0, 0.5, 3.0, -1.0, 2.0])
    b = lam * xs
    x1, hist = O.refine_solve(A, b, np.zeros(6), 4, 0.25, 12.0, 0.0, 1)
    c, theta, delta = O.chebyshev_inverse_coeffs(4, 0.25, 12.0)
    rho = _cheb_T(4, (theta - lam) / delta) / _cheb_T(4, np.array([theta / delta]))[0]
    assert np.allclose(x1 - xs, rho * (0 - xs), atol=1e-13)
    assert len(hist) == 2 and hist[0] == 1.0


def test_refine_solve_reaches_direct_solution():
    # catches: an update that stalls or converges to the wrong vector
    from scipy.sparse import csr_matrix
    from scipy.sparse.linalg import spsolve
    A = S.knn_graph_laplacian(1500, k=26, seed=2)
    b = S.uniform_vector(A.n, 9)
    lmax = 2.0 * np.max(np.diff(A.rowptr)) + 0.1  # Gershgorin bound
    x, hist = O.refine_solve(A, b, np.zeros(A.n), 16, 0.1, lmax, 1e-10, 300)
    assert hist[-1] <= 1e-10 and len(hist) < 300
    xs = spsolve(csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).tocsc(), b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert all(h1 < h0 for h0, h1 in zip(hist, hist[1:]))  # each step contracts


def test_bf16_rounding_hand_constants():
    # BF16 keeps 8 significant bits: near 1 the spacing is 2^-7.  catches: truncation
    # instead of rounding, ties rounded away from even, a wrong bit count
    from oracle import mpk_oracle as M
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2.0 ** -20 * 1.75],
                 dtype=np.float32)
    want = [1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -6, -1.0, 2.0 ** -20 * 1.75]
    assert [float(t) for t in M._bf16_rne(v)] == want


def test_bf16_rowscale_hand_worked():
    # row [6, -1, 0.1]: s = 6, q = bf16(1), bf16(-1/6), bf16(0.1/6).  -1/6 lies in
    # [2^-3, 2^-2) where BF16 spacing is 2^-10: 1024/6 = 170.67 -> 171, so the entry
    # becomes -6 * 171/1024; 0.1/6 = 0.016667 in [2^-6, 2^-5), spacing 2^-13:
    # 8192 * 0.016667 = 136.53 -> 137 (via its FP32 value), entry 6 * 137/8192.
    # catches: scaling by something other than the row maximum, a lost sign
    from fractions import Fraction
    A = S.from_dense([[6.0, -1.0, 0.1], [0.0, 0.0, 0.0], [1.0 / 3.0, 0.0, 2.0]])
    got = [Fraction(float(v)) for v in O.round_values_bf16_rowscale(A).val]
    assert got[:3] == [Fraction(6), Fraction(-6 * 171, 1024), Fraction(6 * 137, 8192)]
    # row 2: s = 2, 1/6 -> 171/1024 again
    assert got[3:] == [Fraction(2 * 171, 1024), Fraction(2)]


@pytest.mark.parametrize("p", [1, 4, 8])
def test_bf16_rowscale_mpk_within_perturbation_bound(p):
    # |a~ - a| <= (2^-8 + 2^-22) |a| (BF16 rounding plus the FP32 quotient and scale
    # roundings), so |A~^k x - A^k x| <= ((1 + u)^k - 1) |A|^k |x|.  catches: a scale
    # applied twice, a missing scale, precision lost beyond one BF16 rounding
    A = S.laplacian_3d(9, 8, 7)
    x = S.uniform_vector(A.n, 2)
    u = 2.0 ** -8 + 2.0 ** -22
    bound = O.mpk(A._replace(val=np.abs(A.val)), np.abs(x), p)
    err = np.abs(O.mpk(O.round_values_bf16_rowscale(A), x, p) - O.mpk(A, x, p))
    for k in range(p):
        assert np.all(err[k] <= ((1 + u) ** (k + 1) - 1) * bound[k] * (1 + 1e-12)), k
    assert err.max() > 0  # -1/6 is not a BF16 value: the stencil is perturbed


def test_mpk_hand_worked_grid3x3(golden_dir):
    rows = {}
    with open(os.path.join(golden_dir, "grid3x3_power2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tag, *vals = line.split()
            rows[tag] = np.array([float(v) for v in vals])
    A = S.laplacian_2d(3)
    x = np.zeros(9)
    x[4] = 1.0
    Y = O.mpk(A, x, 2)
    assert np.array_equal(Y[0], rows["y1"])
    assert np.array_equal(Y[1], rows["y2"])


def _sine_mode_1d(n, j):
    i = np.arange(1, n + 1)
    return np.sin(j * np.pi * i / (n + 1)), 2.0 - 2.0 * math.cos(j * math.pi / (n + 1))


def _grid_mode(shape, js):
    vec = np.ones(1)
    lam = 0.0
    # row index i + nx*(j + ny*k): the first axis varies fastest
    for n, j in reversed(list(zip(shape, js))):
        v, l = _sine_mode_1d(n, j)
        vec = np.kron(vec, v)
        lam += l
    return vec, lam


@pytest.mark.parametrize("case", [("1d", (30,), (25,)), ("2d", (12, 9), (10, 8)),
                                  ("3d", (7, 6, 5), (6, 5, 4))])
@pytest.mark.parametrize("p", [1, 4, 8])
def test_mpk_laplacian_eigen_relation(case, p):
    # closed form: A^p v = lambda^p v for sine modes of the Dirichlet Laplacians
    # catches: wrong stencil sign or coefficient, a transposed or shifted index
    name, shape, js = case
    A = {"1d": lambda: S.laplacian_1d(*shape), "2d": lambda: S.laplacian_2d(*shape),
         "3d": lambda: S.laplacian_3d(*shape)}[name]()
    v, lam = _grid_mode(shape, js)
    normA = 4.0 * len(shape)
    assert lam >= normA / 2
    Y = O.mpk(A, v, p)
    for k in range(1, p + 1):
        err = np.linalg.norm(Y[k - 1] - lam ** k * v)
        bound = 20 * k * len(shape) * EPS * np.linalg.norm(v) * normA ** k
        assert err <= bound, (k, err, bound)


# ------------------------------------------------------------ polynomial forms
@pytest.mark.parametrize("seed", [0, 1])
def test_newton_basis_on_eigenvector(seed):
    # closed form: V_k = prod_{i<=k} (lambda - lambda_i) / sigma_i * v
    # catches: shift applied to the wrong vector, shifts out of order, sigma misuse
    shape, js = (11, 8), (9, 7)
    A = S.laplacian_2d(*shape)
    v, lam = _grid_mode(shape, js)
    rng = np.random.default_rng(seed)
    lambdas = rng.uniform(0, 2, 6)
    sigmas = rng.uniform(1, 3, 6)
    V = O.newton_basis(A, v, lambdas, sigmas)
    f = 1.0
    assert np.array_equal(V[0], v)
    for k in range(1, 7):
        f *= (lam - lambdas[k - 1]) / sigmas[k - 1]
        assert np.linalg.norm(V[k] - f * v) <= 1e-12 * np.linalg.norm(v) * 8 ** k


def test_newton_basis_integer_exact():
    A = S.laplacian_3d(4, 3, 3)
    x = S.integer_vector(A.n, 3, bound=1 << 12)
    lambdas = [1.0, -2.0, 3.0, 0.0]
    M = int_dense(A)
    y = x.astype(np.int64)
    V = O.newton_basis(A, x, lambdas)
    for k, lm in enumerate(lambdas, start=1):
        y = M @ y - int(lm) * y
        assert np.array_equal(V[k], y.astype(np.float64))


def test_poly_monomial_on_diagonal():
    # Eq. (3) on A = diag(d): (sum_k c_k d_i^k) x_i, evaluated by Horner's rule
    # catches: off-by-one in the coefficient index
    rng = np.random.default_rng(4)
    d = rng.uniform(-1.5, 1.5, 300)
    x = rng.uniform(-1, 1, 300)
    c = rng.uniform(-1, 1, 9)
    ref = np.zeros_like(d)
    for ck in c[::-1]:
        ref = ref * d + ck
    got = O.poly_monomial(S.diagonal(d), x, c)
    assert np.max(np.abs(got - ref * x)) <= 1e-13


def test_poly_newton_on_diagonal():
    rng = np.random.default_rng(5)
    d = rng.uniform(-1, 1, 200)
    x = rng.uniform(-1, 1, 200)
    c = rng.uniform(-1, 1, 7)
    lam = rng.uniform(-1, 1, 6)
    ref = np.zeros_like(d)
    phi = np.ones_like(d)
    for k in range(7):
        if k:
            phi = phi * (d - lam[k - 1])
        ref += c[k] * phi
    got = O.poly_newton(S.diagonal(d), x, c, lam)
    assert np.max(np.abs(got - ref * x)) <= 1e-13


@pytest.mark.parametrize("theta,delta", [(0.0, 1.0), (2.0, 1.9), (6.0, 5.5)])
def test_poly_chebyshev_on_diagonal(theta, delta):
    # closed form T_k(u) = cos(k arccos u) for |u| <= 1
    # catches: missing factor 2, wrong sign of t_{k-1}, theta/delta swapped
    rng = np.random.default_rng(6)
    u = rng.uniform(-1, 1, 400)
    d = theta + delta * u
    x = rng.uniform(-1, 1, 400)
    c = rng.uniform(-1, 1, 10)
    ref = sum(c[k] * np.cos(k * np.arccos(u)) for k in range(10))
    got = O.poly_chebyshev(S.diagonal(d), x, c, theta, delta)
    assert np.max(np.abs(got - ref * x)) <= 1e-12


def test_chebyshev_basis_on_laplacian_mode():
    shape, js = (10, 10), (8, 9)
    A = S.laplacian_2d(*shape)
    v, lam = _grid_mode(shape, js)
    theta, delta = 4.0, 4.0
    u = (lam - theta) / delta
    T = O.chebyshev_basis(A, v, 8, theta, delta)
    for k in range(9):
        assert np.linalg.norm(T[k] - math.cos(k * math.acos(u)) * v) <= 1e-12 * 3 ** k * np.linalg.norm(v)


# -------------------------------------------------------------- special cases
def test_special_cases():
    x = S.uniform_vector(37, 1)
    assert np.array_equal(O.mpk(S.identity(37), x, 5), np.tile(x, (5, 1)))
    d = S.uniform_vector(37, 2)
    Y = O.mpk(S.diagonal(d), x, 4)
    for k in range(4):
        ref = x.copy()
        for _ in range(k + 1):
            ref = d * ref
        assert np.array_equal(Y[k], ref)
    Y = O.mpk(S.cyclic_shift(37), x, 6)
    for k in range(6):
        assert np.array_equal(Y[k], np.roll(x, -(k + 1)))
    Z = S.CSR(37, np.zeros(38, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert np.array_equal(O.mpk(Z, x, 3), np.zeros((3, 37)))
    one = S.from_dense([[3.0]])
    assert np.array_equal(O.mpk(one, np.array([2.0]), 3)[:, 0], [6.0, 18.0, 54.0])


# --------------------------------------------------------------------- levels
def _levels_of(A, root=None):
    level, nl, roots = O.bfs_levels(A, root)
    return level, nl, roots


def test_levels_path_hand_worked(golden_dir):
    lines = [l.split() for l in open(os.path.join(golden_dir, "path7_levels.txt"))
             if l.strip() and not l.startswith("#")]
    edges = [tuple(map(int, e.split("-"))) for e in lines[0][1:]]
    root = int(lines[1][1])
    want = {int(a): int(b) for a, b in lines[2:]}
    M = np.eye(7) * 2
    for a, b in edges:
        M[a, b] = M[b, a] = -1
    level, nl, roots = _levels_of(S.from_dense(M))
    assert roots == [root]
    assert nl == 7
    assert {i: int(level[i]) for i in range(7)} == want


def test_levels_closed_forms():
    lv, nl, r = _levels_of(S.laplacian_1d(50))
    assert np.array_equal(lv, np.arange(50)) and nl == 50 and r == [0]
    nx, ny = 13, 9
    lv, nl, r = _levels_of(S.laplacian_2d(nx, ny))
    idx = np.arange(nx * ny)
    assert np.array_equal(lv, idx % nx + idx // nx) and nl == nx + ny - 1
    n3 = (6, 5, 4)
    lv, nl, r = _levels_of(S.laplacian_3d(*n3))
    idx = np.arange(np.prod(n3))
    i, j, k = idx % 6, (idx // 6) % 5, idx // 30
    assert np.array_equal(lv, i + j + k) and nl == 6 + 5 + 4 - 2
    # a directed cyclic shift symmetrises to a ring: level(i) = min(i, n - i)
    lv, nl, r = _levels_of(S.cyclic_shift(20))
    assert np.array_equal(lv, np.minimum(np.arange(20), 20 - np.arange(20)))


def test_levels_64x64_grid_count():
    lv, nl, _ = _levels_of(S.laplacian_2d(64))
    assert nl == 127
    counts = np.bincount(lv)
    ell = np.arange(127)
    assert np.array_equal(counts, np.minimum(ell + 1, 127 - ell))


def test_levels_single_long_range_entry():
    # upper triangular pattern with one entry (0, n-1): symmetrisation makes 0 and
    # n-1 neighbours (reading R1); every other row is its own component (R3)
    n = 9
    M = np.eye(n)
    M[0, n - 1] = 5.0
    lv, nl, roots = _levels_of(S.from_dense(M))
    want = np.array([0] + [i + 1 for i in range(1, n - 1)] + [1])
    assert np.array_equal(lv, want) and nl == n


def test_levels_explicit_root():
    lv, nl, roots = _levels_of(S.laplacian_2d(8, 8), root=27)
    i, j = np.arange(64) % 8, np.arange(64) // 8
    assert roots == [27]
    assert np.array_equal(lv, np.abs(i - 3) + np.abs(j - 3))


@pytest.mark.parametrize("seed", range(6))
def test_levels_against_scipy_and_invariants(seed):
    # SciPy's unweighted shortest paths are an independent BFS
    blocks = [S.random_pattern(60 + 10 * seed, 1.2 + 0.4 * (seed % 3), seed + b) for b in range(3)]
    A = S.block_diagonal(*blocks) if seed % 2 else blocks[0]
    n = A.n
    level, nl, roots = O.bfs_levels(A)
    ptr, adj = O.pattern_graph(A)
    G = csr_matrix((np.ones(adj.size), adj, ptr), shape=(n, n))
    D = shortest_path(G, unweighted=True, directed=False, indices=roots)
    assigned = np.zeros(n, dtype=bool)
    base = 0
    for r, drow in zip(roots, D):
        comp = np.isfinite(drow) & ~assigned
        assert np.array_equal(level[comp], base + drow[comp].astype(np.int64))
        base += int(drow[comp].max()) + 1
        assigned |= comp
    assert assigned.all() and base == nl
    # invariants: neighbours differ by <= 1 level, each non-root has a parent one level up
    rows = np.repeat(np.arange(n), np.diff(ptr))
    assert np.all(np.abs(level[rows] - level[adj]) <= 1)
    has_parent = np.zeros(n, dtype=bool)
    np.logical_or.at(has_parent, rows, level[adj] == level[rows] - 1)
    is_root = np.zeros(n, dtype=bool)
    is_root[roots] = True
    assert np.all(has_parent | is_root)
    # roots are the components' lowest vertices' pseudo-peripheral nodes: check
    # George-Liu's stopping rule holds (the last BFS does not increase the eccentricity)
    for r in roots:
        lay = O.bfs_layers(ptr, adj, r, np.full(n, -1, dtype=np.int64))
        last = lay[-1]
        xm = int(last[np.argmin(ptr[last + 1] - ptr[last])])
        lay_x = O.bfs_layers(ptr, adj, xm, np.full(n, -1, dtype=np.int64))
        assert len(lay_x) <= len(lay)


def test_bfs_queue_and_layers_agree():
    A = S.random_pattern(300, 2.5, 11)
    ptr, adj = O.pattern_graph(A)
    q = O.bfs_layers_queue(ptr, adj, 0, A.n)
    dist = np.full(A.n, -1, dtype=np.int64)
    O.bfs_layers(ptr, adj, 0, dist)
    assert list(dist) == q


def test_permutation_and_permuted_matrix():
    A = S.random_pattern(120, 4, 21, integer=True)
    level, nl, _ = O.bfs_levels(A)
    perm, iperm, level_ptr = O.level_permutation(level, nl)
    assert np.array_equal(np.sort(perm), np.arange(120))
    assert np.array_equal(perm[iperm], np.arange(120))
    assert np.all(np.diff(level[perm]) >= 0)
    for l in range(nl):
        seg = perm[level_ptr[l]:level_ptr[l + 1]]
        assert np.all(level[seg] == l) and np.all(np.diff(seg) > 0)
    B = O.permute_symmetric(A, perm, iperm)
    assert np.array_equal(dense(B), dense(A)[np.ix_(perm, perm)])
    x = S.integer_vector(120, 2, bound=1 << 10)
    assert np.array_equal(O.mpk(B, x[perm], 4), O.mpk(A, x, 4)[:, perm])


# ------------------------------------------ level groups and wavefront (R14, R15)
def test_group_levels_hand_worked_chain():
    # 1D chain of 10 rows from root 0: level l = row l; end rows hold 2 entries,
    # interior rows 3, so w = 2*12+20 = 44 or 3*12+20 = 56 bytes.  C = 1000, q = 4
    # gives B = 250: 44+56+56+56 = 212, +56 = 268 > 250 -> cut before level 4;
    # 4*56 = 224, +56 = 280 > 250 -> cut before level 8; 56+44 = 100.
    A = S.laplacian_1d(10)
    level, nl, _ = O.bfs_levels(A, 0)
    perm, iperm, lp = O.level_permutation(level, nl)
    assert list(O.group_levels(A, lp, perm, 1000, 4)) == [0, 4, 8, 10]
    # a floor of 5 rows per group keeps level 4 in group 0 (268 bytes, 5 rows) and
    # cuts before level 5; group 1 reaches 224 bytes at level 8 but holds only 4
    # rows when level 9 would overflow it, so it runs to the end
    assert list(O.group_levels(A, lp, perm, 1000, 4, min_group_rows=5)) == [0, 5, 10]
    # one group when everything fits; one level per group when nothing does
    assert list(O.group_levels(A, lp, perm, 10 ** 6, 4)) == [0, 10]
    assert list(O.group_levels(A, lp, perm, 4, 4)) == list(range(11))


def test_wavefront_schedule_hand_worked():
    # groups [0,3], [4,7], [8,9] over L = 10 levels, q = 2 (R15)
    tasks = O.wavefront_schedule(np.array([0, 4, 8, 10]), 2)
    assert tasks == [(0, 1, 0, 3), (1, 1, 4, 7), (1, 2, 0, 2), (2, 1, 8, 9), (2, 2, 3, 6), (3, 2, 7, 9)]


SCHED_CASES = {
    "lap3d": lambda: S.laplacian_3d(14, 11, 9),
    "lap2d": lambda: S.laplacian_2d(40, 31),
    "rand_nonsym": lambda: S.random_pattern(1500, 4, 5),
    "disconnected": lambda: S.block_diagonal(S.laplacian_2d(9, 8), S.identity(30), S.laplacian_1d(90)),
    "knn": lambda: S.knn_graph_laplacian(1200, k=26, seed=3),
}


def _sched_setup(A):
    level, nl, _ = O.bfs_levels(A)
    perm, iperm, lp = O.level_permutation(level, nl)
    return O.permute_symmetric(A, perm, iperm), perm, lp


@pytest.mark.parametrize("name", sorted(SCHED_CASES))
@pytest.mark.parametrize("cache,q", [(20_000, 2), (60_000, 4), (5_000, 5), (10 ** 9, 3)])
def test_schedule_valid_and_equal_to_plain(name, cache, q):
    # P5: coverage, read-after-write order, one task per k per stage, G + q - 1
    # stages; executing it gives the plain MPK bitwise
    A = SCHED_CASES[name]()
    B, perm, lp = _sched_setup(A)
    gp = O.group_levels(A, lp, perm, cache, q)
    tasks = O.wavefront_schedule(gp, q)
    O.validate_schedule(B, lp, tasks, q)
    assert max(t[0] for t in tasks) <= len(gp) - 1 + q - 1
    x = S.uniform_vector(A.n, 1)
    p = 2 * q + 1  # two full blocks and a remainder
    got = O.run_schedule(B, x, p, q, lp, lambda qb: O.wavefront_schedule(gp, qb))
    assert np.array_equal(got, O.mpk(B, x, p))


def test_schedule_validator_catches_planted_mistakes():
    # mistakes planted in the oracle's own schedule must be rejected
    A = S.laplacian_2d(30, 20)
    B, perm, lp = _sched_setup(A)
    gp = O.group_levels(A, lp, perm, 8_000, 3)
    assert len(gp) > 4
    tasks = O.wavefront_schedule(gp, 3)
    # 1) run power 2 of group 1 one stage early (before its inputs exist)
    bad = [(s - 1, k, lo, hi) if (k == 2 and s == 2) else (s, k, lo, hi) for s, k, lo, hi in tasks]
    with pytest.raises(AssertionError):
        O.validate_schedule(B, lp, bad, 3)
    # 2) forget the shift by k - 1 levels (reads the next group's fresh rows)
    L = int(gp[-1])
    G = len(gp) - 1
    noshift = [(g + k - 1, k, int(gp[g]), L - 1 if g == G - 1 else int(gp[g + 1]) - 1)
               for g in range(G) for k in range(1, 4)]
    with pytest.raises(AssertionError):
        O.validate_schedule(B, lp, sorted(noshift), 3)
    # 3) drop a task (rows never computed)
    with pytest.raises(AssertionError):
        O.validate_schedule(B, lp, tasks[:-1], 3)


# ------------------------------------------------- plain C reference (mpk_ref.c)
@pytest.fixture(scope="module")
def ref_c():
    from oracle import ref_c as R
    if not os.path.exists(R.LIB):
        R.build()
    return R


@pytest.mark.parametrize("mk", [lambda: S.laplacian_3d(6, 5, 4), lambda: S.random_pattern(80, 5, 6, integer=True),
                                lambda: S.block_diagonal(S.identity(7), S.laplacian_1d(20))])
def test_c_reference_exact_against_integer_dense_powers(ref_c, mk):
    # catches: a dropped power, a transposed operand, an off-by-one in the row loop
    A = mk()
    x = S.integer_vector(A.n, 3, bound=1 << 14)
    M = int_dense(A)
    y = x.astype(np.int64)
    Y = ref_c.mpk(A, x, 6)
    for k in range(6):
        y = M @ y
        assert np.array_equal(Y[k], y.astype(np.float64)), k


@pytest.mark.parametrize("seed", range(4))
def test_c_reference_equals_numpy_oracle_bitwise(ref_c, seed):
    # both sum each row in stored order from zero without fused multiply-adds; the
    # OpenMP split over rows leaves every row's sum to one thread
    A = S.random_pattern(4000, 7, seed) if seed % 2 else S.knn_graph_laplacian(3000, k=12, seed=seed)
    x = S.uniform_vector(A.n, seed + 7)
    ref = O.mpk(A, x, 5)
    assert np.array_equal(ref_c.mpk(A, x, 5), ref)
    Y, used = ref_c.mpk_omp(A, x, 5, 4)
    assert used >= 1 and np.array_equal(Y, ref)


def test_c_reference_order_sensitive_case(ref_c):
    # the hand-worked order case of the SpMV pin: 1e16 + 1 - 1e16 = 0 left to right
    A = S.CSR(3, np.array([0, 3, 3, 3], dtype=np.int32), np.array([0, 1, 2], dtype=np.int32),
              np.array([1e16, 1.0, -1e16]))
    assert ref_c.mpk(A, np.ones(3), 1)[0, 0] == 0.0
