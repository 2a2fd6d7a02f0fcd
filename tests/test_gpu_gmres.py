"""GPU parity of the s-step GMRES solve (Sec. 4, Alg. 3a/3c, with the right Chebyshev
polynomial preconditioner of Sec. 5; readings R17-R19) through the C ABI.

The GPU computes a Newton basis step (M - lambda I) v / sigma as one Chebyshev
polynomial of degree d in A (M = I - T_d((theta I - A)/delta) / T_d(theta/delta)),
the oracle as A (s(A) v); Gram products, Cholesky factors and least squares differ
from the oracle's only in rounding order.  So after a fixed number of cycles the
iterates agree to a tolerance derived from that rounding: each basis vector differs
by O(d eps) relative, the least-squares problem of a cycle of m columns amplifies it
by at most its condition (here below 1e3), hence the bound 1e-9 relative below.
Blocked, plain and staged polynomial launches give bitwise equal vectors, and every
sum is reduced in a fixed order, so those runs and repeated runs are bitwise equal."""
import math

import numpy as np
import pytest

import scipy.sparse.linalg as spla
from scipy.sparse import csr_matrix

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU-only hosts, never run there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_02228_amd import Plan, MPKError  # noqa: E402

DEV = "cuda:0"
FIXED_CYCLE_RTOL = 1e-9
BLOCK_BASIS_RTOL = 1e-8


def lap_bounds(dims):
    return (sum(2 - 2 * math.cos(math.pi / (m + 1)) for m in dims),
            sum(2 + 2 * math.cos(math.pi / (m + 1)) for m in dims))


def knn_problem(n, seed):
    A = S.knn_graph_laplacian(n, k=26, seed=seed)
    lmax = 2.0 * np.max(np.diff(A.rowptr)) + 0.1  # Gershgorin; lmin = 0.1 is the shift
    return A, 0.1, lmax, S.uniform_vector(A.n, seed + 1)


def solve(hi, lo, b, s, m, d, lmin, lmax, tol, cycles, x0=None, **kw):
    """Runs the GPU solve in original row order; returns (x, iters, cycles, relres)."""
    perm = hi.levels()["perm"].astype(np.int64)
    xd = None if x0 is None else torch.tensor(x0[perm], device=DEV)
    x, it, cy, rel = hi.sstep_gmres(lo, torch.tensor(b[perm], device=DEV), s, m, d, lmin, lmax, tol=tol,
                                    max_cycles=cycles, x=xd, **kw)
    hi.check()
    lo.check()
    out = np.empty(b.size)
    out[perm] = x.cpu().numpy()
    return out, it, cy, rel


@pytest.mark.parametrize("s,m,d", [(1, 8, 4), (4, 16, 8), (8, 32, 8), (5, 12, 3), (8, 24, 1), (16, 48, 2)])
def test_fixed_cycle_matches_oracle_on_ragged_stencil(s, m, d):
    dims = (37, 29)
    A = S.laplacian_2d(*dims)
    lmin, lmax = lap_bounds(dims)
    b = S.uniform_vector(A.n, 3)
    hi = Plan.from_csr(A, p_block=4).upload(DEV)
    x, it, cy, rel = solve(hi, hi, b, s, m, d, lmin, lmax, 0.0, 1)
    xo, hist, ito = O.sstep_gmres(A, b, np.zeros(A.n), s, m, d, lmin, lmax, 0.0, 1)
    assert it == ito == m and cy == 1
    assert np.linalg.norm(x - xo) <= FIXED_CYCLE_RTOL * np.linalg.norm(xo)
    assert abs(rel - hist[-1]) <= 1e-6 * hist[-1] + 1e-13  # absolute floor: FP64 rounding of b - A x


@pytest.mark.parametrize("values", ["f64", "f32"])
def test_two_cycles_match_oracle_on_knn(values):
    A, lmin, lmax, b = knn_problem(20000, 0)
    hi = Plan.from_csr(A).upload(DEV)
    lo = hi if values == "f64" else Plan.from_csr(A, values="f32").upload(DEV)
    x, it, cy, rel = solve(hi, lo, b, 8, 16, 8, lmin, lmax, 0.0, 2)
    xo, hist, ito = O.sstep_gmres(A, b, np.zeros(A.n), 8, 16, 8, lmin, lmax, 0.0, 2,
                                  values=None if values == "f64" else np.float32)
    assert it == ito == 32 and cy == 2
    assert np.linalg.norm(x - xo) <= FIXED_CYCLE_RTOL * np.linalg.norm(xo)


@pytest.mark.parametrize("values", ["f64", "f32"])
def test_solve_to_1e10_like_oracle(values):
    A, lmin, lmax, b = knn_problem(20000, 3)
    hi = Plan.from_csr(A).upload(DEV)
    lo = hi if values == "f64" else Plan.from_csr(A, values="f32").upload(DEV)
    x, it, cy, rel = solve(hi, lo, b, 8, 32, 8, lmin, lmax, 1e-10, 50)
    xo, hist, ito = O.sstep_gmres(A, b, np.zeros(A.n), 8, 32, 8, lmin, lmax, 1e-10, 50,
                                  values=None if values == "f64" else np.float32)
    assert rel <= 1e-10 and cy == len(hist) - 1 and abs(it - ito) <= 8
    # the true residual, in FP64 on the host
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1.0000001e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 2e-10 * (lmax / lmin) * np.linalg.norm(xo)


def test_blocked_plain_staged_bitwise_and_io_orders():
    dims = (20, 18, 16)
    A = S.laplacian_3d(*dims)
    lmin, lmax = lap_bounds(dims)
    b = S.uniform_vector(A.n, 5)
    hi = Plan.from_csr(A, p_block=8).upload(DEV)
    xb, ib, cb, rb = solve(hi, hi, b, 8, 32, 8, lmin, lmax, 1e-10, 30)
    xp, ip, cp, rp = solve(hi, hi, b, 8, 32, 8, lmin, lmax, 1e-10, 30, plain=True)
    xs, is_, cs, rs = solve(hi, hi, b, 8, 32, 8, lmin, lmax, 1e-10, 30, staged=True)
    assert rb <= 1e-10 and np.array_equal(xb, xp) and np.array_equal(xb, xs) and ib == ip == is_
    # original-order I/O: the library permutes in and out
    x, it, cy, rel = hi.sstep_gmres(hi, torch.tensor(b, device=DEV), 8, 32, 8, lmin, lmax, tol=1e-10,
                                    max_cycles=30, permuted=False)
    assert np.array_equal(x.cpu().numpy(), xb) and it == ib
    # repeated calls are identical
    xr, ir, cr, rr = solve(hi, hi, b, 8, 32, 8, lmin, lmax, 1e-10, 30)
    assert np.array_equal(xr, xb) and rr == rb


def test_dependent_column_ends_cycle_exactly():
    # M has 3 distinct eigenvalues (d = 3): the 4th column of the first block is
    # dependent, the cycle ends with 3 columns and the solution is exact
    diag = np.repeat([1.0, 2.5, 4.0], 700)
    A = S.diagonal(diag)
    b = S.uniform_vector(A.n, 1)
    hi = Plan.from_csr(A).upload(DEV)
    x, it, cy, rel = solve(hi, hi, b, 4, 8, 3, 1.0, 4.0, 1e-13, 2)
    assert it == 3 and cy == 1 and rel <= 1e-13
    np.testing.assert_allclose(x, b / diag, rtol=1e-12)
    # an eigenvector right-hand side: one column
    n = 1000
    A = S.laplacian_1d(n)
    j = 600
    lam = 2 - 2 * math.cos(j * math.pi / (n + 1))
    b = np.sin(j * math.pi * np.arange(1, n + 1) / (n + 1))
    hi = Plan.from_csr(A).upload(DEV)
    x, it, cy, rel = solve(hi, hi, b, 4, 8, 4, *lap_bounds((n,)), 1e-11, 2)
    assert it == 1
    np.testing.assert_allclose(x, b / lam, atol=1e-11 * np.abs(b / lam).max())


def test_edge_cases():
    A = S.laplacian_2d(9, 7)
    lmin, lmax = lap_bounds((9, 7))
    hi = Plan.from_csr(A).upload(DEV)
    b = S.uniform_vector(A.n, 2)
    x0 = S.uniform_vector(A.n, 4)
    # no cycle: the initial guess comes back, with its residual
    x, it, cy, rel = solve(hi, hi, b, 4, 8, 4, lmin, lmax, 1e-10, 0, x0=x0)
    assert np.array_equal(x, x0) and it == 0 and cy == 0
    assert abs(rel - np.linalg.norm(b - O.spmv(A, x0)) / np.linalg.norm(b)) <= 1e-12
    # b = 0 from x0 = 0: nothing to do
    x, it, cy, rel = solve(hi, hi, np.zeros(A.n), 4, 8, 4, lmin, lmax, 1e-10, 5)
    assert not x.any() and it == 0 and rel == 0.0
    # a nonzero initial guess converges like the oracle
    x, it, cy, rel = solve(hi, hi, b, 3, 9, 5, lmin, lmax, 0.0, 1, x0=x0)
    xo, hist, ito = O.sstep_gmres(A, b, x0, 3, 9, 5, lmin, lmax, 0.0, 1)
    assert np.linalg.norm(x - xo) <= FIXED_CYCLE_RTOL * np.linalg.norm(xo)
    # N = 1
    one = S.diagonal(np.array([3.0]))
    h1 = Plan.from_csr(one).upload(DEV)
    x, it, cy, rel = solve(h1, h1, np.array([6.0]), 2, 4, 2, 1.0, 5.0, 1e-12, 3)
    assert abs(x[0] - 2.0) <= 1e-14 and it == 1
    # a work buffer that is too small is refused
    with pytest.raises(MPKError):
        hi.sstep_gmres(hi, torch.tensor(b, device=DEV), 4, 8, 4, lmin, lmax,
                       work=torch.empty(16, dtype=torch.float64, device=DEV))


@pytest.mark.slow
def test_full_size_160_cubed_mixed_precision_solve():
    # 3D 7-point 160^3 with FP32-valued basis and preconditioner, FP64 residuals, to 1e-10;
    # the true residual is recomputed on the host in FP64
    from scipy.sparse import csr_matrix
    n1 = 160
    A = S.laplacian_3d(n1)
    lmin, lmax = lap_bounds((n1, n1, n1))
    b = S.uniform_vector(A.n, 11)
    hi = Plan.from_csr(A, p_block=8).upload(DEV)
    lo = Plan.from_csr(A, p_block=8, values="f32").upload(DEV)
    x, it, cy, rel = solve(hi, lo, b, 8, 64, 32, lmin, lmax, 1e-10, 40)
    M = csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))
    true = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
    assert rel <= 1e-10 and true <= 1.0000001e-10 and abs(true - rel) <= 1e-12


# ------------------------------- without a preconditioner and with Jacobi (reading R22)
def jacobi_knn(n, seed, shift=0.1):
    # A D^{-1} is similar to D^{-1/2} A D^{-1/2}, whose spectrum lies in (0, 2) by
    # Gershgorin and above shift / (max degree + shift) since A >= shift I
    A = S.knn_graph_laplacian(n, k=26, seed=seed, shift=shift)
    dmax = float(np.max(np.diff(A.rowptr))) - 1.0
    return A, shift / (dmax + shift), 2.0


def gmres_plans(A, precond, values="f64", q=8):
    hi = Plan.from_csr(A, p_block=q).upload(DEV)
    if precond == "jacobi":
        lo = Plan.from_csr(A, p_block=q, values=values, column_scaling="jacobi").upload(DEV)
    else:
        lo = hi if values == "f64" else Plan.from_csr(A, p_block=q, values=values).upload(DEV)
    return hi, lo


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("values", ["f64", "f32"])
@pytest.mark.parametrize("s,m", [(1, 8), (4, 16), (8, 32), (5, 12)])
def test_fixed_cycle_without_and_with_jacobi_matches_oracle(precond, values, s, m):
    if precond == "none":
        dims = (37, 29)
        A = S.laplacian_2d(*dims)
        lmin, lmax = lap_bounds(dims)
    else:
        # well-conditioned Newton blocks (shift 2): with the 0.1 shift an 8-column block
        # over [0.003, 2] is so ill-conditioned that Cholesky QR, which squares the
        # condition, lets two correct runs differ in the third digit after one cycle;
        # that case is covered by the converged solve below
        A, lmin, lmax = jacobi_knn(6000, 2, shift=2.0)
    b = S.uniform_vector(A.n, 3)
    hi, lo = gmres_plans(A, precond, values)
    x, it, cy, rel = solve(hi, lo, b, s, m, 1, lmin, lmax, 0.0, 1, precond=precond)
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), s, m, precond, lmin, lmax, 0.0, 1,
                                          values=None if values == "f64" else np.float32)
    assert it == ito == m and cy == 1
    # the block's basis comes from one MPK whose columns are only as independent as the
    # Newton polynomials make them; Cholesky QR amplifies rounding by about kappa(W)^2,
    # and for blocks of up to 8 columns over these intervals kappa(W) stays below ~1e4,
    # so u kappa^2 ~ 1e-8 bounds the difference of two correct runs after one cycle
    assert np.linalg.norm(x - xo) <= BLOCK_BASIS_RTOL * np.linalg.norm(xo)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_blocked_basis_solve_to_1e10(precond):
    if precond == "none":
        dims = (37, 29)
        A = S.laplacian_2d(*dims)
        lmin, lmax = lap_bounds(dims)
    else:
        A, lmin, lmax = jacobi_knn(20000, 3)
    b = S.uniform_vector(A.n, 4)
    hi, lo = gmres_plans(A, precond)
    x, it, cy, rel = solve(hi, lo, b, 8, 64, 1, lmin, lmax, 1e-10, 80, precond=precond)
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), 8, 64, precond, lmin, lmax, 1e-10, 80)
    assert rel <= 1e-10 and abs(cy - (len(hist) - 1)) <= 1 and abs(it - ito) <= 64
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1.0000001e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 2e-10 * (lmax / lmin) * np.linalg.norm(xo)
    # blocked, plain and staged bases give the same solution bitwise
    xp, ip, cp, rp = solve(hi, lo, b, 8, 64, 1, lmin, lmax, 1e-10, 80, precond=precond, plain=True)
    xs, is_, cs, rs = solve(hi, lo, b, 8, 64, 1, lmin, lmax, 1e-10, 80, precond=precond, staged=True)
    assert np.array_equal(x, xp) and np.array_equal(x, xs) and it == ip == is_


def test_preconditioner_plan_forms_are_checked():
    A = S.laplacian_2d(9, 7)
    lmin, lmax = lap_bounds((9, 7))
    b = torch.tensor(S.uniform_vector(A.n, 2), device=DEV)
    hi = Plan.from_csr(A).upload(DEV)
    jac = Plan.from_csr(A, column_scaling="jacobi").upload(DEV)
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        hi.sstep_gmres(hi, b, 4, 8, 1, lmin / 4, lmax / 4, precond="jacobi")   # lo must hold A D^-1
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        hi.sstep_gmres(jac, b, 4, 8, 1, lmin, lmax, precond="none")           # lo must hold A
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        jac.sstep_gmres(jac, b, 4, 8, 1, lmin, lmax, precond="jacobi")        # hi must hold A
    # a nonpositive lmin is allowed without the Chebyshev preconditioner
    x, it, cy, rel = hi.sstep_gmres(hi, b, 4, 8, 1, -1.0, lmax, tol=1e-10, max_cycles=40, precond="none")
    assert rel <= 1e-10


# ------------------------------------------------------------ GS2 preconditioner (R21, R22)
def dominant_nonsym(n, seed):
    A = S.random_pattern(n, 6, seed, symmetric=False)
    rp, c, v = A.rowptr, A.col, A.val.copy()
    for i in range(n):
        seg = slice(rp[i], rp[i + 1])
        d = np.nonzero(c[seg] == i)[0]
        v[rp[i] + d[0]] = 1.0 + np.abs(v[seg]).sum()
    return S.CSR(n, rp, c, v)


@pytest.mark.parametrize("gamma", [0, 1, 2])
@pytest.mark.parametrize("values", ["f64", "f32"])
@pytest.mark.parametrize("s,m", [(1, 8), (4, 8), (8, 8)])
def test_gs2_fixed_cycle_matches_oracle(gamma, values, s, m):
    # diagonally dominant, so A P^{-1} has its spectrum near 1 and the blocks are well
    # conditioned; each block's basis is one GS2 chain of s powers
    A = dominant_nonsym(3000, 8)
    b = S.uniform_vector(A.n, 3)
    hi = Plan.from_csr(A, p_block=8).upload(DEV)
    lo = Plan.from_csr(A, p_block=8, values=values, split_lower=True).upload(DEV)
    x, it, cy, rel = solve(hi, lo, b, s, m, gamma, 0.3, 1.7, 0.0, 1, precond="gs2")
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), s, m, "gs2", 0.3, 1.7, 0.0, 1,
                                          values=None if values == "f64" else np.float32, gamma=gamma)
    assert it == ito == m and cy == 1
    assert np.linalg.norm(x - xo) <= BLOCK_BASIS_RTOL * np.linalg.norm(xo)


@pytest.mark.parametrize("gamma", [1, 2])
def test_gs2_gmres_solves_laplacian_like_oracle(gamma):
    dims = (37, 29)
    A = S.laplacian_2d(*dims)
    b = S.uniform_vector(A.n, 3)
    hi = Plan.from_csr(A, p_block=8).upload(DEV)
    lo = Plan.from_csr(A, p_block=8, split_lower=True).upload(DEV)
    x, it, cy, rel = solve(hi, lo, b, 8, 64, gamma, 0.002, 2.0, 1e-10, 40, precond="gs2")
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), 8, 64, "gs2", 0.002, 2.0, 1e-10, 40, gamma=gamma)
    lmin, lmax = lap_bounds(dims)
    assert rel <= 1e-10 and abs(cy - (len(hist) - 1)) <= 1
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1.0000001e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 2e-10 * (lmax / lmin) * np.linalg.norm(xo)
    xp, ip, cp, rp = solve(hi, lo, b, 8, 64, gamma, 0.002, 2.0, 1e-10, 40, precond="gs2", plain=True)
    xs, is_, cs, rs = solve(hi, lo, b, 8, 64, gamma, 0.002, 2.0, 1e-10, 40, precond="gs2", staged=True)
    assert np.array_equal(x, xp) and np.array_equal(x, xs) and it == ip == is_


def test_gs2_gmres_needs_a_split_plan():
    A = S.laplacian_2d(9, 7)
    b = torch.tensor(S.uniform_vector(A.n, 2), device=DEV)
    hi = Plan.from_csr(A).upload(DEV)
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        hi.sstep_gmres(hi, b, 4, 8, 1, 0.01, 2.0, precond="gs2")
    split = Plan.from_csr(A, split_lower=True).upload(DEV)
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        hi.sstep_gmres(split, b, 4, 8, 17, 0.01, 2.0, precond="gs2")  # gamma > 16


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("values", ["f64", "f32"])
@pytest.mark.parametrize("s,m", [(1, 8), (2, 8), (4, 16)])
def test_jacobi_k_sweeps_fixed_cycle_matches_oracle(k, values, s, m):
    # each block's basis is one Jacobi chain of s k sub-powers with the Newton shifts applied
    # as each link closes; shift 2 keeps the blocks well conditioned.  With k > 1 most of
    # A P^{-1}'s spectrum clusters near 1, and 8-column Newton blocks are then so nearly
    # dependent that two correct runs differ by ~1e-6 after one cycle (measured), so s = 8
    # is checked through the converged solve below
    A, lmin, lmax = jacobi_knn(6000, 2, shift=2.0)
    # A P^{-1} = I - (I - B)^k with B's spectrum in [lmin, 2 - lmin]: |1 - beta| <= 1 - lmin,
    # so it lies in [1 - (1 - lmin)^k, 1] for even k and [1 - (1 - lmin)^k, 1 + (1 - lmin)^k] for odd k
    lo_i = 1.0 - (1.0 - lmin) ** k
    hi_i = 1.0 if k % 2 == 0 else 1.0 + (1.0 - lmin) ** k
    b = S.uniform_vector(A.n, 3)
    hi, lo = gmres_plans(A, "jacobi", values)
    x, it, cy, rel = solve(hi, lo, b, s, m, k, lo_i, hi_i, 0.0, 1, precond="jacobi")
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), s, m, "jacobi", lo_i, hi_i, 0.0, 1,
                                          values=None if values == "f64" else np.float32, ksweeps=k)
    assert it == ito == m and cy == 1
    assert np.linalg.norm(x - xo) <= BLOCK_BASIS_RTOL * np.linalg.norm(xo)


def test_jacobi_k_sweeps_solve_and_executors():
    A, lmin, lmax = jacobi_knn(20000, 3)
    b = S.uniform_vector(A.n, 4)
    hi, lo = gmres_plans(A, "jacobi")
    x, it, cy, rel = solve(hi, lo, b, 8, 64, 2, 0.0, 1.0, 1e-10, 80, precond="jacobi")
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), 8, 64, "jacobi", 0.0, 1.0, 1e-10, 80, ksweeps=2)
    assert rel <= 1e-10 and abs(cy - (len(hist) - 1)) <= 1
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1.0000001e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 2e-10 * (lmax / lmin) * np.linalg.norm(xo)
    xp, ip, cp, rp = solve(hi, lo, b, 8, 64, 2, 0.0, 1.0, 1e-10, 80, precond="jacobi", plain=True)
    xs, is_, cs, rs = solve(hi, lo, b, 8, 64, 2, 0.0, 1.0, 1e-10, 80, precond="jacobi", staged=True)
    assert np.array_equal(x, xp) and np.array_equal(x, xs) and it == ip == is_


# ---- Newton shifts from Ritz values (reading R24): no spectrum interval given --------
def ritz_problem(precond):
    if precond == "none":
        return S.laplacian_2d(37, 29), 1
    if precond == "jacobi":
        return jacobi_knn(6000, 2, shift=2.0)[0], 1
    return dominant_nonsym(3000, 8), 1  # gs2 with gamma = 1


@pytest.mark.parametrize("precond", ["none", "jacobi", "gs2"])
@pytest.mark.parametrize("s,m", [(4, 16), (8, 32)])
def test_ritz_shift_fixed_cycle_matches_oracle(precond, s, m):
    # the GPU's Arnoldi (classical Gram-Schmidt twice) and the oracle's (modified
    # Gram-Schmidt) give Ritz values equal to rounding, so the shifts agree closely; the
    # GMRES iterate depends on the Krylov space only, so the bound of the interval case holds
    A, deg = ritz_problem(precond)
    b = S.uniform_vector(A.n, 3)
    if precond == "gs2":
        hi = Plan.from_csr(A, p_block=8).upload(DEV)
        lo = Plan.from_csr(A, p_block=8, split_lower=True).upload(DEV)
    else:
        hi, lo = gmres_plans(A, precond)
    x, it, cy, rel = solve(hi, lo, b, s, m, deg, None, None, 0.0, 1, precond=precond)
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), s, m, precond, None, None, 0.0, 1, gamma=deg)
    assert it == ito == m and cy == 1
    assert np.linalg.norm(x - xo) <= BLOCK_BASIS_RTOL * np.linalg.norm(xo)


@pytest.mark.parametrize("precond", ["none", "jacobi", "gs2"])
def test_ritz_shift_solve_to_1e10(precond):
    if precond == "jacobi":
        A = jacobi_knn(20000, 3)[0]
    else:
        A = S.laplacian_2d(37, 29)
    b = S.uniform_vector(A.n, 4)
    if precond == "gs2":
        hi = Plan.from_csr(A, p_block=8).upload(DEV)
        lo = Plan.from_csr(A, p_block=8, split_lower=True).upload(DEV)
    else:
        hi, lo = gmres_plans(A, precond)
    x, it, cy, rel = solve(hi, lo, b, 8, 64, 1, None, None, 1e-10, 80, precond=precond)
    xo, hist, ito = O.sstep_gmres_precond(A, b, np.zeros(A.n), 8, 64, precond, None, None, 1e-10, 80, gamma=1)
    n, rp, c, v = A
    ref = spla.spsolve(csr_matrix((v, c, rp), shape=(n, n)).tocsc(), b)
    assert rel <= 1e-10 and hist[-1] <= 1e-10
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1.0000001e-10 * np.linalg.norm(b)
    # both solutions are within kappa * tol of the direct one (kappa below 4e3 here)
    assert np.linalg.norm(x - ref) <= 1e-10 * 4000 * np.linalg.norm(ref)
    assert np.linalg.norm(x - xo) <= 2e-10 * 4000 * np.linalg.norm(xo)
    xp, ip, cp, rp_ = solve(hi, lo, b, 8, 64, 1, None, None, 1e-10, 80, precond=precond, plain=True)
    assert np.array_equal(x, xp) and it == ip


def test_ritz_shifts_are_refused_with_the_chebyshev_preconditioner():
    A = S.laplacian_2d(12)
    hi = Plan.from_csr(A, p_block=4).upload(DEV)
    b = torch.ones(A.n, dtype=torch.float64, device=DEV)
    with pytest.raises(MPKError, match="RITZ"):
        hi.sstep_gmres(hi, b, 4, 8, 4, None, None)
