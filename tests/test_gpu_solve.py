"""GPU parity of the mixed-precision refinement solve (readings R12, R13)
through the C ABI.

The GPU iterates follow the oracle's map x <- x + s(A~) (b - A x), so after a
fixed number of steps they agree to FP64 round-off; run to 1e-10 they stop
within one step of the oracle.  With FP64 values on both plans the blocked and
plain corrections use the same row arithmetic, so the solutions are bitwise
equal."""
import numpy as np
import pytest

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU-only hosts, never run there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_02228_amd import Plan, MPKError  # noqa: E402

DEV = "cuda:0"


def knn_problem(n, seed):
    A = S.knn_graph_laplacian(n, k=26, seed=seed)
    lmax = 2.0 * np.max(np.diff(A.rowptr)) + 0.1  # Gershgorin; lmin = 0.1 is the shift
    return A, 0.1, lmax, S.uniform_vector(A.n, seed + 1)


def plans(A):
    hi = Plan.from_csr(A).upload(DEV)
    lo = Plan.from_csr(A, values="f32").upload(DEV)
    return hi, lo, hi.levels()["perm"].astype(np.int64)


def solve_orig(hi, lo, perm, b, d, lmin, lmax, tol, it, plain=False):
    x, k, rel = hi.refine_solve(lo, torch.tensor(b[perm], device=DEV), d, lmin, lmax, tol=tol, max_iter=it,
                                plain=plain)
    hi.check()
    lo.check()
    out = np.empty(b.size)
    out[perm] = x.cpu().numpy()
    return out, k, rel


@pytest.mark.parametrize("d", [1, 4, 16])
def test_fixed_steps_match_oracle(d):
    A, lmin, lmax, b = knn_problem(20000, 0)
    hi, lo, perm = plans(A)
    x, k, rel = solve_orig(hi, lo, perm, b, d, lmin, lmax, 0.0, 3)
    xo, hist = O.refine_solve(A, b, np.zeros(A.n), d, lmin, lmax, 0.0, 3)
    assert k == 3 and len(hist) == 4
    assert np.linalg.norm(x - xo) <= 1e-11 * np.linalg.norm(xo)
    assert abs(rel - hist[-1]) <= 1e-9 * hist[-1]


def test_solve_to_1e10_like_oracle():
    A, lmin, lmax, b = knn_problem(20000, 3)
    hi, lo, perm = plans(A)
    x, k, rel = solve_orig(hi, lo, perm, b, 16, lmin, lmax, 1e-10, 500)
    xo, hist = O.refine_solve(A, b, np.zeros(A.n), 16, lmin, lmax, 1e-10, 500)
    assert rel <= 1e-10 and abs(k - (len(hist) - 1)) <= 1
    # the true residual, in FP64 on the host
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1.0000001e-10 * np.linalg.norm(b)
    # both sit within kappa * 2 tol of the exact solution
    assert np.linalg.norm(x - xo) <= 2e-10 * (lmax / lmin) * np.linalg.norm(xo)


def test_fp64_blocked_and_plain_bitwise_and_io_orders():
    A = S.laplacian_3d(20, 18, 16)
    lmin = sum(2 - 2 * np.cos(np.pi / (m + 1)) for m in (20, 18, 16))
    lmax = sum(2 + 2 * np.cos(np.pi / (m + 1)) for m in (20, 18, 16))
    b = S.uniform_vector(A.n, 5)
    hi = Plan.from_csr(A).upload(DEV)
    perm = hi.levels()["perm"].astype(np.int64)
    xb, kb, rb = solve_orig(hi, hi, perm, b, 24, lmin, lmax, 1e-10, 400)
    xp, kp, rp = solve_orig(hi, hi, perm, b, 24, lmin, lmax, 1e-10, 400, plain=True)
    assert rb <= 1e-10 and kb == kp and rb == rp and np.array_equal(xb, xp)
    xo, _, _ = hi.refine_solve(hi, torch.tensor(b, device=DEV), 24, lmin, lmax, tol=1e-10, max_iter=400,
                               permuted=False)
    assert np.array_equal(xo.cpu().numpy(), xb)
    x2, k2, r2 = solve_orig(hi, hi, perm, b, 24, lmin, lmax, 1e-10, 400)  # repeatable
    assert k2 == kb and r2 == rb and np.array_equal(x2, xb)


def test_initial_guess_and_argument_errors():
    A, lmin, lmax, b = knn_problem(5000, 6)
    hi, lo, perm = plans(A)
    xs, k, rel = solve_orig(hi, lo, perm, b, 8, lmin, lmax, 1e-10, 800)
    x0 = torch.tensor(xs[perm], device=DEV)
    _, k0, rel0 = hi.refine_solve(lo, torch.tensor(b[perm], device=DEV), 8, lmin, lmax, tol=1e-10, x=x0)
    assert k0 == 0 and rel0 <= 1e-10  # already converged: no correction
    with pytest.raises(MPKError):
        lo.refine_solve(hi, torch.tensor(b[perm], device=DEV), 8, lmin, lmax)  # hi must be FP64
    other = Plan.from_csr(S.knn_graph_laplacian(5000, k=26, seed=7)).upload(DEV)
    with pytest.raises(MPKError):
        hi.refine_solve(other, torch.tensor(b[perm], device=DEV), 8, lmin, lmax)  # different matrix
    with pytest.raises(MPKError):
        hi.refine_solve(lo, torch.tensor(b[perm], device=DEV), 8, lmax, lmin)  # lmin >= lmax


def test_bf16_corrections_still_reach_1e10():
    # corrections from BF16 values (u ~ 2^-8) still contract: the FP64 residual decides
    A, lmin, lmax, b = knn_problem(20000, 8)
    hi = Plan.from_csr(A).upload(DEV)
    lo = Plan.from_csr(A, values="bf16").upload(DEV)
    perm = hi.levels()["perm"].astype(np.int64)
    x, k, rel = solve_orig(hi, lo, perm, b, 16, lmin, lmax, 1e-10, 800)
    assert rel <= 1e-10 and 0 < k < 800
    assert np.linalg.norm(b - O.spmv(A, x)) <= 1.0000001e-10 * np.linalg.norm(b)
