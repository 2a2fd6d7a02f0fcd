"""GPU parity of the AMG pre-smoother fused with the residual (Sec. 5.3 with the GS2
smoother of Sec. 5.1; reading R23) through the C ABI.

`sweeps` outer GS2 sweeps (gamma + 1 sub-powers each) and the residual run as one chain
of sub-powers.  The oracle computes each sweep and the residual with separate row loops;
the GPU sums rows in level order with FMAs, so the two differ in rounding only.  Bounds:
the smoothed x within 1e-12 relative L2 (each sweep contracts earlier differences), and
the residual within 1e-12 (|b| + |A| |x|) in L2, the scale of the rounding of b - A x
itself.  Blocked, plain and staged executors and both I/O orders share the row arithmetic
and agree bitwise."""
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
TOL = 1e-12


def nonsym_dominant(n, seed):
    A = S.random_pattern(n, 6, seed, symmetric=False)
    rp, c, v = A.rowptr, A.col, A.val.copy()
    for i in range(n):
        seg = slice(rp[i], rp[i + 1])
        d = np.nonzero(c[seg] == i)[0]
        v[rp[i] + d[0]] = 1.0 + np.abs(v[seg]).sum()
    return S.CSR(n, rp, c, v)


MATS = {"lap3d": lambda: S.laplacian_3d(23, 19, 17), "knn12": lambda: S.knn_graph_laplacian(5000, k=12, seed=4),
        "nonsym": lambda: nonsym_dominant(5000, 8)}


def make_plan(A, q=4, values="f64"):
    return Plan.from_csr(A, split_lower=True, p_block=q, values=values).upload(DEV)


def run(plan, b, x0, sweeps, gamma, permuted=True, **kw):
    perm = plan.levels()["perm"].astype(np.int64)
    bd = torch.tensor(b[perm] if permuted else b, device=DEV)
    xd = torch.tensor(x0[perm] if permuted else x0, device=DEV)
    xd, rd = plan.gs2_smooth(bd, xd, sweeps, gamma, permuted=permuted, **kw)
    plan.check()
    x, r = xd.cpu().numpy(), rd.cpu().numpy()
    if permuted:
        xo, ro = np.empty_like(x), np.empty_like(r)
        xo[perm], ro[perm] = x, r
        x, r = xo, ro
    return x, r


def abs_scale(A, b, x):
    # |b| + |A| |x|: the size of the terms whose difference is the residual
    n, rp, c, v = A
    rows = np.repeat(np.arange(n), np.diff(rp))
    return np.abs(b) + np.bincount(rows, weights=np.abs(v) * np.abs(x[c]), minlength=n)


def check(A, b, x, r, xr, rr):
    assert np.linalg.norm(x - xr) <= TOL * np.linalg.norm(xr)
    assert np.linalg.norm(r - rr) <= TOL * np.linalg.norm(abs_scale(A, b, xr))


@pytest.mark.parametrize("sweeps", [1, 3])
@pytest.mark.parametrize("gamma", [0, 1, 2])
@pytest.mark.parametrize("mk", list(MATS))
def test_smoother_and_residual_match_oracle(mk, gamma, sweeps):
    A = MATS[mk]()
    b = S.uniform_vector(A.n, 2)
    x0 = S.uniform_vector(A.n, 3)
    plan = make_plan(A)
    x, r = run(plan, b, x0, sweeps, gamma)
    xr, rr = O.gs2_smooth_residual(A, b, x0, sweeps, gamma)
    check(A, b, x, r, xr, rr)


def test_blocking_engages_on_the_stencil():
    plan = make_plan(S.laplacian_3d(40), q=8)
    assert plan.block_powers("gs2_smooth") >= 2


@pytest.mark.parametrize("gamma,sweeps,q", [(1, 3, 4), (0, 5, 3), (2, 2, 8), (3, 3, 15), (1, 1, 2)])
def test_blocked_plain_staged_and_io_orders_bitwise(gamma, sweeps, q):
    # chains of 4 to 13 sub-powers straddle launches of 2 to 15 sub-powers
    A = S.laplacian_2d(61, 47)
    b = S.uniform_vector(A.n, 6)
    x0 = S.uniform_vector(A.n, 7)
    plan = make_plan(A, q=q)
    xb, rb = run(plan, b, x0, sweeps, gamma)
    xp, rp = run(plan, b, x0, sweeps, gamma, plain=True)
    xs, rs = run(plan, b, x0, sweeps, gamma, staged=True)
    xo, ro = run(plan, b, x0, sweeps, gamma, permuted=False)
    for x, r in ((xp, rp), (xs, rs), (xo, ro)):
        assert np.array_equal(xb, x) and np.array_equal(rb, r)
    xr, rr = O.gs2_smooth_residual(A, b, x0, sweeps, gamma)
    check(A, b, xb, rb, xr, rr)


def test_zero_sweeps_is_the_residual_and_leaves_x():
    A = MATS["nonsym"]()
    b = S.uniform_vector(A.n, 4)
    x0 = S.uniform_vector(A.n, 5)
    plan = make_plan(A)
    x, r = run(plan, b, x0, 0, 2)
    assert np.array_equal(x, x0)
    _, rr = O.gs2_smooth_residual(A, b, x0, 0, 2)
    assert np.linalg.norm(r - rr) <= TOL * np.linalg.norm(abs_scale(A, b, x0))


def test_from_zero_one_sweep_is_the_gs2_preconditioner():
    # x0 = 0, one sweep: x = P^{-1} b, the vector mpk_gs2_apply's preconditioner forms
    A = MATS["knn12"]()
    b = S.uniform_vector(A.n, 8)
    plan = make_plan(A)
    x, r = run(plan, b, np.zeros(A.n), 1, 2)
    np.testing.assert_allclose(x, O.gs2_precondition(A, b, 2), rtol=0, atol=TOL * np.abs(x).max() * 10)


def test_many_sweeps_reduce_the_residual():
    # the strongly dominant matrix converges to rounding in 40 sweeps (oracle: 4e-16 of the
    # first sweep's residual); the graph Laplacian's smooth modes only to about 4e-2
    A = MATS["nonsym"]()
    b = S.uniform_vector(A.n, 9)
    plan = make_plan(A, q=8)
    _, r1 = run(plan, b, np.zeros(A.n), 1, 1)
    x, r = run(plan, b, np.zeros(A.n), 40, 1)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(r1)
    xr, rr = O.gs2_smooth_residual(A, b, np.zeros(A.n), 40, 1)
    check(A, b, x, r, xr, rr)


@pytest.mark.parametrize("values", ["f32", "bf16"])
def test_reduced_precision_values_match_the_oracle_of_the_stored_matrix(values):
    A = MATS["lap3d"]()
    Ar = O.round_values(A) if values == "f32" else O.round_values_bf16_rowscale(A)
    b = S.uniform_vector(A.n, 10)
    x0 = S.uniform_vector(A.n, 11)
    plan = make_plan(A, values=values)
    x, r = run(plan, b, x0, 2, 1)
    xr, rr = O.gs2_smooth_residual(Ar, b, x0, 2, 1)
    check(Ar, b, x, r, xr, rr)


def test_repeated_calls_are_identical():
    A = S.laplacian_3d(30)
    b = S.uniform_vector(A.n, 12)
    x0 = S.uniform_vector(A.n, 13)
    plan = make_plan(A, q=6)
    first = run(plan, b, x0, 3, 1)
    for _ in range(3):
        again = run(plan, b, x0, 3, 1)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])


def test_errors():
    A = S.laplacian_2d(20)
    plan = Plan.from_csr(A, p_block=4).upload(DEV)
    b = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    with pytest.raises(MPKError, match="split_lower"):
        plan.gs2_smooth(b, b.clone(), 1, 1)
    split = make_plan(A)
    with pytest.raises(MPKError, match="gamma"):
        split.gs2_smooth(b, b.clone(), 1, 17)
    with pytest.raises(MPKError, match="sweeps"):
        split.gs2_smooth(b, b.clone(), -1, 1)
