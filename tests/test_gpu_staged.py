"""GPU parity of the level-group wavefront executor (readings R14, R15) through
the C ABI: one launch per stage of the schedule that mpk_get_schedule returns.
Its row arithmetic is the SpMV kernel's, so every result must equal the plain
path bitwise, whatever the cache size (one group, or one level per group)."""
import numpy as np
import pytest

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU-only hosts, never run there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_02228_amd import Plan  # noqa: E402

DEV = "cuda:0"
TOL = 1e-12

CASES = {
    "lap3d": lambda: S.laplacian_3d(22, 19, 17),
    "knn": lambda: S.knn_graph_laplacian(15000, k=26, seed=2),
    "rand_nonsym": lambda: S.random_pattern(6000, 4, 7),
    "blocks": lambda: S.block_diagonal(S.laplacian_2d(30, 20), S.identity(100), S.laplacian_1d(700)),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("cache_mib,pb", [(1, 4), (1, 3), (256, 4), (1, 15)])
def test_staged_mpk_equals_plain(name, cache_mib, pb):
    A = CASES[name]()
    plan = Plan.from_csr(A, p_block=pb, cache_mib=cache_mib).upload(DEV)
    ng, tasks = plan.schedule(min(pb, 15))
    perm = plan.levels()["perm"].astype(np.int64)
    x = S.uniform_vector(A.n, 3)
    xd = torch.tensor(x[perm], device=DEV)
    p = 2 * pb + 1
    st = plan.apply(xd, p, staged=True).cpu().numpy()
    pl = plan.apply(xd, p, plain=True).cpu().numpy()
    plan.check()
    assert np.array_equal(st, pl), (ng, len(tasks))
    Y = np.empty_like(st)
    Y[:, perm] = st
    ref = O.mpk(A, x, p)
    assert np.all(np.linalg.norm(Y - ref, axis=1) <= TOL * np.linalg.norm(ref, axis=1))


@pytest.mark.parametrize("kind", ["monomial", "newton", "chebyshev"])
def test_staged_poly_sstep_and_solve_equal_plain(kind):
    A = S.knn_graph_laplacian(12000, k=26, seed=4)
    plan = Plan.from_csr(A, p_block=4, cache_mib=1).upload(DEV)
    perm = plan.levels()["perm"].astype(np.int64)
    x = torch.tensor(S.uniform_vector(A.n, 5)[perm], device=DEV)
    rng = np.random.default_rng(3)
    c = rng.uniform(-1, 1, 10) / 60.0 ** np.arange(10)
    params = {"monomial": None, "newton": rng.uniform(0.1, 60, 9), "chebyshev": np.array([30.0, 30.0])}[kind]
    a = plan.poly(kind, c, x, params=params, staged=True).cpu().numpy()
    b = plan.poly(kind, c, x, params=params, plain=True).cpu().numpy()
    assert np.array_equal(a, b)
    lam = rng.uniform(0.1, 50, 7)
    assert np.array_equal(plan.sstep(x, lam, staged=True).cpu().numpy(), plan.sstep(x, lam, plain=True).cpu().numpy())
    if kind == "chebyshev":
        lmax = 2.0 * np.max(np.diff(A.rowptr)) + 0.1
        xs, ks, rs = plan.refine_solve(plan, x, 12, 0.1, lmax, tol=1e-10, max_iter=300, staged=True)
        xp, kp, rp = plan.refine_solve(plan, x, 12, 0.1, lmax, tol=1e-10, max_iter=300, plain=True)
        assert ks == kp and rs == rp <= 1e-10 and torch.equal(xs, xp)
    plan.check()
