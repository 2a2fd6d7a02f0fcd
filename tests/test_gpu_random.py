"""Seeded randomised parity sweep through the C ABI: random sizes (ragged
last chunks, matrices smaller than one chunk), densities (empty rows,
disconnected components), nonsymmetric patterns, block sizes, chunks per
wave, value storage and all three executors (blocked, staged, plain).  Every
case must match the oracle within the FP64 tolerance (against the rounded
matrix for reduced storage) and the three executors must agree bitwise."""
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
ROUND = {"f64": lambda A: A, "f32": O.round_values, "bf16": O.round_values_bf16_rowscale}


def case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.choice([1, 5, 63, 64, 65, 200, 1000, 4097, 9000]))
    kind = rng.integers(3)
    if kind == 0:
        A = S.random_pattern(n, float(rng.uniform(0.3, 8)), seed, symmetric=bool(rng.integers(2)),
                             diag=bool(rng.integers(2)))  # without the diagonal some rows are empty
    elif kind == 1:
        m = max(1, int(round(n ** 0.5)))
        A = S.laplacian_2d(m, max(1, n // m))
    else:
        parts = [S.random_pattern(max(1, n // 3), 2.5, seed + 7), S.identity(max(1, n // 5)),
                 S.laplacian_1d(max(2, n // 4))]
        A = S.block_diagonal(*parts)
    pb = int(rng.choice([1, 2, 3, 4, 7, 15]))
    G = int(rng.choice([0, 1, 2, 4]))
    values = str(rng.choice(["f64", "f64", "f32", "bf16"]))
    p = int(rng.integers(1, 13))
    return A, pb, G, values, p


@pytest.mark.parametrize("seed", range(40))
def test_random_case(seed):
    A, pb, G, values, p = case(seed)
    plan = Plan.from_csr(A, p_block=pb, chunks_per_worker=G, values=values, cache_mib=1).upload(DEV)
    perm = plan.levels()["perm"].astype(np.int64)
    x = S.uniform_vector(A.n, seed)
    xd = torch.tensor(x[perm], device=DEV)
    blocked = plan.apply(xd, p).cpu().numpy()
    staged = plan.apply(xd, p, staged=True).cpu().numpy()
    plain = plan.apply(xd, p, plain=True).cpu().numpy()
    plan.check()
    assert np.array_equal(blocked, plain) and np.array_equal(staged, plain), (A.n, pb, G, values, p)
    Y = np.empty_like(blocked)
    Y[:, perm] = blocked
    ref = O.mpk(ROUND[values](A), x, p)
    num = np.linalg.norm(Y - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    assert np.all(num <= TOL * np.where(den > 0, den, 1.0)), (A.n, pb, G, values, p, num / np.maximum(den, 1e-300))


def test_empty_matrix_calls_succeed():
    A = S.from_dense(np.zeros((0, 0)))
    plan = Plan.from_csr(A).upload(DEV)
    x = torch.empty(0, dtype=torch.float64, device=DEV)
    assert plan.apply(x, 3).shape == (3, 0)
    assert plan.poly("chebyshev", np.ones(4), x, params=np.array([1.0, 1.0])).shape == (0,)
    plan.check()
