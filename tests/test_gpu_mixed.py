"""GPU parity of reduced-precision matrix-value storage through the C ABI:
FP32 values (reading R11) and BF16 values with a per-row FP32 scale (R16).

The device keeps each matrix value rounded once while vectors, products and
sums stay FP64, so the result must match the oracle's FP64 MPK of the rounded
matrix within the FP64 tolerance, and blocked and plain kernels must agree
bitwise.  Each test also states the error against the FP64 oracle of the
unrounded matrix and checks it against the perturbation bound
((1 + u)^k - 1) |A|^k |x| (relative L2), u = 2^-24 for FP32 and 2^-8 + 2^-22
for BF16, since every reduced-precision result must state that error."""
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
U = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8 + 2.0 ** -22}
ROUND = {"f32": O.round_values, "bf16": O.round_values_bf16_rowscale}
VALUES = ["f32", "bf16"]


def rel_err(got, ref):
    num = np.linalg.norm(got - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


def apply_orig(plan, perm, x, p, plain=False):
    Yp = plan.apply(torch.tensor(x[perm], device=DEV), p, plain=plain).cpu().numpy()
    plan.check()
    Y = np.empty_like(Yp)
    Y[:, perm] = Yp
    return Y


def f32_plan(A, values="f32", **kw):
    plan = Plan.from_csr(A, values=values, **kw).upload(DEV)
    return plan, plan.levels()["perm"].astype(np.int64)


def fp64_error_bound(A, x, p, values="f32"):
    """Relative L2 bound per power from |A~ - A| <= u |A|, plus the FP64 tolerance."""
    absA = A._replace(val=np.abs(A.val))
    ab = O.mpk(absA, np.abs(x), p)
    ref = O.mpk(A, x, p)
    k = np.arange(1, p + 1)
    return ((1 + U[values]) ** k - 1) * np.linalg.norm(ab, axis=-1) / np.linalg.norm(ref, axis=-1) + TOL


CASES = {
    "knn_20k": lambda: S.knn_graph_laplacian(20000, k=26, seed=0),
    "rand_nonsym": lambda: S.random_pattern(5000, 4, 1),
    "lap3d_ragged": lambda: S.laplacian_3d(19, 23, 17),
    "wide_rows": lambda: S.random_pattern(3000, 40, 5),
}


@pytest.mark.parametrize("values", VALUES)
@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("p", [1, 4, 9])
def test_f32_values_match_rounded_oracle(name, p, values):
    A = CASES[name]()
    plan, perm = f32_plan(A, values, p_block=4)
    x = S.uniform_vector(A.n, 2)
    got = apply_orig(plan, perm, x, p)
    assert np.all(rel_err(got, O.mpk(ROUND[values](A), x, p)) <= TOL)
    assert np.array_equal(apply_orig(plan, perm, x, p, plain=True), got)
    err64 = rel_err(got, O.mpk(A, x, p))  # the stated error against the FP64 oracle
    assert np.all(err64 <= fp64_error_bound(A, x, p, values)), err64


def test_f32_values_integer_matrix_equals_fp64_bitwise():
    # integer-valued stencils are exact in FP32: storage changes nothing
    A = S.laplacian_3d(21, 17, 13)
    plan, perm = f32_plan(A, p_block=8)
    xi = S.integer_vector(A.n, 3)
    assert np.array_equal(apply_orig(plan, perm, xi, 8), O.mpk(A, xi, 8))
    x = S.uniform_vector(A.n, 4)
    p64 = Plan.from_csr(A, p_block=8).upload(DEV)
    assert np.array_equal(apply_orig(plan, perm, x, 8), apply_orig(p64, perm, x, 8))


@pytest.mark.parametrize("values", VALUES)
@pytest.mark.parametrize("G", [1, 2, 4])
@pytest.mark.parametrize("mk", [lambda: S.knn_graph_laplacian(9000, k=26, seed=6),  # wide rows: G = 1
                                lambda: S.laplacian_3d(23, 19, 21)])                # narrow rows
def test_f32_values_chunks_per_worker(G, mk, values):
    A = mk()
    plan, perm = f32_plan(A, values, p_block=5, chunks_per_worker=G)
    x = S.uniform_vector(A.n, 6)
    got = apply_orig(plan, perm, x, 12)
    assert np.all(rel_err(got, O.mpk(ROUND[values](A), x, 12)) <= TOL)
    assert np.array_equal(apply_orig(plan, perm, x, 12, plain=True), got)


@pytest.mark.parametrize("values", VALUES)
@pytest.mark.parametrize("kind", ["newton", "chebyshev"])
def test_f32_values_poly_and_sstep(kind, values):
    A = S.knn_graph_laplacian(12000, k=26, seed=3)
    Ar = ROUND[values](A)
    plan, perm = f32_plan(A, values, p_block=4)
    x = S.uniform_vector(A.n, 5)
    rng = np.random.default_rng(7)
    c = rng.uniform(-1, 1, 9) / 60.0 ** np.arange(9)
    if kind == "newton":
        params = rng.uniform(0.1, 60, 8)
        ref = O.poly_newton(Ar, x, c, params)
    else:
        params = np.array([30.0, 30.0])
        c = rng.uniform(-1, 1, 9)
        ref = O.poly_chebyshev(Ar, x, c, 30.0, 30.0)
    out = plan.poly(kind, c, torch.tensor(x[perm], device=DEV), params=params).cpu().numpy()
    plan.check()
    got = np.empty_like(out)
    got[perm] = out
    assert rel_err(got, ref) <= TOL
    lam = rng.uniform(0.1, 50, 6)
    Vp = plan.sstep(torch.tensor(x[perm], device=DEV), lam).cpu().numpy()
    plan.check()
    V = np.empty_like(Vp)
    V[:, perm] = Vp
    assert np.all(rel_err(V, O.newton_basis(Ar, x, lam)) <= TOL)


@pytest.mark.slow
def test_f32_values_full_size_160_cubed():
    # the benchmarked stencil has integer values: FP32 storage must reproduce FP64 exactly
    A = S.laplacian_3d(160)
    plan, perm = f32_plan(A, p_block=4)
    x = S.uniform_vector(A.n, 0)
    got = apply_orig(plan, perm, x, 4)
    assert np.all(rel_err(got, O.mpk(A, x, 4)) <= TOL)
    assert np.array_equal(apply_orig(plan, perm, x, 4, plain=True), got)


@pytest.mark.slow
def test_bf16_values_full_size_160_cubed():
    # the stencil's -1/6 is not a BF16 value: the result differs from FP64, within the bound
    A = S.laplacian_3d(160)
    plan, perm = f32_plan(A, "bf16", p_block=4)
    x = S.uniform_vector(A.n, 0)
    got = apply_orig(plan, perm, x, 4)
    assert np.all(rel_err(got, O.mpk(O.round_values_bf16_rowscale(A), x, 4)) <= TOL)
    assert np.array_equal(apply_orig(plan, perm, x, 4, plain=True), got)
    err64 = rel_err(got, O.mpk(A, x, 4))
    assert np.all(err64 <= fp64_error_bound(A, x, 4, "bf16")) and err64.max() > 0, err64
