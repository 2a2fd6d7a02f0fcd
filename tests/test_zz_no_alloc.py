"""poly_apply_static (the entry point for callers that cannot allocate device memory)
against poly_apply, through the C ABI: two calls in a row, the second on a smaller
input, both equal to poly_apply's result (same kernels: bitwise) and within 1e-12
of the FP64 oracle; requests larger than the static scratch are refused."""
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


def rel_err(got, ref):
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


def check(A, kind, c, params, permuted, seed):
    plan = Plan.from_csr(A, p_block=4).upload(DEV)
    assert plan.block_powers({"monomial": "poly_monomial", "newton": "poly_newton",
                              "chebyshev": "poly_chebyshev"}[kind]) >= 2
    perm = plan.levels()["perm"].astype(np.int64)
    x = S.uniform_vector(A.n, seed)
    xd = torch.tensor(x[perm] if permuted else x, device=DEV)
    ref_gpu = plan.poly(kind, c, xd, params=params, permuted=permuted).cpu().numpy()
    got = plan.poly_static(kind, c, xd, params=params, permuted=permuted).cpu().numpy()
    plan.check()
    assert np.array_equal(got, ref_gpu)
    if permuted:
        back = np.empty_like(got)
        back[perm] = got
        got = back
    if kind == "monomial":
        ref = O.poly_monomial(A, x, c)
    elif kind == "newton":
        ref = O.poly_newton(A, x, c, params)
    else:
        ref = O.poly_chebyshev(A, x, c, params[0], params[1])
    assert rel_err(got, ref) <= TOL


def test_static_scratch_two_calls_second_smaller():
    rng = np.random.default_rng(3)
    # first call: 40^3 Laplacian (64,000 rows), degree-8 Chebyshev on its spectrum
    check(S.laplacian_3d(40), "chebyshev", rng.uniform(-1, 1, 9), [6.0, 6.0], True, 1)
    # second call, smaller: 50x50 Laplacian (2,500 rows), degree-5 Newton, original order
    check(S.laplacian_2d(50), "newton", rng.uniform(-1, 1, 6), [1.0, 2.0, 3.0, 4.0, 5.0], False, 2)


def test_static_scratch_refuses_oversize_requests():
    # 8 n (p_block + 2) bytes above 64 MiB: n = 1.5 M rows with a ring of 6 vectors
    A = S.laplacian_3d(115)
    assert A.n * 8 * 6 > 64 << 20
    plan = Plan.from_csr(A, p_block=4)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    with pytest.raises(MPKError) as e:
        plan.poly_static("monomial", [1.0, 2.0], x)
    assert e.value.code == -1 and "static scratch" in str(e.value)
