"""GPU parity of the Jacobi-preconditioned MPK (Sec. 5.1; reading R20) through the C ABI.

The plan stores B = A D^{-1} (each value divided by its column's diagonal entry in FP64,
rounded once); k = 1 is the MPK of B, k > 1 applies A P^{-1} = I - (I - B)^k as a Newton
polynomial.  The oracle runs the paper's Jacobi iteration literally, so the two differ in
rounding only: B's entries carry one rounding each, and (I - B)^k has norm at most 1 on
these matrices, so the error per power stays within a few units of k * eps relative;
the tolerance is the 1e-12 relative L2 per power used for every FP64 power here."""
import math

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


def run(A, x, p, k, permuted=True, **kw):
    plan = Plan.from_csr(A, column_scaling="jacobi", **{q: v for q, v in kw.items() if q in ("p_block", "values")})
    plan.upload(DEV)
    perm = plan.levels()["perm"].astype(np.int64)
    xin = x[perm] if permuted else x
    W = plan.jacobi_apply(torch.tensor(xin, device=DEV), p, k, permuted=permuted,
                          **{q: v for q, v in kw.items() if q in ("plain", "staged")})
    plan.check()
    W = W.cpu().numpy()
    if permuted:
        out = np.empty_like(W)
        out[:, perm] = W
        W = out
    return W


def rel_err(W, R):
    return max(np.linalg.norm(W[j] - R[j]) / np.linalg.norm(R[j]) for j in range(R.shape[0]))


def nonsym_dominant(n, seed):
    A = S.random_pattern(n, 6, seed, symmetric=False)
    rp, c, v = A.rowptr, A.col, A.val.copy()
    for i in range(n):  # make every diagonal entry dominant
        seg = slice(rp[i], rp[i + 1])
        d = np.nonzero(c[seg] == i)[0]
        v[rp[i] + d[0]] = 1.0 + np.abs(v[seg]).sum()
    return S.CSR(n, rp, c, v)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
@pytest.mark.parametrize("mk", ["lap3d", "knn", "nonsym"])
def test_jacobi_mpk_matches_oracle(mk, k):
    A = {"lap3d": lambda: S.laplacian_3d(23, 19, 17), "knn": lambda: S.knn_graph_laplacian(6000, seed=4),
         "nonsym": lambda: nonsym_dominant(5000, 8)}[mk]()
    x = S.uniform_vector(A.n, 2)
    p = 6
    W = run(A, x, p, k, p_block=4)
    R = O.jacobi_mpk(A, x, p, k)
    assert rel_err(W, R) <= TOL


@pytest.mark.parametrize("k,q", [(1, 4), (3, 4), (2, 3), (5, 4), (4, 8), (2, 15)])
def test_blocked_plain_staged_and_io_orders_bitwise(k, q):
    # in level order the k p sub-powers run as one chain blocked across links (links
    # straddle launches when q is not a multiple of k); original-order I/O applies one
    # Newton polynomial per power: the same arithmetic, so all four agree bitwise
    A = S.laplacian_2d(61, 47)
    x = S.uniform_vector(A.n, 6)
    Wb = run(A, x, 5, k, p_block=q)
    Wp = run(A, x, 5, k, p_block=q, plain=True)
    Ws = run(A, x, 5, k, p_block=q, staged=True)
    Wo = run(A, x, 5, k, p_block=q, permuted=False)
    assert np.array_equal(Wb, Wp) and np.array_equal(Wb, Ws) and np.array_equal(Wb, Wo)


def test_closed_form_on_laplacian_eigenvector():
    # D = 6 I for the 3D stencil: A P^{-1} v = (1 - (1 - lam/6)^k) v
    nx, ny, nz = 20, 16, 12
    A = S.laplacian_3d(nx, ny, nz)
    a, b, c = 17, 3, 9
    ix, iy, iz = np.meshgrid(np.arange(1, nx + 1), np.arange(1, ny + 1), np.arange(1, nz + 1), indexing="ij")
    v = (np.sin(a * np.pi * ix / (nx + 1)) * np.sin(b * np.pi * iy / (ny + 1)) *
         np.sin(c * np.pi * iz / (nz + 1))).transpose(2, 1, 0).ravel()  # natural order i + nx (j + ny k)
    lam = (2 - 2 * math.cos(a * math.pi / (nx + 1))) + (2 - 2 * math.cos(b * math.pi / (ny + 1))) + \
          (2 - 2 * math.cos(c * math.pi / (nz + 1)))
    for k in (1, 2, 4):
        mu = 1 - (1 - lam / 6) ** k
        W = run(A, v, 3, k)
        for j in range(3):
            np.testing.assert_allclose(W[j], mu ** (j + 1) * v, atol=1e-12)


def test_fp32_scaled_values_state_their_error():
    # FP32 storage of B = A D^{-1}: the kNN Laplacian's scaled values are not exact in
    # FP32; the error against the FP64 oracle is bounded by the rounding of B
    A = S.knn_graph_laplacian(6000, seed=5)
    x = S.uniform_vector(A.n, 3)
    W = run(A, x, 4, 2, values="f32")
    R = O.jacobi_mpk(A, x, 4, 2)
    err = rel_err(W, R)
    assert 0 < err <= 4 * 2 * 4 * 2.0 ** -24  # p * k * (|B| + 1) * u32, with |I - B| <= 1


def test_errors():
    A = S.laplacian_2d(9)
    plain = Plan.from_csr(A).upload(DEV)
    x = torch.tensor(S.uniform_vector(A.n, 1), device=DEV)
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        plain.jacobi_apply(x, 2, 1)
    jac = Plan.from_csr(A, column_scaling="jacobi").upload(DEV)
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        jac.jacobi_apply(x, 2, 0)
