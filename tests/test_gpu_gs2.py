"""GPU parity of the GS2-preconditioned MPK (Sec. 5.1, two-stage Gauss-Seidel; reading
R21) through the C ABI.

Each power is gamma + 2 sub-powers (D^{-1}, gamma sweeps with the strictly lower
triangle L, then A) and the sub-powers of all powers run as one chain.  The oracle
follows the paper's iteration with plain row loops; the GPU sums the lower entries in
level order during the full row's gather, so the two differ in summation order only,
and every power is held to the 1e-12 relative L2 bound used for FP64 powers here.
Blocked, plain and staged executors and both I/O orders share the row arithmetic and
agree bitwise."""
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


def run(A, x, p, gamma, permuted=True, q=4, values="f64", **kw):
    plan = Plan.from_csr(A, split_lower=True, p_block=q, values=values).upload(DEV)
    perm = plan.levels()["perm"].astype(np.int64)
    xin = x[perm] if permuted else x
    W = plan.gs2_apply(torch.tensor(xin, device=DEV), p, gamma, permuted=permuted, **kw)
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
    for i in range(n):
        seg = slice(rp[i], rp[i + 1])
        d = np.nonzero(c[seg] == i)[0]
        v[rp[i] + d[0]] = 1.0 + np.abs(v[seg]).sum()
    return S.CSR(n, rp, c, v)


MATS = {"lap3d": lambda: S.laplacian_3d(23, 19, 17), "knn12": lambda: S.knn_graph_laplacian(5000, k=12, seed=4),
        "nonsym": lambda: nonsym_dominant(5000, 8)}


@pytest.mark.parametrize("gamma", [0, 1, 2, 4])
@pytest.mark.parametrize("mk", list(MATS))
def test_gs2_mpk_matches_oracle(mk, gamma):
    A = MATS[mk]()
    x = S.uniform_vector(A.n, 2)
    W = run(A, x, 5, gamma)
    R = O.gs2_mpk(A, x, 5, gamma)
    assert rel_err(W, R) <= TOL


@pytest.mark.parametrize("gamma,q", [(1, 4), (2, 3), (2, 8), (0, 5), (3, 15)])
def test_blocked_plain_staged_and_io_orders_bitwise(gamma, q):
    A = S.laplacian_2d(61, 47)
    x = S.uniform_vector(A.n, 6)
    Wb = run(A, x, 4, gamma, q=q)
    Wp = run(A, x, 4, gamma, q=q, plain=True)
    Ws = run(A, x, 4, gamma, q=q, staged=True)
    Wo = run(A, x, 4, gamma, q=q, permuted=False)
    assert np.array_equal(Wb, Wp) and np.array_equal(Wb, Ws) and np.array_equal(Wb, Wo)


def test_fp32_values_state_their_error():
    # FP32 storage of A (the 0.1 shift of the kNN Laplacian is not representable): the
    # GPU computes the GS2 MPK of the rounded matrix; its error against FP64 is bounded
    A = S.knn_graph_laplacian(5000, k=12, seed=5)
    x = S.uniform_vector(A.n, 3)
    W = run(A, x, 3, 2, values="f32")
    R = O.gs2_mpk(A, x, 3, 2)
    err = rel_err(W, R)
    assert 0 < err <= 3 * 4 * 8 * 2.0 ** -24  # p (gamma + 2) times a few u32 per sub-power


def test_errors():
    A = S.laplacian_2d(9)
    x = torch.tensor(S.uniform_vector(A.n, 1), device=DEV)
    plain = Plan.from_csr(A).upload(DEV)
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        plain.gs2_apply(x, 2, 1)
    split = Plan.from_csr(A, split_lower=True).upload(DEV)
    with pytest.raises(MPKError, match="MPK_ERR_ARG"):
        split.gs2_apply(x, 2, 17)
