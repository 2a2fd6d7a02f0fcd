"""GPU test of the block-size tuner (p_opt of Sec. 3): the tuned block size is admissible,
and powers computed with it, with any fixed cap and with the plain launches agree bitwise
(the row arithmetic does not depend on where a block ends)."""
import numpy as np
import pytest

import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU-only hosts, never run there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_02228_amd import Plan  # noqa: E402

DEV = "cuda:0"


def test_tuned_block_is_admissible_and_results_unchanged():
    A = S.laplacian_3d(40, 36, 30)
    plan = Plan.from_csr(A, p_block=8).upload(DEV)
    x = plan.permute(torch.tensor(S.uniform_vector(A.n, 1), device=DEV), 0)
    bound = plan.info()["p_block"]
    q, t = plan.tune_block(x, 8)
    assert 1 <= q <= min(8, bound) and t > 0
    tuned = plan.apply(x, 8).cpu().numpy()
    plain = plan.apply(x, 8, plain=True).cpu().numpy()
    assert np.array_equal(tuned, plain)
    for cap in (1, 2, 3, 5, 0):
        plan.set_block(cap)
        assert np.array_equal(plan.apply(x, 8).cpu().numpy(), plain), cap
    plan.check()


def test_tuning_a_single_power_keeps_one():
    A = S.laplacian_2d(30, 20)
    plan = Plan.from_csr(A).upload(DEV)
    x = plan.permute(torch.tensor(S.uniform_vector(A.n, 2), device=DEV), 0)
    q, t = plan.tune_block(x, 1)
    assert q == 1
