"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: level sets and permutations bit-exact (checked on the host planner
too); FP64 powers within 1e-12 relative L2 per power; integer inputs, whose
powers are exact in FP64 for any summation order, bit-exact; the blocked and
plain kernels bitwise identical (same per-row arithmetic)."""
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
    num = np.linalg.norm(got - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


def to_orig(Yp, perm):
    Y = np.empty_like(Yp)
    Y[..., perm] = Yp
    return Y


def make_plan(A, **kw):
    plan = Plan.from_csr(A, **kw).upload(DEV)
    perm = plan.levels()["perm"].astype(np.int64)
    return plan, perm


def run_apply(plan, perm, x, p, plain=False, permuted=True):
    if permuted:
        xd = torch.tensor(x[perm], device=DEV)
        Y = plan.apply(xd, p, plain=plain).cpu().numpy()
        plan.check()
        return to_orig(Y, perm)
    xd = torch.tensor(x, device=DEV)
    Y = plan.apply(xd, p, plain=plain, permuted=False).cpu().numpy()
    plan.check()
    return Y


CASES = {
    "lap2d_64x64": lambda: S.laplacian_2d(64),
    "lap2d_ragged_37x29": lambda: S.laplacian_2d(37, 29),
    "lap3d_24": lambda: S.laplacian_3d(24),
    "lap3d_ragged": lambda: S.laplacian_3d(19, 23, 17),
    "rand_nonsym": lambda: S.random_pattern(5000, 4, 1),
    "rand_disconnected": lambda: S.random_pattern(3000, 0.9, 2),
    "blocks": lambda: S.block_diagonal(S.laplacian_2d(30, 20), S.identity(100), S.laplacian_1d(700)),
    "knn_20k": lambda: S.knn_graph_laplacian(20000, k=26, seed=0),
    "wide_rows": lambda: S.random_pattern(3000, 40, 5),
    "band_nonsym": lambda: S.banded_random(20000, 6, 40, 1),
    "band_wide": lambda: S.banded_random(20000, 40, 60, 2),
}
# plans whose levels are narrow enough that the blocked kernel must run (not the
# plain fallback); the random patterns have a small diameter and wide levels
ENGAGED = {"lap2d_64x64", "lap2d_ragged_37x29", "lap3d_24", "lap3d_ragged", "band_nonsym", "band_wide",
           "knn_20k"}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("p", [1, 4, 9])
def test_mpk_apply_matches_oracle(name, p):
    A = CASES[name]()
    plan, perm = make_plan(A, p_block=4)
    if name in ENGAGED:
        assert plan.block_powers() >= 2
    x = S.uniform_vector(A.n, 0)
    ref = O.mpk(A, x, p)
    got = run_apply(plan, perm, x, p)
    assert np.all(rel_err(got, ref) <= TOL), rel_err(got, ref)
    plain = run_apply(plan, perm, x, p, plain=True)
    assert np.array_equal(plain, got)  # same row arithmetic: bitwise equal


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_config1_blocked_p4_seeds(seed):
    # 2D 5-point 64x64, x uniform[-1,1] from seed, p = 4
    A = S.laplacian_2d(64)
    plan, perm = make_plan(A)
    x = S.uniform_vector(A.n, seed)
    got = run_apply(plan, perm, x, 4)
    assert np.all(rel_err(got, O.mpk(A, x, 4)) <= TOL)
    got_io = run_apply(plan, perm, x, 4, permuted=False)
    assert np.array_equal(got_io, got)


@pytest.mark.parametrize("mk", [lambda: S.laplacian_2d(64), lambda: S.laplacian_3d(21, 17, 13)])
def test_integer_input_bit_exact(mk):
    A = mk()
    plan, perm = make_plan(A, p_block=8)
    x = S.integer_vector(A.n, 3)
    got = run_apply(plan, perm, x, 8)
    assert np.array_equal(got, O.mpk(A, x, 8))


@pytest.mark.parametrize("pb", [1, 2, 3, 5, 15])
def test_block_sizes_and_remainder(pb):
    A = S.laplacian_3d(16, 16, 16)
    plan, perm = make_plan(A, p_block=pb)
    x = S.uniform_vector(A.n, 4)
    got = run_apply(plan, perm, x, 11)
    assert np.all(rel_err(got, O.mpk(A, x, 11)) <= TOL)


def test_special_matrices():
    x = S.uniform_vector(257, 1)
    for A, ref in [(S.identity(257), np.tile(x, (5, 1))),
                   (S.cyclic_shift(257), np.stack([np.roll(x, -(k + 1)) for k in range(5)])),
                   (S.CSR(257, np.zeros(258, np.int32), np.zeros(0, np.int32), np.zeros(0)), np.zeros((5, 257)))]:
        plan, perm = make_plan(A)
        got = run_apply(plan, perm, x, 5)
        assert np.array_equal(got, ref)
    A = S.from_dense([[3.0]])
    plan, perm = make_plan(A)
    assert np.array_equal(run_apply(plan, perm, np.array([2.0]), 3)[:, 0], [6.0, 18.0, 54.0])


def test_long_range_entry_nonsymmetric():
    M = np.eye(300) * 2.0
    M[0, 299] = 5.0
    M[17, 3] = -1.0
    A = S.from_dense(M)
    plan, perm = make_plan(A)
    x = S.uniform_vector(300, 7)
    got = run_apply(plan, perm, x, 6)
    assert np.all(rel_err(got, O.mpk(A, x, 6)) <= TOL)


def test_ldy_and_strided_output():
    A = S.laplacian_2d(33, 31)
    plan, perm = make_plan(A)
    x = S.uniform_vector(A.n, 2)
    buf = torch.full((5, A.n + 77), float("nan"), dtype=torch.float64, device=DEV)
    Y = buf[:, :A.n]
    plan.apply(torch.tensor(x[perm], device=DEV), 5, Y=Y)
    plan.check()
    got = to_orig(Y.cpu().numpy(), perm)
    assert np.all(rel_err(got, O.mpk(A, x, 5)) <= TOL)
    assert torch.isnan(buf[:, A.n:]).all()  # padding untouched


@pytest.mark.parametrize("kind", ["monomial", "newton", "chebyshev"])
@pytest.mark.parametrize("d", [0, 1, 3, 8, 13])
def test_poly_apply_matches_oracle(kind, d):
    A = S.laplacian_3d(18, 15, 12)
    plan, perm = make_plan(A, p_block=4)
    x = S.uniform_vector(A.n, 5)
    rng = np.random.default_rng(d)
    c = rng.uniform(-1, 1, d + 1)
    if kind == "monomial":
        c = c / 12.0 ** np.arange(d + 1)  # keep the terms comparable
        params, ref = None, O.poly_monomial(A, x, c)
    elif kind == "newton":
        params = rng.uniform(0, 12, d)
        c = c / 12.0 ** np.arange(d + 1)
        ref = O.poly_newton(A, x, c, params)
    else:
        params = np.array([6.0, 6.0])
        ref = O.poly_chebyshev(A, x, c, 6.0, 6.0)
    for permuted in (True, False):
        xin = torch.tensor(x[perm] if permuted else x, device=DEV)
        out = plan.poly(kind, c, xin, params=params, permuted=permuted).cpu().numpy()
        plan.check()
        got = to_orig(out, perm) if permuted else out
        assert rel_err(got, ref) <= TOL, (permuted, rel_err(got, ref))
    plain = plan.poly(kind, c, torch.tensor(x[perm], device=DEV), params=params, plain=True).cpu().numpy()
    blocked = plan.poly(kind, c, torch.tensor(x[perm], device=DEV), params=params).cpu().numpy()
    assert np.array_equal(plain, blocked)


@pytest.mark.parametrize("s", [1, 4, 8])
@pytest.mark.parametrize("scaled", [False, True])
def test_sstep_basis_matches_oracle(s, scaled):
    A = S.knn_graph_laplacian(12000, k=26, seed=3)
    plan, perm = make_plan(A, p_block=4)
    v = S.uniform_vector(A.n, 8)
    rng = np.random.default_rng(s)
    lam = rng.uniform(0.1, 50, s)
    sig = rng.uniform(20, 60, s) if scaled else None
    ref = O.newton_basis(A, v, lam, sig)
    Vp = plan.sstep(torch.tensor(v[perm], device=DEV), lam, sig).cpu().numpy()
    plan.check()
    got = to_orig(Vp, perm)
    assert np.array_equal(got[0], v)
    assert np.all(rel_err(got, ref) <= TOL), rel_err(got, ref)
    Vo = plan.sstep(torch.tensor(v, device=DEV), lam, sig, permuted=False).cpu().numpy()
    assert np.array_equal(Vo, got)
    Vpl = plan.sstep(torch.tensor(v[perm], device=DEV), lam, sig, plain=True).cpu().numpy()
    assert np.array_equal(Vpl, Vp)


def test_sstep_integer_shifts_exact():
    A = S.laplacian_2d(40, 40)
    plan, perm = make_plan(A)
    v = S.integer_vector(A.n, 1, bound=1 << 12)
    lam = [1.0, -3.0, 2.0, 0.0, 4.0]
    got = to_orig(plan.sstep(torch.tensor(v[perm], device=DEV), lam).cpu().numpy(), perm)
    assert np.array_equal(got, O.newton_basis(A, v, lam))


def test_permute_roundtrip():
    A = S.random_pattern(4000, 3, 3)
    plan, perm = make_plan(A)
    x = S.uniform_vector(A.n, 1)
    xd = torch.tensor(x, device=DEV)
    xp = plan.permute(xd, 0)
    assert np.array_equal(xp.cpu().numpy(), x[perm])
    assert np.array_equal(plan.permute(xp, 1).cpu().numpy(), x)


def test_repeated_calls_alternate_inputs_into_one_buffer():
    # two inputs alternate into the same Y buffer: a value left from the previous
    # launch must never be taken for this launch's
    A = S.laplacian_3d(20)
    plan, perm = make_plan(A, p_block=3)
    assert plan.block_powers() == 3
    xs = [S.uniform_vector(A.n, 9), S.uniform_vector(A.n, 10)]
    refs = [O.mpk(A, x, 7) for x in xs]
    xds = [torch.tensor(x[perm], device=DEV) for x in xs]
    Y = torch.empty((7, A.n), dtype=torch.float64, device=DEV)
    for i in range(12):
        plan.apply(xds[i % 2], 7, Y=Y)
        plan.check()
        assert np.all(rel_err(to_orig(Y.cpu().numpy(), perm), refs[i % 2]) <= TOL), i


def test_non_finite_inputs_and_the_pending_pattern():
    # NaN, infinities and the bit pattern the blocked kernel uses for entries not
    # yet written (a signalling NaN) in x: arithmetic quiets NaNs, so the launch
    # must finish and give bitwise the plain kernel's results
    A = S.laplacian_3d(18, 17, 16)
    plan, perm = make_plan(A, p_block=4)
    assert plan.block_powers() == 4
    x = S.uniform_vector(A.n, 4)
    pend = np.array([0x7FF05E471A3E0001], dtype=np.uint64).view(np.float64)[0]
    x[[5, 700, 2900]] = [np.nan, np.inf, -np.inf]
    x[[17, 1800, A.n - 1]] = pend
    blocked = run_apply(plan, perm, x, 4).view(np.int64)
    plain = run_apply(plan, perm, x, 4, plain=True).view(np.int64)
    assert np.array_equal(blocked, plain)
    assert not np.any(blocked == np.int64(0x7FF05E471A3E0001))
    fin = np.isfinite(O.mpk(A, np.nan_to_num(x, nan=0.0, posinf=0.0, neginf=0.0), 4))
    assert fin.all()


def test_watchdog_reports_and_recovers():
    # forced from the host: every dependency wait gives up at once; all waves exit
    A = S.laplacian_2d(64)
    plan, perm = make_plan(A, watchdog_polls=-1)
    assert plan.block_powers() >= 2
    x = torch.tensor(S.uniform_vector(A.n, 0)[perm], device=DEV)
    plan.apply(x, 4)
    with pytest.raises(MPKError) as e:
        plan.check()
    assert e.value.code == -7 and "watchdog" in str(e.value)
    plan.check()  # status cleared
    ok, perm2 = make_plan(A)
    Y = ok.apply(x, 4)
    ok.check()
    assert np.all(rel_err(to_orig(Y.cpu().numpy(), perm2), O.mpk(A, S.uniform_vector(A.n, 0), 4)) <= TOL)


def test_device_status_belongs_to_the_stream_that_failed():
    # one plan, two streams: a launch forced to give up on stream a reports on a
    # only; the later good launch on stream b reports success
    A = S.laplacian_2d(64)
    plan, perm = make_plan(A)
    x0 = S.uniform_vector(A.n, 0)
    x = torch.tensor(x0[perm], device=DEV)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    plan.set_watchdog(-1)
    plan.apply(x, 4, stream=sa)
    sa.synchronize()
    plan.set_watchdog(0)
    Y = plan.apply(x, 4, stream=sb)
    plan.check(stream=sb)
    assert np.all(rel_err(to_orig(Y.cpu().numpy(), perm), O.mpk(A, x0, 4)) <= TOL)
    with pytest.raises(MPKError) as e:
        plan.check(stream=sa)
    assert e.value.code == -7
    plan.check(stream=sa)  # cleared by the report


@pytest.mark.slow
def test_full_size_160_cubed():
    # 3D 7-point 160^3 (N = 4,096,000; 28,518,400 nnz), the benchmarked workload
    A = S.laplacian_3d(160)
    plan = Plan.from_csr(A, p_block=4)
    lv = plan.levels()
    level, nl, _ = O.bfs_levels(A)
    assert lv["nlevels"] == nl == 478
    assert np.array_equal(lv["level_of_row"], level)
    perm, iperm, lp = O.level_permutation(level, nl)
    assert np.array_equal(lv["perm"], perm) and np.array_equal(lv["level_ptr"], lp)
    plan.upload(DEV)
    x = S.uniform_vector(A.n, 0)
    got = run_apply(plan, perm, x, 4)
    assert np.all(rel_err(got, O.mpk(A, x, 4)) <= TOL)
    plain = run_apply(plan, perm, x, 4, plain=True)
    assert np.array_equal(plain, got)
    xi = S.integer_vector(A.n, 1)
    assert np.array_equal(run_apply(plan, perm, xi, 4), O.mpk(A, xi, 4))


@pytest.mark.parametrize("pb", [4, 8])
@pytest.mark.parametrize("mk", [lambda: S.laplacian_3d(100), lambda: S.laplacian_2d(1100, 1000)])
def test_wide_units_of_the_fp64_kernels(mk, pb):
    # rows of 7 slots, enough units per partition to fill every resident wave: the FP64
    # kernels carry 5 chunks per wave at 2 waves per SIMD, the plain powers' 6, the GS2
    # chain's 3 and the smoother's 2
    A = mk()
    plan, perm = make_plan(A, p_block=pb)
    w, g, reg = plan.block_shape("powers")
    assert (g, reg) == (6, 7)
    q = plan.block_powers()
    assert q >= 2 and plan.min_workers(q, 6) <= w
    for op in ("poly_monomial", "poly_newton", "poly_chebyshev", "newton_basis", "jacobi_chain", "gs2_chain"):
        wo, go, _ = plan.block_shape(op)
        assert go == (3 if op == "gs2_chain" else 5) and plan.min_workers(plan.block_powers(op), go) <= wo, op
    assert plan.block_shape("gs2_smooth")[1] == 2
    x = S.uniform_vector(A.n, 7)
    got = run_apply(plan, perm, x, 2 * pb + 1)
    assert np.all(rel_err(got, O.mpk(A, x, 2 * pb + 1)) <= TOL)
    assert np.array_equal(run_apply(plan, perm, x, 2 * pb + 1, plain=True), got)
    assert np.array_equal(run_apply(plan, perm, x, 2 * pb + 1, permuted=False), got)
    # an explicit group of 2 gives the same values bit for bit
    plan2, perm2 = make_plan(A, p_block=pb, chunks_per_worker=2)
    assert plan2.block_shape("powers")[1] == 2
    assert np.array_equal(run_apply(plan2, perm2, x, 2 * pb + 1), got)
    # every kind runs the kernel built for its unit table: blocked equals plain bitwise
    # for the polynomials and the Newton basis too (a kernel of another G would leave
    # part of each unit's rows unwritten)
    xd = torch.tensor(x[perm], device=DEV)
    c = np.linspace(0.5, -0.3, 2 * pb + 1)
    for kind, params in (("monomial", None), ("newton", np.linspace(0.1, 2.0, 2 * pb)),
                         ("chebyshev", np.array([6.0, 6.0]))):
        yb = plan.poly(kind, c, xd, params=params)
        yp = plan.poly(kind, c, xd, params=params, plain=True)
        plan.check()
        assert torch.equal(yb, yp), kind
    lam = np.linspace(0.5, 5.0, pb)
    Vb = plan.sstep(xd, lam)
    Vp = plan.sstep(xd, lam, plain=True)
    plan.check()
    assert torch.equal(Vb, Vp)


@pytest.mark.parametrize("G", [1, 2, 4])
@pytest.mark.parametrize("mk", [lambda: S.laplacian_3d(23, 19, 21), lambda: S.random_pattern(9000, 5, 4)])
def test_chunks_per_worker(G, mk):
    A = mk()
    plan, perm = make_plan(A, p_block=5, chunks_per_worker=G)
    x = S.uniform_vector(A.n, 6)
    got = run_apply(plan, perm, x, 12)
    assert np.all(rel_err(got, O.mpk(A, x, 12)) <= TOL)
    assert np.array_equal(run_apply(plan, perm, x, 12, plain=True), got)
