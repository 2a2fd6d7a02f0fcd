"""GPU tests of the request server (mpk_server_*) through the C ABI.

Requests served together on several worker streams must give what the same
call gives alone: every kernel's row arithmetic is fixed and the solve's
reductions have a fixed order, so the comparison is bitwise.  One apply is
also checked against the oracle's powers (Eq. 1 recursion), and the
admission rules (arrival order, pool budget, per-request errors) are
exercised with host-side conditions only.  The mix holds matrix powers,
refinement solves and s-step GMRES solves."""
import threading

import numpy as np
import pytest

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU-only hosts, never run there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_02228_amd import Plan, MPKError  # noqa: E402
from paper_2309_02228_amd.mpk import Server, CALL_APPLY  # noqa: E402

DEV = "cuda:0"
MODES = {"blocked": {}, "plain": {"plain": True}, "staged": {"staged": True}}


def lap_bounds(dims):
    lmin = sum(2 - 2 * np.cos(np.pi / (m + 1)) for m in dims)
    lmax = sum(2 + 2 * np.cos(np.pi / (m + 1)) for m in dims)
    return lmin, lmax


@pytest.fixture(scope="module")
def problems():
    dims = (24, 22, 20)
    A = S.laplacian_3d(*dims)
    B = S.random_pattern(7000, 9, seed=11, symmetric=True)
    hi = Plan.from_csr(A).upload(DEV)
    lo = Plan.from_csr(A, values="f32").upload(DEV)
    pb = Plan.from_csr(B, p_block=3).upload(DEV)
    return {"A": A, "B": B, "hi": hi, "lo": lo, "pb": pb, "bounds": lap_bounds(dims)}


def alone_apply(plan, x, p, permuted, mode):
    Y = plan.apply(torch.tensor(x, device=DEV), p, permuted=permuted, **MODES[mode])
    plan.check()
    return Y.cpu().numpy()


def alone_solve(hi, lo, b, d, lmin, lmax, tol, it):
    x, k, rel = hi.refine_solve(lo, torch.tensor(b, device=DEV), d, lmin, lmax, tol=tol, max_iter=it)
    hi.check()
    lo.check()
    return x.cpu().numpy(), k, rel


def alone_gmres(hi, lo, b, s, m, d, lmin, lmax, tol, cycles):
    x, it, cy, rel = hi.sstep_gmres(lo, torch.tensor(b, device=DEV), s, m, d, lmin, lmax, tol=tol,
                                    max_cycles=cycles)
    hi.check()
    lo.check()
    return x.cpu().numpy(), it, rel


def request_mix(pr, seed, napply=20, nsolve=3, ngmres=3):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(napply):
        name = ["hi", "lo", "pb"][i % 3]
        n = pr["A"].n if name != "pb" else pr["B"].n
        reqs.append(("apply", name, S.uniform_vector(n, seed * 100 + i), int(rng.choice([1, 3, 4, 6, 9])),
                     bool(rng.integers(2)), str(rng.choice(list(MODES)))))
    for i in range(nsolve):
        reqs.append(("solve", "hi", S.uniform_vector(pr["A"].n, seed * 100 + 50 + i), 8 + 4 * i))
    for i in range(ngmres):
        s = (4, 8, 5)[i % 3]
        reqs.append(("gmres", "hi", S.uniform_vector(pr["A"].n, seed * 100 + 70 + i), s, 4 * s, 6 + 2 * i))
    rng.shuffle(reqs)
    return reqs


def expected(pr, reqs):
    lmin, lmax = pr["bounds"]
    out = []
    for r in reqs:
        if r[0] == "apply":
            out.append(alone_apply(pr[r[1]], r[2], r[3], r[4], r[5]))
        elif r[0] == "solve":
            out.append(alone_solve(pr["hi"], pr["lo"], r[2], r[3], lmin, lmax, 1e-10, 300))
        else:
            out.append(alone_gmres(pr["hi"], pr["lo"], r[2], r[3], r[4], r[5], lmin, lmax, 1e-10, 60))
    return out


def submit(srv, pr, r):
    lmin, lmax = pr["bounds"]
    if r[0] == "apply":
        return srv.submit_apply(pr[r[1]], r[2], r[3], permuted=r[4], **MODES[r[5]])
    if r[0] == "solve":
        return srv.submit_solve(pr["hi"], pr["lo"], r[2], r[3], lmin, lmax, tol=1e-10, max_iter=300)
    return srv.submit_gmres(pr["hi"], pr["lo"], r[2], r[3], r[4], r[5], lmin, lmax, tol=1e-10, max_cycles=60)


def check(r, got, want):
    if r[0] == "apply":
        assert np.array_equal(got["Y"], want), r[:2] + r[3:]
    else:
        x, k, rel = want
        assert got["iters"] == k and got["relres"] == rel and rel <= 1e-10
        assert np.array_equal(got["x"], x)


@pytest.mark.parametrize("workers", [1, 4])
def test_served_requests_equal_calls_made_alone(problems, workers):
    reqs = request_mix(problems, seed=workers)
    want = expected(problems, reqs)
    srv = Server(workers=workers, device_bytes=256 << 20)
    try:
        tickets = [submit(srv, problems, r) for r in reqs]
        for r, t, w in zip(reqs, tickets, want):
            got = srv.wait(t)
            assert got["latency_s"] >= got["queue_s"] >= 0.0
            check(r, got, w)
    finally:
        srv.close()


def test_served_apply_matches_oracle(problems):
    A, hi = problems["A"], problems["hi"]
    x = S.uniform_vector(A.n, 77)
    perm = hi.levels()["perm"].astype(np.int64)
    srv = Server(workers=2, device_bytes=64 << 20)
    try:
        got = srv.wait(srv.submit_apply(hi, x, 7, permuted=False))["Y"]
        got_p = srv.wait(srv.submit_apply(hi, x[perm], 7, permuted=True))["Y"]
        last = srv.wait(srv.submit_apply(hi, x, 7, permuted=False, last_only=True))["Y"]
    finally:
        srv.close()
    ref = O.mpk(A, x, 7)  # rows y_1..y_7
    scale = np.max(np.abs(ref), axis=1, keepdims=True)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)
    assert np.array_equal(got_p, got[:, perm])
    assert last.shape == (A.n,) and np.array_equal(last, got[-1])


def test_submit_and_wait_from_many_host_threads(problems):
    reqs = request_mix(problems, seed=9, napply=24, nsolve=2, ngmres=2)
    want = expected(problems, reqs)
    srv = Server(workers=3, device_bytes=256 << 20)
    errors = []

    def client(idx):
        try:
            for i in idx:
                check(reqs[i], srv.wait(submit(srv, problems, reqs[i])), want[i])
        except Exception as e:  # reported on the main thread
            errors.append(e)

    threads = [threading.Thread(target=client, args=(range(c, len(reqs), 6),)) for c in range(6)]
    try:
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in threads)
    finally:
        srv.close()
    assert not errors, errors[0]


def test_pool_budget_admits_in_arrival_order(problems):
    hi = problems["hi"]
    n, p = hi.n, 4
    per = 2 * 256 + n * 8 + n * 8 * p + hi.work_bytes(CALL_APPLY, p, 1) + 256 + 256
    xs = [S.uniform_vector(n, 300 + i) for i in range(6)]
    want = [alone_apply(hi, x, p, True, "blocked") for x in xs]
    srv = Server(workers=4, device_bytes=per)  # room for one request at a time
    try:
        with pytest.raises(MPKError, match="MPK_ERR_NOMEM"):
            srv.submit_apply(hi, xs[0], 64)  # larger than the whole pool
        tickets = [srv.submit_apply(hi, x, p) for x in xs]
        res = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for got, w in zip(res, want):
        assert np.array_equal(got["Y"], w)
    # one at a time, oldest first: the last request waited for the five before it
    assert res[-1]["queue_s"] > 0.0 and res[-1]["latency_s"] > res[0]["latency_s"]


def test_request_errors_stay_with_their_request(problems):
    A = problems["A"]
    idle = Plan.from_csr(A, values="f32")  # never uploaded
    lmin, lmax = problems["bounds"]
    b = S.uniform_vector(A.n, 5)
    srv = Server(workers=2, device_bytes=64 << 20)
    try:
        bad = srv.submit_solve(problems["hi"], idle, b, 4, lmin, lmax)
        good = srv.submit_apply(problems["hi"], b, 2)
        with pytest.raises(MPKError, match="MPK_ERR_STATE"):
            srv.wait(bad)
        assert np.array_equal(srv.wait(good)["Y"], alone_apply(problems["hi"], b, 2, True, "blocked"))
        with pytest.raises(MPKError, match="MPK_ERR_ARG"):
            srv.wait(good)  # a ticket is waited for once
    finally:
        srv.close()


def test_lanes_and_any_fit_admission_equal_alone(problems):
    # one general worker, two workers for matrix powers, any-fit admission: the mix
    # still equals the calls made alone bitwise
    reqs = request_mix(problems, seed=21, napply=24, nsolve=2, ngmres=3)
    want = expected(problems, reqs)
    srv = Server(workers=1, apply_workers=2, device_bytes=256 << 20, max_wait_s=0.05)
    try:
        tickets = [submit(srv, problems, r) for r in reqs]
        for r, t, w in zip(reqs, tickets, want):
            check(r, srv.wait(t), w)
    finally:
        srv.close()


def test_applies_do_not_wait_behind_a_solve(problems):
    # a long GMRES solve holds the only general worker; matrix powers submitted after it
    # run on the apply lane and finish first
    lmin, lmax = problems["bounds"]
    A, hi = problems["A"], problems["hi"]
    b = S.uniform_vector(A.n, 61)
    srv = Server(workers=1, apply_workers=1, device_bytes=256 << 20, max_wait_s=0.05)
    try:
        solve = srv.submit_gmres(hi, problems["lo"], b, 1, 200, 32, lmin, lmax, tol=1e-13, max_cycles=3)
        applies = [srv.submit_apply(hi, S.uniform_vector(A.n, 62 + i), 3) for i in range(4)]
        lat = [srv.wait(t)["latency_s"] for t in applies]
        s = srv.wait(solve)
    finally:
        srv.close()
    assert s["latency_s"] > 0.0
    assert max(lat) < s["latency_s"], (lat, s["latency_s"])


def test_plan_cache_hits_value_updates_and_eviction():
    from paper_2309_02228_amd import PlanCache
    A = S.laplacian_3d(30, 28, 26)
    B = S.knn_graph_laplacian(20000, k=26, seed=2)
    x = S.uniform_vector(A.n, 1)
    cache = PlanCache(device_bytes=512 << 20)
    try:
        p1, how = cache.get(A)
        assert how == "planned"
        perm = p1.levels()["perm"].astype(np.int64)
        xd = torch.tensor(x[perm], device=DEV)
        y1 = p1.apply(xd, 4).cpu().numpy()
        p2, how = cache.get(A)  # same pattern, same values
        h1 = p1._h.value
        assert how == "hit" and p2._h.value == h1
        p1.release()
        p2.release()
        # same pattern, new values (a shifted stencil): refilled, equal to a fresh plan
        A2 = S.CSR(A.n, A.rowptr, A.col, A.val * 0.5 + (A.col == np.repeat(np.arange(A.n), np.diff(A.rowptr))) * 3.0)
        p3, how = cache.get(A2)
        assert how == "new values" and p3._h.value == h1
        fresh = Plan.from_csr(A2).upload(DEV)
        assert np.array_equal(p3.apply(xd, 4).cpu().numpy(), fresh.apply(xd, 4).cpu().numpy())
        assert not np.array_equal(p3.apply(xd, 4).cpu().numpy(), y1)
        # a plan in use cannot take other values
        with pytest.raises(MPKError, match="MPK_ERR_STATE"):
            cache.get(A)
        p3.release()
        assert cache.stats() == {**cache.stats(), "plans": 1, "hits": 1, "value_updates": 1, "misses": 1}
    finally:
        cache.close()
    # a budget for one plan: the second pattern evicts the first once it is released
    one = Plan.from_csr(A).device_bytes
    cache = PlanCache(device_bytes=max(one, Plan.from_csr(B).device_bytes) + 256)
    try:
        pa, _ = cache.get(A)
        with pytest.raises(MPKError, match="MPK_ERR_NOMEM"):
            cache.get(B)  # the only plan is in use
        pa.release()
        pb, how = cache.get(B)
        assert how == "planned" and cache.stats()["plans"] == 1
        xb = S.uniform_vector(B.n, 3)
        permb = pb.levels()["perm"].astype(np.int64)
        got = pb.apply(torch.tensor(xb[permb], device=DEV), 3).cpu().numpy()
        back = np.empty_like(got)
        back[:, permb] = got
        ref = O.mpk(B, xb, 3)
        assert np.all(np.linalg.norm(back - ref, axis=1) <= 1e-12 * np.linalg.norm(ref, axis=1))
        pb.release()
    finally:
        cache.close()
