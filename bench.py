#!/usr/bin/env python3
"""Benchmark of the temporally blocked matrix power kernel on one MI355X.

Workload: 3D 7-point Laplacian on a 160^3 grid (N = 4,096,000 rows,
28,518,400 nonzeros, FP64), x uniform[-1, 1] from seed 0, p = 4 powers
y_k = A^k x, all four stored.  A step is one MPK call with inputs and outputs
resident in HBM in level order (the plan's permuted space); the plan (BFS
levels, permutation, layout, schedule) is built once beforehand and its cost
is reported separately, as the paper treats it as a one-time preprocessing
cost.  The plain comparator (p back-to-back SpMV launches on the same layout)
is timed the same way.  GF/s counts 2 flops per nonzero per power.

One JSON line goes to stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mpk_block_lap3d160_p4.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2309_02228_amd", "csrc", "mpk.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n, nnz, p):
    """Bytes the blocked MPK must move: the CSR matrix once (8-byte values,
    4-byte column indices, 4-byte row pointers), x read once, p outputs written."""
    b_mat = nnz * 12 + 4 * (n + 1)
    return b_mat + 8 * n * (p + 1), b_mat


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def load_traffic(sha):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != sha:
        return None
    return t.get("ea_bytes_per_launch")


def cpu_child(grid, p, reps):
    """Runs in a child process (no GPU): times the plain C reference of the oracle on
    the 3D 7-point Laplacian, pinned to one core, then with OpenMP on every host core
    this process may use, then the NumPy oracle; prints one JSON line."""
    import numpy as np
    import oracle
    import synth
    from oracle import ref_c
    if not os.path.exists(ref_c.LIB):
        ref_c.build()
    A = synth.laplacian_3d(grid)
    x = synth.uniform_vector(A.n, 0)
    flops = 2.0 * A.col.size * p
    allowed = sorted(os.sched_getaffinity(0))

    def median_time(fn):
        fn()  # warm-up
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    os.sched_setaffinity(0, {allowed[0]})
    t1 = median_time(lambda: ref_c.mpk(A, x, p))
    os.sched_setaffinity(0, set(allowed))
    used = [0]

    def par():
        used[0] = ref_c.mpk_omp(A, x, p, len(allowed))[1]
    tp = median_time(par)
    os.sched_setaffinity(0, {allowed[0]})
    tn = median_time(lambda: oracle.mpk(A, x, p))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    print(json.dumps({"c_1core_s": t1, "c_omp_s": tp, "omp_threads": used[0], "numpy_1core_s": tn,
                      "gflop": flops / 1e9, "allowed_cpus": len(allowed), "nproc": os.cpu_count(),
                      "cpu_model": model}), flush=True)


def cpu_baseline(grid, p):
    """The oracle on the host: the plain C reference on one core (the baseline), and the
    same loops with OpenMP on every core the process may use, both timed in a child
    process that never touches the GPU."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", "--grid", str(grid), "--p", str(p)],
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"value": None, "unit": "GFLOP/s", "cores": 1, "kind": "oracle", "error": r.stderr[-500:]}
    c = json.loads(r.stdout.strip().splitlines()[-1])
    sample = (f"full {grid}^3 matrix, p={p}: median of 5 complete MPK calls after one warm-up")
    return {
        "value": round(c["gflop"] / c["c_1core_s"], 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
        "sample": sample + " (oracle/mpk_ref.c, gcc -O2 -ffp-contract=off, pinned to one core)",
        "ms_per_mpk": round(c["c_1core_s"] * 1e3, 2),
        "all_cores": {"value": round(c["gflop"] / c["c_omp_s"], 3), "unit": "GFLOP/s",
                      "threads": c["omp_threads"], "ms_per_mpk": round(c["c_omp_s"] * 1e3, 2),
                      "note": "the same loops with OpenMP over rows, every CPU this process may use"},
        "numpy_oracle_1core": {"value": round(c["gflop"] / c["numpy_1core_s"], 3), "unit": "GFLOP/s"},
        "host": {"nproc": c["nproc"], "cpus_allowed": c["allowed_cpus"], "cpu_model": c["cpu_model"]},
    }


def knn_bench(args, dev, stream):
    """The unstructured workload: the shifted graph Laplacian of the symmetrised
    26-NN graph of uniform points in the unit cube (Morton order), FP64.  Blocked
    against plain powers, the tuned block size, the degree-8 Chebyshev polynomial
    and s-step GMRES (s = 8) with that polynomial as right preconditioner."""
    import numpy as np
    import torch
    import oracle
    import synth
    from paper_2309_02228_amd import Plan
    t0 = time.perf_counter()
    A = synth.knn_graph_laplacian(args.knn_points, k=26, seed=0)
    t_gen = time.perf_counter() - t0
    n, nnz = A.n, int(A.col.size)
    t0 = time.perf_counter()
    plan = Plan.from_csr(A, p_block=8)
    t_plan = time.perf_counter() - t0
    plan.upload(dev)
    info = plan.info()
    log(f"knn: {n} rows, {nnz} nonzeros ({t_gen:.1f} s to generate), plan {t_plan:.2f} s, {info}")
    x = plan.permute(torch.tensor(synth.uniform_vector(n, 0), device=dev), 0)

    def tm(fn, reps=10):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        plan.check()
        return e0.elapsed_time(e1) / reps * 1e-3
    powers = {}
    Y = torch.empty((8, n), dtype=torch.float64, device=dev)
    for pp in (1, 2, 4, 8):
        tb = tm(lambda: plan.apply(x, pp, Y=Y[:pp]))
        tp = tm(lambda: plan.apply(x, pp, Y=Y[:pp], plain=True))
        f = 2.0 * nnz * pp
        powers[str(pp)] = {"blocked_us": round(tb * 1e6, 1), "plain_us": round(tp * 1e6, 1),
                           "blocked_gflops": round(f / tb / 1e9, 1), "plain_gflops": round(f / tp / 1e9, 1),
                           "speedup": round(tp / tb, 3)}
    q_opt, t_opt = plan.tune_block(x, 8, Y=Y)
    plan.set_block(0)
    lmax = 2.0 * float(np.max(np.diff(A.rowptr))) + 0.1
    c, th, de = oracle.chebyshev_inverse_coeffs(8, 0.1, lmax)
    prm = np.array([th, de])
    tb = tm(lambda: plan.poly("chebyshev", c, x, params=prm))
    tp = tm(lambda: plan.poly("chebyshev", c, x, params=prm, plain=True))
    cheb = {"blocked_us": round(tb * 1e6, 1), "plain_us": round(tp * 1e6, 1), "speedup": round(tp / tb, 3)}
    bvec = plan.permute(torch.tensor(synth.uniform_vector(n, 1), device=dev), 0)
    work = torch.empty(plan.gmres_work_bytes(8, 64, 8) // 8 + 64, dtype=torch.float64, device=dev)
    lat, res = [], None
    for r in range(6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.sstep_gmres(plan, bvec, 8, 64, 8, 0.1, lmax, tol=1e-8, max_cycles=50, work=work)
        torch.cuda.synchronize()
        if r > 0:
            lat.append(time.perf_counter() - t0)
    plan.check()
    true = float(torch.linalg.norm(bvec - plan.apply(res[0], 1)[0]) / torch.linalg.norm(bvec))
    lat = np.array(lat) * 1e3
    gm = {"p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
          "basis_vectors": res[1], "cycles": res[2], "final_rel_residual": res[3], "true_rel_residual": true}
    out = {
        "workload": f"shifted graph Laplacian (+0.1 I) of the symmetrised 26-NN graph of {n} uniform points in "
                    f"[0,1)^3, Morton order, FP64; {nnz} nonzeros ({nnz / n:.2f} per row), {info['nlevels']} BFS levels",
        "plan_build_s": round(t_plan, 2),
        "powers_per_blocked_launch": {"mpk": plan.block_powers("powers"),
                                      "chebyshev": plan.block_powers("poly_chebyshev")},
        "register_slots": info["reg_slots"],
        "mpk": powers,
        "p_opt": {"p": 8, "q_opt": q_opt, "us_per_call": round(t_opt * 1e6, 1),
                  "note": "mpk_tune_block over q = 1..min(8, deadlock bound); q = 1 is the plain kernel"},
        "chebyshev_degree8": cheb,
        "sstep_gmres": {**gm, "setup": "s = 8, m = 64, degree-8 Chebyshev right preconditioner on "
                                        f"[0.1, {lmax:g}], tol 1e-8, FP64, 5 solves after one warm-up"},
    }
    log("knn: " + ", ".join(f"p={k}: {v['speedup']}x" for k, v in powers.items())
        + f"; q_opt {q_opt}; chebyshev {cheb['speedup']}x; gmres p50 {gm['p50_ms']} ms ({gm['basis_vectors']} "
          f"vectors, true residual {true:.1e})")
    del plan, Y, work
    return out


def natural_order_library_spmv(A, x, p, steps, warmup, dev, y_ref, to_level):
    """p chained SpMVs y_k = A y_{k-1} on the matrix in its natural row order, FP64 CSR with
    32-bit indices, through torch's sparse CSR product (rocSPARSE underneath): a vendor-library
    comparator for the plain path, timed with events like the rest.  y_p is checked against
    the library's own y_p (`y_ref`, level order) to a rounding-order tolerance."""
    import torch
    try:
        M = torch.sparse_csr_tensor(torch.as_tensor(A.rowptr, dtype=torch.int32),
                                    torch.as_tensor(A.col, dtype=torch.int32),
                                    torch.as_tensor(A.val, dtype=torch.float64), size=(A.n, A.n)).to(dev)
        x0 = torch.as_tensor(x, dtype=torch.float64, device=dev).reshape(-1, 1)

        def chain():
            # sparse CSR times a one-column matrix; torch.mv on the same operands measured
            # about 47x slower on this stack, so the faster of the two is the comparator
            y = x0
            for _ in range(p):
                y = M @ y
            return y
        for _ in range(warmup):
            y = chain()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            y = chain()
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / steps
        yl = to_level(y.reshape(-1))
        rel = float((yl - y_ref).abs().max() / y_ref.abs().max())
        nnz = int(A.rowptr[-1])
        bytes_spmv = nnz * 12 + 4 * (A.n + 1) + 16 * A.n
        return {"us_per_step": round(us, 1), "us_per_spmv": round(us / p, 1),
                "gflops": round(2 * nnz * p / (us * 1e-6) / 1e9, 2),
                "gbs_per_spmv": round(bytes_spmv / (us / p * 1e-6) / 1e9, 1),
                "max_rel_diff_vs_blocked": rel,
                "note": "torch sparse CSR @ one dense column (rocSPARSE), natural row order, "
                        "FP64 values, int32 indices; a comparator, not part of the library"}
    except Exception as e:  # an unsupported sparse type on this torch build
        return {"error": f"{type(e).__name__}: {str(e)[:200]}"}


def serving_bench(args, A160, plan160, dev):
    """Open-loop serving of a mixed request stream through the library's request
    server: Poisson arrivals of matrix powers y_p = A^p x (p uniform in 2..10,
    FP64 or FP32 matrix values) and s-step GMRES solves to 1e-8 with a Chebyshev
    polynomial preconditioner (FP64 residuals and orthogonalisation, FP32-valued basis
    and preconditioner) on a catalogue of 2D/3D Laplacians and 26-NN
    graph Laplacians with N from 1e4 to 4.1e6.  Requests carry host vectors
    (pinned), so latencies include the PCIe copies.  Every request is first run
    alone (one worker, one request at a time); its alone latency sets the
    arrival rate and the per-request slowdown, and a sample of results is
    compared bit for bit between the two runs."""
    import numpy as np
    import torch
    import synth
    from paper_2309_02228_amd import Plan, PlanCache
    from paper_2309_02228_amd.mpk import Server

    rng = np.random.default_rng(args.serve_seed)
    # the catalogue's plans come from the library's plan cache, keyed by sparsity pattern
    # (the 160^3 stencil reuses the plan of the headline measurement)
    cache = PlanCache(device_bytes=12 << 30)

    def lap_bounds(dims):
        return (sum(2 - 2 * np.cos(np.pi / (m + 1)) for m in dims),
                sum(2 + 2 * np.cos(np.pi / (m + 1)) for m in dims))

    cat = []
    t0 = time.perf_counter()
    for name, make, dims in [("lap2d_100^2", lambda: synth.laplacian_2d(100), (100, 100)),
                             ("lap3d_50^3", lambda: synth.laplacian_3d(50), (50, 50, 50)),
                             ("knn26_3e4", lambda: synth.knn_graph_laplacian(30000, seed=3), None),
                             ("knn26_3e5", lambda: synth.knn_graph_laplacian(300000, seed=4), None),
                             ("lap2d_700^2", lambda: synth.laplacian_2d(700), (700, 700)),
                             ("lap3d_100^3", lambda: synth.laplacian_3d(100), (100, 100, 100)),
                             ("lap3d_160^3", None, (160, 160, 160))]:
        A = A160 if make is None else make()
        if dims is not None:
            lmin, lmax = lap_bounds(dims)
        else:
            lmin, lmax = 0.1, 2.0 * float(np.max(np.diff(A.rowptr))) + 0.1
        # blocks of up to 8 powers (the deadlock bound lowers q where levels are wide):
        # one launch for most applies, and the fastest block for the solves' polynomials
        hi = plan160 if make is None else cache.get(A, p_block=8)[0]
        lo = cache.get(A, p_block=8, values="f32")[0]
        # preconditioner degree: about a third of sqrt(kappa), 4..32, so that GMRES
        # needs a few dozen basis vectors
        deg = int(min(32, max(4, np.ceil(np.sqrt(lmax / lmin) / 3))))
        cat.append({"name": name, "n": A.n, "A": A, "hi": hi, "lo": lo, "lmin": lmin, "lmax": lmax, "degree": deg,
                    "x": synth.uniform_vector(A.n, 10), "b": synth.uniform_vector(A.n, 11)})
    torch.cuda.synchronize()
    log(f"serving: catalogue of {len(cat)} matrices planned in {time.perf_counter() - t0:.1f} s")

    nreq = args.serve_requests
    reqs = []
    for i in range(nreq):
        m = int(rng.integers(len(cat)))
        if rng.random() < 0.75:
            reqs.append(("apply", m, int(rng.integers(2, 11)), "f64" if rng.random() < 0.5 else "f32"))
        else:
            reqs.append(("solve", m))
    total = sum(cat[r[1]]["n"] for r in reqs)
    pinned = torch.empty(total + sum(c["n"] for c in cat) * 2, dtype=torch.float64, pin_memory=True).numpy()
    at = 0
    for c in cat:  # inputs in pinned host memory, shared read-only by the requests
        for key in ("x", "b"):
            pinned[at:at + c["n"]] = c[key]
            c[key] = pinned[at:at + c["n"]]
            at += c["n"]
    outs = []
    for r in reqs:
        outs.append(pinned[at:at + cat[r[1]]["n"]])
        at += cat[r[1]]["n"]

    def submit(srv, i):
        r, c = reqs[i], cat[reqs[i][1]]
        if r[0] == "apply":
            plan = c["hi"] if r[3] == "f64" else c["lo"]
            return srv.submit_apply(plan, c["x"], r[2], permuted=False, last_only=True, Y=outs[i])
        outs[i][:] = 0.0
        return srv.submit_gmres(c["hi"], c["lo"], c["b"], 8, 64, c["degree"], c["lmin"], c["lmax"], tol=1e-8,
                                max_cycles=50, x0=outs[i], permuted=False)

    pool = args.serve_pool_gib << 30
    # alone: one worker, one request at a time
    check_idx = list(range(min(64, nreq)))
    alone, ref = np.zeros(nreq), {}
    srv = Server(workers=1, device_bytes=pool)
    for i in range(nreq):
        res = srv.wait(submit(srv, i))
        alone[i] = res["latency_s"]
        if i in check_idx:
            ref[i] = outs[i].copy()
        if reqs[i][0] == "solve" and res["relres"] > 1e-8:
            raise RuntimeError(f"served solve {i} ended at relres {res['relres']:.3g}")
    srv.close()
    log(f"serving: {nreq} requests alone, {alone.sum():.2f} s of service, mean {alone.mean() * 1e3:.2f} ms")

    rate = args.serve_load / alone.mean()
    gaps = rng.exponential(1.0 / rate, size=nreq)
    arrive = np.cumsum(gaps) - gaps[0]
    srv = Server(workers=args.serve_workers, device_bytes=pool, apply_workers=args.serve_apply_workers,
                 max_wait_s=args.serve_max_wait)
    lat, queue = np.zeros(nreq), np.zeros(nreq)
    tickets = [None] * nreq
    import threading
    submitted = threading.Semaphore(0)

    failed = []

    def waiter():
        for i in range(nreq):
            submitted.acquire()
            if tickets[i] is None:  # the submitting loop stopped early
                return
            try:
                res = srv.wait(tickets[i])
            except Exception as e:  # re-raised on the main thread
                failed.append(e)
                continue
            lat[i], queue[i] = res["latency_s"], res["queue_s"]

    th = threading.Thread(target=waiter)
    th.start()
    t_start = time.perf_counter()
    try:
        for i in range(nreq):
            delay = t_start + arrive[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[i] = submit(srv, i)
            submitted.release()
            if (i + 1) % 128 == 0:
                log(f"serving: {i + 1} of {nreq} requests submitted")
    finally:
        submitted.release()  # lets the waiter see a missing ticket if the loop stopped early
        th.join()
        makespan = time.perf_counter() - t_start
        srv.close()
    if failed:
        raise failed[0]
    same = all(np.array_equal(ref[i], outs[i]) for i in check_idx)
    if not same:
        raise RuntimeError("served results differ from the same requests run alone")

    def pct(v, q):
        return round(float(np.percentile(v, q)) * 1e3, 3) if len(v) else None

    kinds = np.array([r[0] for r in reqs])
    by = {}
    for k in ("apply", "solve"):
        m = kinds == k
        by[k] = {"count": int(m.sum()), "p50_ms": pct(lat[m], 50), "p99_ms": pct(lat[m], 99),
                 "alone_p50_ms": pct(alone[m], 50), "alone_p99_ms": pct(alone[m], 99)}
    slow = lat / alone
    out = {
        "workload": f"{nreq} requests, Poisson arrivals at {rate:.1f}/s ({args.serve_load:.2f} x the alone "
                    f"service rate); matrices: " + ", ".join(f"{c['name']} (N={c['n']})" for c in cat) +
                    "; plans with blocks of up to 8 powers; 75% y_p = A^p x (p uniform 2..10, FP64 or FP32 values, "
                    "y_p returned), 25% s-step GMRES "
                    "solves to 1e-8 (s = 8, m = 64; right Chebyshev preconditioner of degree "
                    "min(32, max(4, sqrt(kappa) / 3)) through FP32-valued launches; FP64 residuals and "
                    "orthogonalisation)",
        "workers": args.serve_workers, "apply_workers": args.serve_apply_workers,
        "admission": f"any waiting request that fits, oldest first; aging bound {args.serve_max_wait} s",
        "pool_gib": args.serve_pool_gib,
        "throughput_req_s": round(nreq / makespan, 2), "makespan_s": round(makespan, 3),
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "queue_p50_ms": pct(queue, 50),
        "by_kind": by,
        "slowdown_vs_alone": {"p50": round(float(np.percentile(slow, 50)), 3),
                              "p99": round(float(np.percentile(slow, 99)), 3)},
        "alone_service_s": round(float(alone.sum()), 3),
        "bitwise_same_as_alone": f"{len(check_idx)} sampled requests",
        "note": "host buffers in pinned memory; latency = submit to result in host memory, PCIe copies "
                "included; plans built once before the run through the plan cache",
    }
    log(f"serving: {nreq / makespan:.1f} req/s, p50 {out['p50_ms']} ms, p99 {out['p99_ms']} ms "
        f"(solves p50 {by['solve']['p50_ms']} / p99 {by['solve']['p99_ms']} ms)")
    # the plan cache on one pattern with new values (a shifted 100^3 stencil): the levels
    # and layout are kept and only the values refilled, against planning from scratch
    for c in cat:
        for key in ("hi", "lo"):
            if c[key] is not plan160:
                c[key].release()
    A100 = next(c["A"] for c in cat if c["name"] == "lap3d_100^3")
    diag = A100.col == np.repeat(np.arange(A100.n), np.diff(A100.rowptr))
    shifted = synth.CSR(A100.n, A100.rowptr, A100.col, A100.val + 0.5 * diag)
    t0 = time.perf_counter()
    ps, how = cache.get(shifted, p_block=8)
    torch.cuda.synchronize()
    t_upd = time.perf_counter() - t0
    ps.release()
    t0 = time.perf_counter()
    Plan.from_csr(shifted, p_block=8).upload(dev)
    torch.cuda.synchronize()
    t_new = time.perf_counter() - t0
    out["plan_cache"] = {**cache.stats(), "new_values_outcome": how, "new_values_ms": round(t_upd * 1e3, 1),
                         "plan_and_upload_ms": round(t_new * 1e3, 1),
                         "note": "catalogue planned through the cache (FP64 and FP32 plans per pattern); then "
                                 "new values on the 100^3 pattern, refilled in place, against a fresh plan"}
    log(f"plan cache: {out['plan_cache']}")
    for c in cat:
        del c["lo"]
    cache.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--grid", type=int, default=160)
    ap.add_argument("--p-block", type=int, default=0)
    ap.add_argument("--chunks-per-worker", type=int, default=0)
    ap.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-knn", action="store_true", help="skip the unstructured 8M-point kNN workload")
    ap.add_argument("--knn-points", type=int, default=8_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32 and BF16 matrix-value measurements")
    ap.add_argument("--no-solve", action="store_true", help="skip the refinement-solve latency measurement")
    ap.add_argument("--no-sweep", action="store_true", help="skip the p = 1..8 sweep")
    ap.add_argument("--solve-reps", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true", help="skip the request-serving measurement")
    ap.add_argument("--no-cold", action="store_true", help="skip the cold-cache timing (profiler runs)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-apply-workers", type=int, default=4,
                    help="server workers that take matrix power requests only")
    ap.add_argument("--serve-max-wait", type=float, default=0.1,
                    help="aging bound (s) of the server's any-fit admission")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="arrival rate as a fraction of the one-at-a-time service rate")
    ap.add_argument("--serve-pool-gib", type=int, default=8)
    ap.add_argument("--serve-seed", type=int, default=5)
    ap.add_argument("--solve-degree", type=int, default=256)
    ap.add_argument("--gmres-only", action="store_true",
                    help="run only s-step GMRES solves of the 3D stencil (profiler target)")
    ap.add_argument("--gmres-s", type=int, default=8)
    ap.add_argument("--gmres-m", type=int, default=64)
    ap.add_argument("--gmres-degree", type=int, default=32)
    ap.add_argument("--only", choices=["both", "blocked", "plain"], default="both",
                    help="restrict the launches (for profiler runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (scales the HBM byte "
                         "counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.cpu_child:
        cpu_child(args.grid, args.p, 5)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU matrix power "
              "kernel; no multi-GPU path exists (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2309_02228_amd import Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = "cuda:0"
    if args.gmres_only:
        # profiler target: the s-step GMRES solve of the 3D 7-point Laplacian alone
        g = args.grid
        A = synth.laplacian_3d(g)
        cg = np.cos(np.pi / (g + 1))
        lmin, lmax = 3 * (2 - 2 * cg), 3 * (2 + 2 * cg)
        hi8 = Plan.from_csr(A, p_block=8).upload(dev)
        lo8 = Plan.from_csr(A, p_block=8, values="f32").upload(dev)
        bvec = hi8.permute(torch.tensor(synth.uniform_vector(A.n, 1), device=dev), 0)
        for r in range(args.solve_reps):
            res = hi8.sstep_gmres(lo8, bvec, args.gmres_s, args.gmres_m, args.gmres_degree, lmin, lmax, tol=1e-10,
                                  max_cycles=200)
            log(f"gmres solve {r}: {res[1]} vectors, {res[2]} cycles, relres {res[3]:.3e}")
        lo8.check()
        print(json.dumps({"gmres_solves": args.solve_reps, "basis_vectors": res[1], "relres": res[3]}), flush=True)
        return
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": nbytes, "copies": 5}), flush=True)
        return
    g, p = args.grid, args.p
    A = synth.laplacian_3d(g)
    n, nnz = A.n, int(A.col.size)
    log(f"matrix: 3D 7-point Laplacian {g}^3, N={n}, nnz={nnz}")
    t0 = time.perf_counter()
    plan = Plan.from_csr(A, p_block=args.p_block or min(p, 15),
                         chunks_per_worker=args.chunks_per_worker)
    t_plan = time.perf_counter() - t0
    plan.upload(dev)
    torch.cuda.synchronize()
    t_upload = time.perf_counter() - t0 - t_plan
    info = plan.info()
    log(f"plan: {t_plan:.2f} s host planning, {t_upload:.2f} s upload; {info}")

    x = synth.uniform_vector(n, 0)
    xd = plan.permute(torch.tensor(x, device=dev), 0)  # into level order, on the device
    Y = torch.empty((p, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def timed(plain, plan=plan, xd=xd, Y=Y):
        for _ in range(args.warmup):
            plan.apply(xd, p, Y=Y, plain=plain)
        plan.check()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        evs[0].record(stream)
        for k in range(args.steps):
            plan.apply(xd, p, Y=Y, plain=plain)
            evs[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        plan.check()
        per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]) * 1e-3
        return wall, per

    def timed_staged():
        for _ in range(args.warmup):
            plan.apply(xd, p, Y=Y, staged=True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            plan.apply(xd, p, Y=Y, staged=True)
        torch.cuda.synchronize()
        plan.check()
        return time.perf_counter() - t_start, None

    res = {}
    if args.only in ("both", "blocked"):
        wall_b, per_b = timed(False)
        res["blocked"] = (wall_b, per_b)
        log(f"blocked: {wall_b / args.steps * 1e6:.1f} us/step (median event {np.median(per_b) * 1e6:.1f} us)")
    if args.only in ("both", "plain"):
        wall_p, per_p = timed(True)
        res["plain"] = (wall_p, per_p)
        log(f"plain:   {wall_p / args.steps * 1e6:.1f} us/step (median event {np.median(per_p) * 1e6:.1f} us)")

    flops = 2.0 * nnz * p
    b_blk, b_mat = algorithmic_bytes(n, nnz, p)
    key = "blocked" if "blocked" in res else "plain"
    wall, per = res[key]
    value = flops * args.steps / wall / 1e9
    launches_per_step = (-(-p // info["p_block"])) if key == "blocked" else p
    avg_launch = float(np.mean(per)) / launches_per_step
    bytes_per_launch = (b_blk if key == "blocked" else (b_mat + 16 * n)) / launches_per_step
    achieved = bytes_per_launch / avg_launch / 1e9
    sha = kernel_sha()
    traffic = load_traffic(sha) if key == "blocked" else None
    shape = plan.block_shape("powers")  # waves per XCD, chunks per wave, register slots

    out = {
        "metric": "MPK GFLOP/s vs p×SpMV (7-pt 160^3, p=4) + solve p50/p99 latency",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D 7-point Laplacian {g}^3 (N={n}, nnz={nnz}), FP64, SELL-64 in BFS level "
                        f"order, x uniform[-1,1] seed 0, p={p} powers stored, I/O in level order",
            "p": p, "p_block": info["p_block"], "kernel": key,
            "timing": "warm: the calls run back to back with x, Y and the plan resident in HBM (part of the "
                      "matrix may still sit in the 256 MB Infinity Cache from the previous call); HIP events "
                      "on the launch stream; cold_cache_timing gives each call timed alone after writing "
                      "2 GiB",
            "chunks_per_worker": shape[1],
            "workers_per_xcd": shape[0],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_counts": "L2-miss (EA) bytes of FETCH_SIZE + WRITE_SIZE per launch, copy-calibrated; "
                              "they include Infinity Cache hits (no MALL counter on gfx950), so they bound "
                              "the HBM bytes from above",
            "kernel": "mpk_block_kernel" if key == "blocked" else "spmv_kernel",
            "bytes_per_launch": int(bytes_per_launch),
            "avg_launch_us": round(avg_launch * 1e6, 2),
        },
        "plan_build_s": round(t_plan, 3),
        "plan_upload_s": round(t_upload, 3),
    }
    res_cold = None
    if args.only == "both" and not args.no_cold:
        # cold-cache protocol: a 2 GiB write before every run evicts the matrix from L2 and
        # the 256 MB Infinity Cache; 3 warm-ups, then 20 runs timed one by one
        scrub = torch.empty(1 << 28, dtype=torch.float64, device=dev)

        def scrubbed(plain):
            for _ in range(3):
                plan.apply(xd, p, Y=Y, plain=plain)
            ts = []
            for _ in range(20):
                scrub.fill_(1.0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                plan.apply(xd, p, Y=Y, plain=plain)
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e3)
            plan.check()
            ts = np.array(ts)
            return {"median_us": round(float(np.median(ts)), 1), "p10_us": round(float(np.percentile(ts, 10)), 1),
                    "p90_us": round(float(np.percentile(ts, 90)), 1)}
        cold_b, cold_p = scrubbed(False), scrubbed(True)
        del scrub
        res_cold = {"blocked": cold_b, "plain": cold_p,
                    "speedup_median": round(cold_p["median_us"] / cold_b["median_us"], 3),
                    "note": "each MPK call timed alone after writing 2 GiB (L2 and Infinity Cache evicted)"}
        log(f"cold caches: blocked {cold_b['median_us']} us, plain {cold_p['median_us']} us (median of 20)")
    if args.only == "both":
        # the paper's level-group wavefront (one launch per stage) for comparison
        wall_s, _ = timed_staged()
        ng, tasks = plan.schedule(info["p_block"])
        res_staged = {"gflops": round(flops * args.steps / wall_s / 1e9, 2),
                      "ms_per_step": round(wall_s / args.steps * 1e3, 5),
                      "groups": ng, "stages_per_block": int(tasks[:, 0].max()) + 1 if len(tasks) else 0,
                      "cache_mib": 256,
                      "note": "level groups under floor(C/q) bytes, task (k, g) at stage g + k - 1; "
                              "one launch per stage"}
        log(f"staged:  {wall_s / args.steps * 1e6:.1f} us/step ({ng} groups)")
    res_nat = None
    if args.only == "both":
        res_nat = natural_order_library_spmv(A, x, p, args.steps, args.warmup, dev, Y[p - 1].clone(),
                                             lambda v: plan.permute(v, 0))
        if "us_per_spmv" in res_nat:
            log(f"natural order, library CSR SpMV: {res_nat['us_per_spmv']} us per SpMV "
                f"({res_nat['gbs_per_spmv']} GB/s), rel diff {res_nat['max_rel_diff_vs_blocked']:.1e}")
        else:
            log(f"natural order, library CSR SpMV: {res_nat['error']}")
    if "plain" in res and "blocked" in res:
        wp = res["plain"][0]
        out["plain_gflops"] = round(flops * args.steps / wp / 1e9, 2)
        out["speedup_vs_plain"] = round(wp / res["blocked"][0], 3)
        out["plan_build_spmv_equivalents"] = round(t_plan / (wp / args.steps / p), 1)
        out["roofline_equivalent_frac"] = round(value / (flops / (b_blk / (HBM_PEAK_GBS * 1e9)) / 1e9), 4)
    if args.only == "both":
        out["staged_wavefront"] = res_staged
        if res_cold is not None:
            out["cold_cache_timing"] = res_cold
        out["natural_order_library_spmv"] = res_nat
    if args.only == "both" and not args.no_sweep:
        # p = 1..8 with one plan of blocks up to 8 powers (shorter jobs are one block)
        plan8 = Plan.from_csr(A, p_block=8).upload(dev)
        x8 = plan8.permute(torch.tensor(x, device=dev), 0)
        Y8 = torch.empty((8, n), dtype=torch.float64, device=dev)
        sweep = {}
        for pp in range(1, 9):
            tb, tpl = [], []
            for plain_ in (False, True):
                for _ in range(3):
                    plan8.apply(x8, pp, Y=Y8[:pp], plain=plain_)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(10):
                    plan8.apply(x8, pp, Y=Y8[:pp], plain=plain_)
                e1.record(stream)
                e1.synchronize()
                (tpl if plain_ else tb).append(e0.elapsed_time(e1) / 10 * 1e-3)
            plan8.check()
            f = 2.0 * nnz * pp
            sweep[str(pp)] = {"blocked_gflops": round(f / tb[0] / 1e9, 1), "plain_gflops": round(f / tpl[0] / 1e9, 1),
                              "speedup": round(tpl[0] / tb[0], 3)}
        out["p_sweep"] = sweep
        log("p sweep: " + ", ".join(f"p={k}: {v['speedup']}x" for k, v in sweep.items()))
        # p_opt (Sec. 3): the tuner times every admissible block size for 8 powers
        q_opt, t_opt = plan8.tune_block(x8, 8, Y=Y8)
        plan8.set_block(0)
        out["p_opt"] = {"p": 8, "q_opt": q_opt, "us_per_call": round(t_opt * 1e6, 1),
                        "note": "mpk_tune_block over q = 1..min(8, deadlock bound) on the same plan"}
        log(f"p_opt: q = {q_opt} for 8 powers ({t_opt * 1e6:.1f} us per call)")
        del plan8, Y8
    if args.only == "both" and not args.no_sweep:
        # Jacobi-preconditioned MPK (A P^{-1})^j x, j = 1..p, with k Jacobi sweeps: the plan
        # holds A D^{-1}; blocked against plain launches on the same layout
        planj = Plan.from_csr(A, p_block=8, column_scaling="jacobi").upload(dev)
        xj = planj.permute(torch.tensor(x, device=dev), 0)
        Yj = torch.empty((p, n), dtype=torch.float64, device=dev)
        jac = {}
        for k in (1, 2, 4):
            t = {}
            for plain_ in (False, True):
                for _ in range(3):
                    planj.jacobi_apply(xj, p, k, Y=Yj, plain=plain_)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(10):
                    planj.jacobi_apply(xj, p, k, Y=Yj, plain=plain_)
                e1.record(stream)
                e1.synchronize()
                t[plain_] = e0.elapsed_time(e1) / 10 * 1e-3
            planj.check()
            f = 2.0 * nnz * p * k
            jac[f"k={k}"] = {"blocked_us": round(t[False] * 1e6, 1), "plain_us": round(t[True] * 1e6, 1),
                             "blocked_gflops": round(f / t[False] / 1e9, 1), "speedup": round(t[True] / t[False], 3),
                             "sub_powers": p * k}
        # GS2-preconditioned MPK: gamma + 2 sub-powers per power (D^-1, gamma sweeps with L, A)
        plang = Plan.from_csr(A, p_block=8, split_lower=True).upload(dev)
        xg = plang.permute(torch.tensor(x, device=dev), 0)
        gs2 = {}
        for gam in (1, 2):
            t = {}
            for plain_ in (False, True):
                for _ in range(3):
                    plang.gs2_apply(xg, p, gam, Y=Yj, plain=plain_)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(10):
                    plang.gs2_apply(xg, p, gam, Y=Yj, plain=plain_)
                e1.record(stream)
                e1.synchronize()
                t[plain_] = e0.elapsed_time(e1) / 10 * 1e-3
            plang.check()
            gs2[f"gamma={gam}"] = {"blocked_us": round(t[False] * 1e6, 1), "plain_us": round(t[True] * 1e6, 1),
                                   "speedup": round(t[True] / t[False], 3), "sub_powers": p * (gam + 2)}
        out["gs2_mpk"] = {"workload": f"(A P^-1)^j x, j = 1..{p}, P^-1 = one GS2 iteration from zero with gamma "
                                      f"inner sweeps, 3D 7-point Laplacian {g}^3, blocks of up to 8 sub-powers",
                          **gs2}
        log("gs2: " + ", ".join(f"{kk}: {v['blocked_us']} us blocked, {v['speedup']}x" for kk, v in gs2.items()))
        # AMG pre-smoothing fused with the residual (Sec. 5.3): nu outer GS2 sweeps on
        # A x = b, then r = b - A x, as one chain of nu (gamma + 1) + 1 sub-powers; x carries
        # over from call to call (the work per call does not depend on its values)
        bg = plang.permute(torch.tensor(synth.uniform_vector(n, 1), device=dev), 0)
        xs = torch.zeros_like(bg)
        rs = torch.empty_like(bg)
        sm = {}
        for nu, gam in ((2, 1), (3, 1), (2, 2)):
            t = {}
            for plain_ in (False, True):
                for _ in range(3):
                    plang.gs2_smooth(bg, xs, nu, gam, r=rs, plain=plain_)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(10):
                    plang.gs2_smooth(bg, xs, nu, gam, r=rs, plain=plain_)
                e1.record(stream)
                e1.synchronize()
                t[plain_] = e0.elapsed_time(e1) / 10 * 1e-3
            plang.check()
            sm[f"sweeps={nu},gamma={gam}"] = {"blocked_us": round(t[False] * 1e6, 1), "plain_us": round(t[True] * 1e6, 1),
                                              "speedup": round(t[True] / t[False], 3),
                                              "sub_powers": nu * (gam + 1) + 1}
        out["gs2_smoother_residual"] = {
            "workload": f"AMG pre-smoother fused with the residual: sweeps outer GS2 iterations (gamma inner) on "
                        f"A x = b, then r = b - A x, 3D 7-point Laplacian {g}^3, blocks of up to 8 sub-powers "
                        f"(q = {plang.block_powers('gs2_smooth')})", **sm}
        log("smoother: " + ", ".join(f"{kk}: {v['blocked_us']} us blocked, {v['speedup']}x" for kk, v in sm.items()))
        del plang, bg, xs, rs
        out["jacobi_mpk"] = {"workload": f"(A P^-1)^j x, j = 1..{p}, P^-1 = k Jacobi sweeps from zero, "
                                         f"3D 7-point Laplacian {g}^3, plan of A D^-1 with blocks of up to 8",
                             **jac}
        log("jacobi: " + ", ".join(f"{kk}: {v['blocked_us']} us blocked, {v['speedup']}x" for kk, v in jac.items()))
        del planj, Yj
    for vals in ([] if args.no_f32 or args.only != "both" else ["f32", "bf16"]):
        # reduced-precision storage of the matrix values (vectors, products and sums stay FP64),
        # chunks per wave chosen by the planner as for FP64 values
        plan_r = Plan.from_csr(A, p_block=args.p_block or min(p, 15),
                               chunks_per_worker=args.chunks_per_worker, values=vals).upload(dev)
        xd_r = plan_r.permute(torch.tensor(x, device=dev), 0)
        Y_r = torch.empty_like(Y)
        wb_r, _ = timed(False, plan_r, xd_r, Y_r)
        wp_r, _ = timed(True, plan_r, xd_r, Y_r)
        plan.apply(xd, p, Y=Y)
        plan_r.apply(xd_r, p, Y=Y_r)
        torch.cuda.synchronize()
        err = ((Y_r - Y).norm(dim=1) / Y.norm(dim=1)).cpu().numpy()
        vbytes = {"f32": 4, "bf16": 2}[vals]
        out[f"{vals}_values"] = {
            "blocked_gflops": round(flops * args.steps / wb_r / 1e9, 2),
            "plain_gflops": round(flops * args.steps / wp_r / 1e9, 2),
            "ms_per_step": round(wb_r / args.steps * 1e3, 5),
            "speedup_vs_plain": round(wp_r / wb_r, 3),
            "speedup_vs_f64_blocked": round(wall / wb_r, 3) if key == "blocked" else None,
            "chunks_per_worker": plan_r.block_shape("powers")[1],
            "bytes_per_launch": int(bytes_per_launch - (8 - vbytes) * nnz / launches_per_step
                                    + (4 * n if vals == "bf16" else 0) / launches_per_step),
            "max_rel_err_vs_f64_per_power": float(err.max()),
            "note": {"f32": "matrix values rounded once to FP32 at upload; vectors, products and sums "
                            "in FP64; the 7-point stencil's values are integers, so FP32 storage is exact",
                     "bf16": "a_ij ~ s_i q_ij with s_i = fl32(max_j |a_ij|) per row and q_ij in BF16 "
                             "(nearest, ties to even); s_i q_ij is exact in FP64; the stencil's -1/6 "
                             "is not a BF16 value, so the powers carry the stated error"}[vals],
        }
        log(f"{vals} values: blocked {wb_r / args.steps * 1e6:.1f} us/step, plain {wp_r / args.steps * 1e6:.1f} "
            f"us/step, max rel err vs FP64 {err.max():.2e}")
        del plan_r, Y_r
    out["solve_latency_ms"] = {"p50": None, "p99": None, "note": "not measured"}
    if not args.no_solve and args.only == "both":
        # A x = b to 1e-10 by FP64 iterative refinement around a Chebyshev polynomial
        # preconditioner on the exact spectrum bounds of the Dirichlet stencil
        cg = np.cos(np.pi / (g + 1))
        lmin, lmax = 3 * (2 - 2 * cg), 3 * (2 + 2 * cg)
        bvec = plan.permute(torch.tensor(synth.uniform_vector(n, 1), device=dev), 0)
        d = args.solve_degree

        def solves(lo, plain):
            lat, res = [], None
            for r in range(args.solve_reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = plan.refine_solve(lo, bvec, d, lmin, lmax, tol=1e-10, max_iter=2000, plain=plain)
                torch.cuda.synchronize()
                if r > 0:  # first solve is a warm-up
                    lat.append(time.perf_counter() - t0)
            lat = np.array(lat) * 1e3
            return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat, 99)), 3),
                    "corrections": res[1], "final_rel_residual": res[2],
                    "powers_per_solve": res[1] * (d - 1)}
        # corrections with FP32 (or BF16) values and two chunks per wave (the polynomial
        # kernel needs the registers that four chunks would take)
        # (BF16 corrections are not used here: their perturbation of the spectrum, about
        # 2^-8 of |A|, dwarfs lambda_min = 0.0011, and refinement barely contracts)
        plan_lo = Plan.from_csr(A, p_block=args.p_block or min(p, 15), values="f32").upload(dev)
        mixed = solves(plan_lo, False)
        del plan_lo
        fp64_plain = solves(plan, True)
        out["solve"] = {
            "workload": f"A x = b, 3D 7-point Laplacian {g}^3, b uniform[-1,1] seed 1 (level order), x0 = 0, "
                        f"tol 1e-10 relative residual; FP64 iterative refinement around a degree-{d} Chebyshev "
                        f"polynomial preconditioner on [{lmin:.6g}, {lmax:.6g}] (the exact spectrum bounds)",
            "mixed_f32_blocked": mixed,
            "fp64_plain": fp64_plain,
            "speedup_p50": round(fp64_plain["p50_ms"] / mixed["p50_ms"], 3),
            "note": f"{args.solve_reps} sequential solves of one system after one warm-up (no serving or batching)",
        }
        out["solve_latency_ms"] = {"p50": mixed["p50_ms"], "p99": mixed["p99_ms"],
                                   "note": "sequential mixed-precision solves of one system (replaced by the "
                                           "served solves' latency when the serving leg runs)"}
        log(f"solve: mixed {mixed['p50_ms']:.1f} ms p50 ({mixed['corrections']} corrections), fp64 plain "
            f"{fp64_plain['p50_ms']:.1f} ms p50")
    if not args.no_solve and args.only == "both":
        # the same system by s-step GMRES (blocks of s, restart m) with the right
        # degree-d Chebyshev polynomial preconditioner: FP64 residuals and orthogonalisation;
        # basis and preconditioner through FP32-valued blocked launches (mixed), or FP64
        # values with plain SpMV launches (the FP64 plain path)
        gs, gm, gd = args.gmres_s, args.gmres_m, args.gmres_degree
        cg = np.cos(np.pi / (g + 1))
        lmin, lmax = 3 * (2 - 2 * cg), 3 * (2 + 2 * cg)
        bvec = plan.permute(torch.tensor(synth.uniform_vector(n, 1), device=dev), 0)
        hi8 = Plan.from_csr(A, p_block=8).upload(dev)
        lo8 = Plan.from_csr(A, p_block=8, values="f32").upload(dev)
        work = torch.empty(lo8.gmres_work_bytes(gs, gm, gd) // 8 + 64, dtype=torch.float64, device=dev)

        def gmres_solves(lo, plain):
            lat, res = [], None
            for r in range(args.solve_reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = hi8.sstep_gmres(lo, bvec, gs, gm, gd, lmin, lmax, tol=1e-10, max_cycles=200, plain=plain,
                                      work=work)
                torch.cuda.synchronize()
                if r > 0:
                    lat.append(time.perf_counter() - t0)
            lo.check()
            xs = res[0]
            # true residual of the returned solution, FP64 SpMV on the GPU
            true = float(torch.linalg.norm(bvec - hi8.apply(xs, 1)[0]) / torch.linalg.norm(bvec))
            lat = np.array(lat) * 1e3
            return {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat, 99)), 3),
                    "basis_vectors": res[1], "cycles": res[2], "final_rel_residual": res[3],
                    "true_rel_residual": true, "powers_per_solve": res[1] * gd + res[2] * (gd - 1) + res[2] + 1}
        gm_mixed = gmres_solves(lo8, False)
        gm_plain = gmres_solves(hi8, True)
        out["solve_gmres"] = {
            "workload": f"A x = b, 3D 7-point Laplacian {g}^3, b uniform[-1,1] seed 1 (level order), x0 = 0, "
                        f"tol 1e-10 relative residual; s-step GMRES (s = {gs}, restart m = {gm}) with the right "
                        f"degree-{gd} Chebyshev polynomial preconditioner on [{lmin:.6g}, {lmax:.6g}]",
            "mixed_f32_blocked": gm_mixed,
            "fp64_plain": gm_plain,
            "speedup_p50": round(gm_plain["p50_ms"] / gm_mixed["p50_ms"], 3),
            "note": f"{args.solve_reps} sequential solves of one system after one warm-up",
        }
        log(f"gmres: mixed {gm_mixed['p50_ms']:.1f} ms p50 ({gm_mixed['basis_vectors']} vectors, "
            f"{gm_mixed['cycles']} cycles, true residual {gm_mixed['true_rel_residual']:.2e}), fp64 plain "
            f"{gm_plain['p50_ms']:.1f} ms p50")
        # s-step GMRES as in the paper's s-step experiments: a fixed amount of work (two
        # cycles of m = 64, s = 8, FP64) with each block's basis from one MPK of 8 powers,
        # blocked against plain launches; time per 1000 basis vectors
        fixed = {}
        jac8 = Plan.from_csr(A, p_block=8, column_scaling="jacobi").upload(dev)
        gs8 = Plan.from_csr(A, p_block=8, split_lower=True).upload(dev)
        gwork = torch.empty(gs8.gmres_work_bytes(8, 64, 1) // 8 + 64, dtype=torch.float64, device=dev)
        for name, lo_, lmin_, lmax_, deg_, wk_ in (("none", hi8, lmin, lmax, 1, work),
                                                    ("jacobi", jac8, lmin / 6, lmax / 6, 1, work),
                                                    ("gs2", gs8, 0.002, 2.0, 1, gwork)):
            t = {}
            for plain_ in (False, True):
                hi8.sstep_gmres(lo_, bvec, 8, 64, deg_, lmin_, lmax_, tol=0.0, max_cycles=2, plain=plain_, work=wk_,
                                precond=name)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    res = hi8.sstep_gmres(lo_, bvec, 8, 64, deg_, lmin_, lmax_, tol=0.0, max_cycles=2, plain=plain_,
                                          work=wk_, precond=name)
                torch.cuda.synchronize()
                t[plain_] = (time.perf_counter() - t0) / 3 / res[1] * 1e3 * 1e3  # ms per 1000 vectors
            fixed[name] = {"blocked_ms_per_1000_vectors": round(t[False], 2),
                           "plain_ms_per_1000_vectors": round(t[True], 2), "speedup": round(t[True] / t[False], 3)}
        jac8.check()
        out["sstep_gmres_fixed_work"] = {
            "workload": f"s-step GMRES on the 3D 7-point Laplacian {g}^3, s = 8, m = 64, two cycles (128 basis "
                        "vectors), FP64; without a preconditioner, with the fused Jacobi A D^-1, and with GS2 "
                        "(gamma = 1: 3 sub-powers per basis vector); each block's basis is one blocked chain of "
                        "8 powers or one launch per (sub-)power (plain)", **fixed}
        log("s-step gmres: " + ", ".join(f"{k2}: {v['blocked_ms_per_1000_vectors']} ms/1000 vectors blocked, "
                                           f"{v['speedup']}x" for k2, v in fixed.items()))
        del hi8, lo8, work, jac8, gs8, gwork
    if not args.no_knn and args.only == "both":
        out["knn_8m"] = knn_bench(args, dev, stream)
    if not args.no_serve and args.only == "both":
        out["serving"] = serving_bench(args, A, plan, dev)
        sv = out["serving"]["by_kind"]["solve"]
        out["solve_latency_ms"] = {"p50": sv["p50_ms"], "p99": sv["p99_ms"],
                                   "note": "served s-step GMRES solves to 1e-8 in the mixed request stream "
                                           "(serving.workload), PCIe copies included"}
    if not args.no_cpu_baseline and args.only == "both":
        log("cpu baseline: FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(g, p)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
