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
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(A, x, p, budget_s):
    import numpy as np
    import oracle
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.mpk(A, x, p)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 20:
            break
    gf = 2.0 * A.col.size * p * reps / el / 1e9
    return {"value": round(gf, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"full 160^3 matrix, p={p}, {reps} complete MPK calls "
                      f"({el:.1f} s, single-threaded NumPy)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--grid", type=int, default=160)
    ap.add_argument("--p-block", type=int, default=0)
    ap.add_argument("--chunks-per-worker", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32 and BF16 matrix-value measurements")
    ap.add_argument("--no-solve", action="store_true", help="skip the refinement-solve latency measurement")
    ap.add_argument("--no-sweep", action="store_true", help="skip the p = 1..8 sweep")
    ap.add_argument("--solve-reps", type=int, default=10)
    ap.add_argument("--solve-degree", type=int, default=256)
    ap.add_argument("--only", choices=["both", "blocked", "plain"], default="both",
                    help="restrict the launches (for profiler runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (scales the HBM byte "
                         "counters of a profiler run) and exit")
    args = ap.parse_args()
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
            "chunks_per_worker": args.chunks_per_worker or None,
            "workers_per_xcd": info["workers_per_xcd"],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "mpk_block_kernel" if key == "blocked" else "spmv_kernel",
            "bytes_per_launch": int(bytes_per_launch),
            "avg_launch_us": round(avg_launch * 1e6, 2),
        },
        "plan_build_s": round(t_plan, 3),
        "plan_upload_s": round(t_upload, 3),
    }
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
    if "plain" in res and "blocked" in res:
        wp = res["plain"][0]
        out["plain_gflops"] = round(flops * args.steps / wp / 1e9, 2)
        out["speedup_vs_plain"] = round(wp / res["blocked"][0], 3)
        out["plan_build_spmv_equivalents"] = round(t_plan / (wp / args.steps / p), 1)
        out["roofline_equivalent_frac"] = round(value / (flops / (b_blk / (HBM_PEAK_GBS * 1e9)) / 1e9), 4)
    if args.only == "both":
        out["staged_wavefront"] = res_staged
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
        del plan8, Y8
    for vals in ([] if args.no_f32 or args.only != "both" else ["f32", "bf16"]):
        # reduced-precision storage of the matrix values (vectors, products and sums stay FP64)
        # with four chunks per wave: the narrow values leave registers for them (measured
        # faster than two for the power kernel)
        plan_r = Plan.from_csr(A, p_block=args.p_block or min(p, 15),
                               chunks_per_worker=args.chunks_per_worker or 4, values=vals).upload(dev)
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
            "chunks_per_worker": args.chunks_per_worker or 4,
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
                                   "note": "sequential mixed-precision solves of one system; the served "
                                           "(continuously batched) solve is not built"}
        log(f"solve: mixed {mixed['p50_ms']:.1f} ms p50 ({mixed['corrections']} corrections), fp64 plain "
            f"{fp64_plain['p50_ms']:.1f} ms p50")
    if not args.no_cpu_baseline and args.only == "both":
        log("cpu baseline: FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(A, x, p, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
