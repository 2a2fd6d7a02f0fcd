"""Host-side checks of the C ABI (no GPU): the library loads and exports every
declared entry point; the host planner's level sets and permutation are
bit-exact to the oracle (parity with the paper's Sec. 3 level structure); its
chunk partition, dependency lists and deadlock bound equal the test-side model
of the blocked kernel's work hand-out (a design cross-check, not parity);
malformed input is rejected with the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import schedule_model as SM
import synth as S
from paper_2309_02228_amd import mpk as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mpk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:mpk_status|void|const char\s*\*)\s*(\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    assert sorted(M.EXPORTS) == names
    lib = ctypes.CDLL(M.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert "gfx950" in M.version()


MATRICES = {
    "lap1d": lambda: S.laplacian_1d(300),
    "lap2d_64": lambda: S.laplacian_2d(64),
    "lap2d_ragged": lambda: S.laplacian_2d(37, 29),
    "lap3d": lambda: S.laplacian_3d(17, 13, 11),
    "rand_nonsym": lambda: S.random_pattern(3000, 3, 1),
    "rand_sparse_disconnected": lambda: S.random_pattern(2000, 0.8, 2),
    "rand_sym": lambda: S.random_pattern(1500, 5, 3, symmetric=True),
    "blocks": lambda: S.block_diagonal(S.laplacian_2d(9, 7), S.identity(70), S.laplacian_1d(130),
                                       S.random_pattern(200, 2, 9)),
    "knn": lambda: S.knn_graph_laplacian(3000, k=26, seed=1),
    "identity": lambda: S.identity(200),
    "shift": lambda: S.cyclic_shift(257),
    "single": lambda: S.from_dense([[2.0]]),
    "long_entry": lambda: S.from_dense(np.eye(130) + np.diag([0.0] * 129 + [0.0]) +
                                       np.pad(np.array([[0.0] * 129 + [4.0]]), ((0, 129), (0, 0)))),
}


def reference_plan(A, root=None, chunk_rows=64, parts=8):
    """Levels and permutation from the oracle; partition and dependency lists
    from the design model."""
    level, nl, roots = O.bfs_levels(A, root)
    perm, iperm, level_ptr = O.level_permutation(level, nl)
    B = O.permute_symmetric(A, perm, iperm)
    owner = SM.chunk_owner(level_ptr, level[perm], A.n, chunk_rows, parts)
    deps = SM.chunk_dependencies(B, chunk_rows)
    return dict(level=level, nl=nl, perm=perm, iperm=iperm, level_ptr=level_ptr, owner=owner, deps=deps)


@pytest.mark.parametrize("name", sorted(MATRICES))
def test_planner_levels_bit_exact_and_tables_match_design(name):
    A = MATRICES[name]()
    plan = M.Plan.from_csr(A, p_block=6)
    got = plan.levels()
    ref = reference_plan(A)
    assert got["nlevels"] == ref["nl"]
    assert np.array_equal(got["level_of_row"], ref["level"])
    assert np.array_equal(got["perm"], ref["perm"])
    assert np.array_equal(got["iperm"], ref["iperm"])
    assert np.array_equal(got["level_ptr"], ref["level_ptr"])
    # design cross-check: the hand-out tables equal the test-side model
    part = plan.partition()
    assert part["chunk_rows"] == 64 and part["nparts"] == 8
    assert np.array_equal(part["owner"], ref["owner"])
    ptr, idx = plan.deps()
    assert ptr.size == len(ref["deps"]) + 1
    for c, d in enumerate(ref["deps"]):
        assert np.array_equal(idx[ptr[c]:ptr[c + 1]], d), c
    # the deadlock bound is the smallest worker count meeting the model's condition
    G = 1 if plan.info()["reg_slots"] >= 32 else 2
    for q in range(1, 7):
        assert plan.min_workers(q) == SM.min_workers(ref["owner"], ref["deps"], G, q), q


@pytest.mark.parametrize("name", ["lap3d_52", "rand_nonsym_300k", "knn_150k"])
def test_planner_threaded_sizes_levels_bit_exact_and_tables_match_design(name):
    # large enough that the planner splits its table building over threads
    # (2 and 4 ranges) and, for the random and kNN patterns, searches BFS
    # layers of more than 4096 rows with a team of threads: the tables must
    # not depend on either
    A = {"lap3d_52": lambda: S.laplacian_3d(52),
         "rand_nonsym_300k": lambda: S.random_pattern(300000, 2.5, 5),
         "knn_150k": lambda: S.knn_graph_laplacian(150000, k=26, seed=3)}[name]()
    assert A.n >= 2 << 16
    plan = M.Plan.from_csr(A, p_block=4)
    got = plan.levels()
    ref = reference_plan(A)
    assert got["nlevels"] == ref["nl"]
    assert np.array_equal(got["level_of_row"], ref["level"])
    assert np.array_equal(got["perm"], ref["perm"])
    assert np.array_equal(got["level_ptr"], ref["level_ptr"])
    if name != "lap3d_52":
        assert np.bincount(ref["level"]).max() > 4096
    assert np.array_equal(plan.partition()["owner"], ref["owner"])
    ptr, idx = plan.deps()
    assert ptr.size == len(ref["deps"]) + 1
    assert np.array_equal(idx, np.concatenate([np.asarray(d, dtype=idx.dtype) for d in ref["deps"]]))


@pytest.mark.parametrize("G", [1, 2, 4])
def test_planner_unit_bound_by_group(G):
    A = S.laplacian_3d(14, 12, 10)
    plan = M.Plan.from_csr(A, p_block=5, chunks_per_worker=G)
    ref = reference_plan(A)
    for q in range(1, 6):
        assert plan.min_workers(q) == SM.min_workers(ref["owner"], ref["deps"], G, q)


@pytest.mark.parametrize("values", ["f64", "f32", "bf16"])
def test_planner_wide_units(values):
    # plans whose group is left to the planner, on rows of at most 8 slots, also hold
    # units of 3, 5 and 6 chunks; their deadlock bounds are the model's for those sizes
    A = S.laplacian_3d(14, 12, 10)
    ref = reference_plan(A)
    plan = M.Plan.from_csr(A, p_block=5, values=values)
    assert plan.info()["reg_slots"] == 7
    for q in range(1, 6):
        for g in (3, 5, 6):
            assert plan.min_workers(q, g) == SM.min_workers(ref["owner"], ref["deps"], g, q)
        assert plan.min_workers(q, 2) == plan.min_workers(q)
    # none for an explicit group or wide rows
    for p in (M.Plan.from_csr(A, p_block=5, chunks_per_worker=2, values=values),
              M.Plan.from_csr(S.knn_graph_laplacian(3000, k=12, seed=1), p_block=5, values=values)):
        for g in (3, 5, 6):
            with pytest.raises(M.MPKError, match=f"no units of {g}"):
                p.min_workers(2, g)
    with pytest.raises(M.MPKError, match="no units of 0"):
        plan.min_workers(2, 0)


def test_planner_explicit_root():
    A = S.laplacian_2d(40, 33)
    plan = M.Plan.from_csr(A, root=700)
    got = plan.levels()
    ref = reference_plan(A, root=700)
    assert np.array_equal(got["level_of_row"], ref["level"])
    assert np.array_equal(got["perm"], ref["perm"])


def test_planner_info_and_layout():
    A = S.laplacian_3d(20)
    plan = M.Plan.from_csr(A)
    info = plan.info()
    assert info["n"] == 8000 and info["nnz"] == A.col.size
    assert info["nlevels"] == 58 and info["nchunks"] == 125
    assert info["reg_slots"] == 7 and info["p_block"] == 4  # widest row: 7 entries
    # SELL-64 pads each chunk to its widest row: at most 64 * 7 slots per chunk
    assert A.col.size <= info["sell_slots"] <= 125 * 64 * 7
    assert plan.device_bytes > info["sell_slots"] * 12


def test_work_bytes():
    plan = M.Plan.from_csr(S.laplacian_2d(10))
    assert plan.work_bytes(M.CALL_APPLY, 4, M.MPK_IO_PERMUTED) == 0
    assert plan.work_bytes(M.CALL_APPLY, 4, 0) == 100 * 8 * 5
    assert plan.work_bytes(M.CALL_POLY, 8, M.MPK_IO_PERMUTED) == 100 * 8 * (4 + 2)  # ring of p_block + 2
    assert plan.work_bytes(M.CALL_POLY, 8, 0) == 100 * 8 * (4 + 2 + 2)
    assert plan.work_bytes(M.CALL_SOLVE, 8, M.MPK_IO_PERMUTED) == 100 * 8 * (2 + 6) + 8 * (2048 + 8)
    assert plan.work_bytes(M.CALL_SSTEP, 3, 0) == 100 * 8 * 4


def _build(n, rowptr, col, val, **opt):
    o = M.Options()
    for k, v in opt.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    nb = ctypes.c_size_t()
    rp = np.ascontiguousarray(rowptr, np.int32)
    c = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    lib = M.lib()
    code = lib.mpk_build_levels(n, rp.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p),
                                v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o), ctypes.byref(h),
                                ctypes.byref(nb))
    if code == 0:
        lib.mpk_destroy(h)
    return code, lib.mpk_last_error().decode()


def test_malformed_csr_rejected():
    ok = _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0, 1.0, 1.0])
    assert ok[0] == 0
    assert _build(3, [0, 2, 1, 3], [0, 1, 2], [1.0] * 3)[0] == -2          # rowptr not monotone
    assert _build(3, [1, 2, 3, 3], [0, 1, 2], [1.0] * 3)[0] == -2          # rowptr[0] != 0
    assert _build(3, [0, 1, 2, 3], [0, 3, 2], [1.0] * 3)[0] == -2          # column out of range
    assert _build(3, [0, 1, 2, 3], [0, -1, 2], [1.0] * 3)[0] == -2         # negative column
    code, msg = _build(2, [0, 2, 3], [1, 0, 1], [1.0] * 3)                  # unsorted
    assert code == -2 and "ascending" in msg
    assert _build(2, [0, 2, 3], [1, 1, 1], [1.0] * 3)[0] == -2             # duplicate
    assert _build(-1, [0], [], [])[0] == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, p_block=16)[0] == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, root_mode=1, root=3)[0] == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, root_mode=2)[0] == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, chunks_per_worker=3)[0] == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, value_type=3)[0] == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, value_type=2)[0] == 0
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, value_type=1)[0] == 0
    assert _build(0, [0], [], [])[0] == 0                                  # empty matrix


def test_malformed_csr_reports_the_first_bad_row_at_threaded_sizes():
    # the check runs over row ranges in threads; the message names the first
    # offending row, as a row-by-row scan would
    n = 300000
    rowptr = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    col[150000] = n          # out of range
    col[290000] = -1         # later, in another range
    code, msg = _build(n, rowptr, col, np.ones(n))
    assert code == -2 and "row 150000" in msg and "out of range" in msg
    rp = rowptr.copy()
    rp[200001] = rp[200000] - 1  # pointer decreases at row 200000, after the bad column
    code, msg = _build(n, rp, col, np.ones(n))
    assert code == -2 and "row 150000" in msg
    col[150000] = 150000
    code, msg = _build(n, rp, col, np.ones(n))
    assert code == -2 and "rowptr decreases at row 200000" in msg


def test_apply_argument_errors_without_gpu():
    lib = M.lib()
    plan = M.Plan.from_csr(S.laplacian_2d(8))
    dummy = ctypes.c_void_p(0x1000)
    assert lib.mpk_apply(plan._h, dummy, dummy, 64, 0, 1, None, 0, None) == -1   # p = 0
    assert lib.mpk_apply(plan._h, dummy, dummy, 63, 2, 1, None, 0, None) == -1   # ldy < n
    assert lib.mpk_apply(plan._h, dummy, dummy, 64, 2, 0, None, 0, None) == -1   # no work buffer
    assert lib.mpk_apply(plan._h, dummy, dummy, 64, 2, 1, None, 0, None) == -6   # not uploaded
    c = np.ones(3)
    assert lib.poly_apply(plan._h, 7, 2, c.ctypes.data_as(ctypes.c_void_p), None, dummy,
                          ctypes.c_void_p(0x2000), 1, dummy, 1 << 20, None) == -1  # unknown kind
    assert lib.poly_apply(plan._h, 0, -1, c.ctypes.data_as(ctypes.c_void_p), None, dummy,
                          ctypes.c_void_p(0x2000), 1, dummy, 1 << 20, None) == -1  # d < 0
    prm = np.array([1.0, 0.0])
    assert lib.poly_apply(plan._h, 2, 2, c.ctypes.data_as(ctypes.c_void_p),
                          prm.ctypes.data_as(ctypes.c_void_p), dummy, ctypes.c_void_p(0x2000), 1,
                          dummy, 1 << 20, None) == -1  # delta == 0
    lam = np.zeros(2)
    sig = np.array([1.0, 0.0])
    assert lib.sstep_basis(plan._h, 2, lam.ctypes.data_as(ctypes.c_void_p),
                           sig.ctypes.data_as(ctypes.c_void_p), dummy, dummy, 64, 1, None, 0,
                           None) == -1  # zero sigma
    assert lib.sstep_basis(plan._h, 0, lam.ctypes.data_as(ctypes.c_void_p), None, dummy, dummy,
                           64, 1, None, 0, None) == -1  # s = 0
    assert lib.mpk_check_device(plan._h, None) == -6


def test_one_hip_runtime_per_process():
    """Importing the package before torch must not map a second HIP or HSA runtime."""
    import subprocess
    import sys
    code = ("import paper_2309_02228_amd, torch\n"
            "maps = {l.split()[-1] for l in open('/proc/self/maps')}\n"
            "print(sum('libamdhip64' in m for m in maps), sum('libhsa-runtime64' in m for m in maps))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300, check=True).stdout.split()
    assert out == ["1", "1"], out


def test_f32_values_shrink_the_device_buffer():
    A = S.laplacian_3d(20)
    p64 = M.Plan.from_csr(A)
    p32 = M.Plan.from_csr(A, values="f32")
    slots = p64.info()["sell_slots"]
    assert p32.info()["values"] == "f32" and p64.info()["values"] == "f64"
    assert p64.device_bytes - p32.device_bytes >= 4 * slots - 512  # 4 bytes per slot, alignment aside
    with pytest.raises(ValueError):
        M.Plan.from_csr(A, values="f16")
    p16 = M.Plan.from_csr(A, values="bf16")  # 2 bytes per slot plus a 4-byte scale per row
    assert p32.device_bytes - p16.device_bytes >= 2 * slots - 4 * 64 * p16.info()["nchunks"] - 1024


@pytest.mark.parametrize("name", ["lap3d", "rand_nonsym", "blocks", "knn", "lap1d", "single"])
@pytest.mark.parametrize("cache_mib,q,floor,values", [(1, 4, 0, "f64"), (1, 2, 5000, "f64"), (2, 7, 0, "f32"),
                                                      (1, 3, 0, "bf16"),
                                                      (256, 4, 0, "f64"), (1, 15, 0, "f64")])
def test_planner_schedule_bit_exact_to_oracle(name, cache_mib, q, floor, values):
    A = MATRICES[name]()
    plan = M.Plan.from_csr(A, cache_mib=cache_mib, min_group_rows=floor, values=values)
    ng, tasks = plan.schedule(q)
    level, nl, _ = O.bfs_levels(A)
    perm, iperm, lp = O.level_permutation(level, nl)
    gp = O.group_levels(A, lp, perm, cache_mib << 20, q, value_bytes={"f64": 8, "f32": 4, "bf16": 2}[values],
                        min_group_rows=floor)
    assert ng == len(gp) - 1
    want = [(s, k, lp[lo], lp[hi + 1]) for s, k, lo, hi in O.wavefront_schedule(gp, q)]
    assert [tuple(int(v) for v in t) for t in tasks] == [tuple(int(v) for v in t) for t in want]


def test_schedule_argument_errors():
    plan = M.Plan.from_csr(S.laplacian_2d(8))
    lib = M.lib()
    nt, ng = ctypes.c_int32(), ctypes.c_int32()
    assert lib.mpk_get_schedule(plan._h, 0, ctypes.byref(nt), ctypes.byref(ng), None) == -1
    assert lib.mpk_get_schedule(plan._h, 16, ctypes.byref(nt), ctypes.byref(ng), None) == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, cache_mib=-1)[0] == -1
    assert _build(3, [0, 1, 2, 3], [0, 1, 2], [1.0] * 3, min_group_rows=-2)[0] == -1


def test_server_argument_errors_without_gpu():
    lib = M.lib()
    h = ctypes.c_void_p()
    assert lib.mpk_server_create(0, 1 << 20, ctypes.byref(h)) == -1       # no workers
    assert lib.mpk_server_create(65, 1 << 20, ctypes.byref(h)) == -1      # too many workers
    assert lib.mpk_server_create(2, 16, ctypes.byref(h)) == -1            # pool below one alignment unit
    assert lib.mpk_server_create(2, 1 << 20, None) == -1
    plan = M.Plan.from_csr(S.laplacian_2d(8))
    x = np.ones(64)
    t = ctypes.c_int64()
    assert lib.mpk_server_submit_apply(None, plan._h, M._ptr(x), 2, M._ptr(x), 1, ctypes.byref(t)) == -1
    assert lib.mpk_server_submit_solve(None, plan._h, plan._h, M._ptr(x), M._ptr(x), 4, 0.1, 8.0, 1e-10, 10,
                                       1, ctypes.byref(t)) == -1
    assert lib.mpk_server_wait(None, 1, None, None, None, None, None) == -1
    lib.mpk_server_destroy(None)  # no-op


def test_sstep_gmres_argument_errors_without_gpu():
    lib = M.lib()
    A = S.laplacian_2d(8)
    hi = M.Plan.from_csr(A)
    lo = M.Plan.from_csr(A, values="f32")
    other = M.Plan.from_csr(S.laplacian_2d(9))
    nb = ctypes.c_size_t()
    assert lib.mpk_sstep_gmres_work_bytes(hi._h, 8, 32, 8, 1, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.mpk_sstep_gmres_work_bytes(hi._h, 0, 32, 8, 1, ctypes.byref(nb)) == -1   # s < 1
    assert lib.mpk_sstep_gmres_work_bytes(hi._h, 17, 32, 8, 1, ctypes.byref(nb)) == -1  # s > 16
    assert lib.mpk_sstep_gmres_work_bytes(hi._h, 8, 4, 8, 1, ctypes.byref(nb)) == -1    # m < s
    assert lib.mpk_sstep_gmres_work_bytes(hi._h, 8, 257, 8, 1, ctypes.byref(nb)) == -1  # m > 256
    assert lib.mpk_sstep_gmres_work_bytes(hi._h, 8, 32, -1, 1, ctypes.byref(nb)) == -1  # d < 0 (0 is gamma = 0 of GS2)
    need = nb.value
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails first

    def call(h=hi, l=lo, s=8, m=32, d=8, lmin=0.1, lmax=8.0, b=fake, x=fake, tol=1e-10, cyc=10, flags=1,
             work=fake, nbytes=None):
        return lib.mpk_sstep_gmres(h._h if h else None, l._h if l else None, s, m, d, lmin, lmax, b, x, tol, cyc,
                                   flags, work, need if nbytes is None else nbytes, None, None, None, None)

    assert call(h=None) == -1
    assert call(h=lo, l=lo) == -1                  # hi must hold FP64 values
    assert call(l=other) == -1                     # plans of different matrices
    assert call(s=0) == -1 and call(m=7) == -1 and call(d=0) == -1
    assert call(lmin=0.0) == -1 and call(lmin=2.0, lmax=1.0) == -1
    assert call(tol=-1.0) == -1 and call(cyc=-1) == -1
    assert call(flags=64) == -1                    # unknown flag bit
    assert call(b=None) == -1 and call(x=None) == -1
    assert call(nbytes=need - 1) == -1             # work too small
    assert call(work=ctypes.c_void_p((1 << 20) + 8)) == -1  # misaligned
    assert call() == -6                            # not uploaded
    assert "upload" in lib.mpk_last_error().decode()


def test_jacobi_scaling_and_apply_argument_errors_without_gpu():
    lib = M.lib()
    # a row without a stored (or with a zero) diagonal entry is refused for column scaling
    with pytest.raises(M.MPKError, match="MPK_ERR_CSR"):
        M.Plan.from_csr(S.cyclic_shift(6), column_scaling="jacobi")
    with pytest.raises(M.MPKError, match="MPK_ERR_CSR"):
        M.Plan.from_csr(S.from_dense(np.array([[0.0, 1.0], [1.0, 2.0]]), keep_zeros=True),
                        column_scaling="jacobi")
    with pytest.raises(ValueError):
        M.Plan.from_csr(S.laplacian_2d(4), column_scaling="gs2")
    A = S.laplacian_2d(8)
    plain = M.Plan.from_csr(A)
    jac = M.Plan.from_csr(A, column_scaling="jacobi")
    # the level structure does not depend on the values
    assert np.array_equal(plain.levels()["perm"], jac.levels()["perm"])
    nb = ctypes.c_size_t()
    assert lib.mpk_jacobi_work_bytes(jac._h, 1, 4, 1, ctypes.byref(nb)) == 0
    assert lib.mpk_jacobi_work_bytes(jac._h, 0, 4, 1, ctypes.byref(nb)) == -1
    assert lib.mpk_jacobi_work_bytes(jac._h, 65, 4, 1, ctypes.byref(nb)) == -1
    assert lib.mpk_jacobi_work_bytes(jac._h, 2, 0, 1, ctypes.byref(nb)) == -1
    fake = ctypes.c_void_p(1 << 20)
    assert lib.mpk_jacobi_apply(plain._h, 1, fake, fake, 64, 2, 1, None, 0, None) == -1  # not scaled
    assert lib.mpk_jacobi_apply(jac._h, 0, fake, fake, 64, 2, 1, None, 0, None) == -1    # k < 1
    assert lib.mpk_jacobi_apply(jac._h, 2, fake, fake, 64, 0, 1, None, 0, None) == -1    # p < 1
    assert lib.mpk_jacobi_apply(jac._h, 2, fake, fake, 63, 2, 1, None, 0, None) == -1    # ldy < n
    assert lib.mpk_jacobi_apply(jac._h, 2, None, fake, 64, 2, 1, None, 0, None) == -1    # null x
    assert lib.mpk_jacobi_apply(jac._h, 2, fake, fake, 64, 2, 1, None, 0, None) == -1    # no ring work
    assert lib.mpk_jacobi_apply(jac._h, 1, fake, fake, 64, 2, 1, None, 0, None) == -6    # not uploaded
    opt = M.Options()
    lib.mpk_options_default(ctypes.byref(opt))
    opt.column_scaling = 2
    h, nbytes = ctypes.c_void_p(), ctypes.c_size_t()
    rp, c, v = (np.ascontiguousarray(a) for a in (A.rowptr, A.col, A.val))
    assert lib.mpk_build_levels(A.n, M._ptr(rp), M._ptr(c), M._ptr(v), ctypes.byref(opt), ctypes.byref(h),
                                ctypes.byref(nbytes)) == -1


def test_gs2_split_plan_and_apply_argument_errors_without_gpu():
    lib = M.lib()
    with pytest.raises(M.MPKError, match="MPK_ERR_CSR"):
        M.Plan.from_csr(S.cyclic_shift(6), split_lower=True)          # no diagonal
    wide = S.from_dense(np.ones((40, 40)))                             # 40 entries per row
    with pytest.raises(M.MPKError, match="MPK_ERR_UNSUPPORTED"):
        M.Plan.from_csr(wide, split_lower=True)
    A = S.laplacian_2d(8)
    plain = M.Plan.from_csr(A)
    split = M.Plan.from_csr(A, split_lower=True)
    assert np.array_equal(plain.levels()["perm"], split.levels()["perm"])
    nb = ctypes.c_size_t()
    assert lib.mpk_gs2_work_bytes(split._h, 2, 4, 1, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.mpk_gs2_work_bytes(split._h, -1, 4, 1, ctypes.byref(nb)) == -1
    assert lib.mpk_gs2_work_bytes(split._h, 17, 4, 1, ctypes.byref(nb)) == -1
    assert lib.mpk_gs2_work_bytes(split._h, 2, 0, 1, ctypes.byref(nb)) == -1
    need = nb.value
    fake = ctypes.c_void_p(1 << 20)
    assert lib.mpk_gs2_apply(plain._h, 1, fake, fake, 64, 2, 1, fake, need, None) == -1   # not split
    assert lib.mpk_gs2_apply(split._h, 17, fake, fake, 64, 2, 1, fake, need, None) == -1  # gamma
    assert lib.mpk_gs2_apply(split._h, 1, fake, fake, 63, 2, 1, fake, need, None) == -1   # ldy < n
    assert lib.mpk_gs2_apply(split._h, 1, None, fake, 64, 2, 1, fake, need, None) == -1   # null x
    assert lib.mpk_gs2_apply(split._h, 1, fake, fake, 64, 2, 64, fake, need, None) == -1  # flag bit
    assert lib.mpk_gs2_apply(split._h, 2, fake, fake, 64, 4, 1, fake, need - 8, None) == -1  # work
    assert lib.mpk_gs2_apply(split._h, 2, fake, fake, 64, 4, 1, ctypes.c_void_p((1 << 20) + 8), need,
                             None) == -1                                                  # misaligned
    assert lib.mpk_gs2_apply(split._h, 2, fake, fake, 64, 4, 1, fake, need, None) == -6    # not uploaded


def test_gs2_smooth_argument_errors_without_gpu():
    lib = M.lib()
    A = S.laplacian_2d(8)
    plain = M.Plan.from_csr(A)
    split = M.Plan.from_csr(A, split_lower=True)
    nb = ctypes.c_size_t()
    assert lib.mpk_gs2_smooth_work_bytes(split._h, 2, 1, ctypes.byref(nb)) == 0 and nb.value > 0
    need_perm = nb.value
    assert lib.mpk_gs2_smooth_work_bytes(split._h, 2, 0, ctypes.byref(nb)) == 0 and nb.value > need_perm
    assert lib.mpk_gs2_smooth_work_bytes(split._h, -1, 1, ctypes.byref(nb)) == -1
    assert lib.mpk_gs2_smooth_work_bytes(split._h, 17, 1, ctypes.byref(nb)) == -1
    need = need_perm
    fake = ctypes.c_void_p(1 << 20)
    assert lib.mpk_gs2_smooth(plain._h, 1, 2, fake, fake, fake, 1, fake, need, None) == -1   # not split
    assert lib.mpk_gs2_smooth(split._h, 17, 2, fake, fake, fake, 1, fake, need, None) == -1  # gamma
    assert lib.mpk_gs2_smooth(split._h, 1, -1, fake, fake, fake, 1, fake, need, None) == -1  # sweeps
    assert lib.mpk_gs2_smooth(split._h, 1, 1 << 17, fake, fake, fake, 1, fake, need, None) == -1
    assert lib.mpk_gs2_smooth(split._h, 1, 2, None, fake, fake, 1, fake, need, None) == -1   # null b
    assert lib.mpk_gs2_smooth(split._h, 1, 2, fake, fake, None, 1, fake, need, None) == -1   # null r
    assert lib.mpk_gs2_smooth(split._h, 1, 2, fake, fake, fake, 64, fake, need, None) == -1  # flag bit
    assert lib.mpk_gs2_smooth(split._h, 2, 2, fake, fake, fake, 1, fake, need - 8, None) == -1  # work
    assert lib.mpk_gs2_smooth(split._h, 2, 2, fake, fake, fake, 1, ctypes.c_void_p((1 << 20) + 8), need,
                              None) == -1                                                   # misaligned
    assert lib.mpk_gs2_smooth(split._h, 2, 2, fake, fake, fake, 1, fake, need, None) == -6    # not uploaded


def test_block_cap_and_tuner_argument_errors_without_gpu():
    lib = M.lib()
    plan = M.Plan.from_csr(S.laplacian_2d(8))
    assert lib.mpk_set_block(plan._h, 4) == 0 and lib.mpk_set_block(plan._h, 0) == 0
    assert lib.mpk_set_block(plan._h, -1) == -1 and lib.mpk_set_block(plan._h, 16) == -1
    assert lib.mpk_set_block(None, 2) == -1
    q, t = ctypes.c_int32(), ctypes.c_double()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.mpk_tune_block(plan._h, 0, fake, fake, 64, None, ctypes.byref(q), None) == -1   # p < 1
    assert lib.mpk_tune_block(plan._h, 4, fake, fake, 63, None, ctypes.byref(q), None) == -1   # ldy < n
    assert lib.mpk_tune_block(plan._h, 4, None, fake, 64, None, ctypes.byref(q), None) == -1   # null x
    assert lib.mpk_tune_block(plan._h, 4, fake, fake, 64, None, None, None) == -1              # null q_out
    assert lib.mpk_tune_block(plan._h, 4, fake, fake, 64, None, ctypes.byref(q), ctypes.byref(t)) == -6


def test_update_values_checks_the_pattern():
    A = S.laplacian_2d(20, 17)
    plan = M.Plan.from_csr(A)
    plan.update_values(S.CSR(A.n, A.rowptr, A.col, A.val * 2.0))  # same pattern: accepted (host only)
    B = S.laplacian_2d(17, 20)  # same n and nnz, other pattern
    assert B.n == A.n and B.col.size == A.col.size
    with pytest.raises(M.MPKError, match="MPK_ERR_ARG"):
        plan.update_values(B)
    with pytest.raises(M.MPKError, match="MPK_ERR_ARG"):
        plan.update_values(S.laplacian_2d(20, 18))
    with pytest.raises(M.MPKError, match="MPK_ERR_CSR"):
        plan.update_values(S.CSR(A.n, A.rowptr, A.col[::-1].copy(), A.val))


def _ritz(H):
    lib = M.lib()
    k = H.shape[0]
    Hf = np.asfortranarray(H, dtype=np.float64)
    re, im = np.zeros(k), np.zeros(k)
    code = lib.mpk_ritz_values(Hf.ctypes.data_as(ctypes.c_void_p), k, k, re.ctypes.data_as(ctypes.c_void_p),
                               im.ctypes.data_as(ctypes.c_void_p))
    assert code == 0, lib.mpk_last_error()
    return re + 1j * im


def _match(got, ref, tol):
    # eigenvalues as multisets: greedy nearest matching
    ref = list(ref)
    for z in got:
        i = int(np.argmin([abs(z - w) for w in ref]))
        assert abs(z - ref[i]) <= tol * max(1.0, abs(ref[i])), (z, ref[i])
        ref.pop(i)


@pytest.mark.parametrize("k,seed", [(1, 0), (2, 1), (5, 2), (12, 3), (16, 4), (40, 5)])
def test_ritz_values_match_numpy_on_random_hessenberg(k, seed):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((k, k)), -1)
    _match(_ritz(H), np.linalg.eigvals(H), 1e-9)


def test_ritz_values_symmetric_tridiagonal_and_complex_pairs():
    n = 10
    T = np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    ref = 2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    got = _ritz(T)
    assert np.abs(got.imag).max() < 1e-12
    np.testing.assert_allclose(np.sort(got.real), ref, atol=1e-12)
    R = np.array([[1.0, -2.0, 0.5], [2.0, 1.0, 0.3], [0.0, 0.0, 4.0]])  # 1 +- 2i and 4
    _match(_ritz(R), [1 + 2j, 1 - 2j, 4.0], 1e-12)
    # already triangular (every subdiagonal zero) and a rank-deficient block
    U = np.triu(np.arange(1.0, 17.0).reshape(4, 4))
    _match(_ritz(U), np.diag(U), 1e-12)
    Z = np.zeros((3, 3))
    _match(_ritz(Z), [0.0, 0.0, 0.0], 1e-12)


def test_ritz_values_argument_errors():
    lib = M.lib()
    x = np.zeros(4)
    p = x.ctypes.data_as(ctypes.c_void_p)
    assert lib.mpk_ritz_values(None, 0, 0, None, None) == 0                 # k = 0: nothing to do
    assert lib.mpk_ritz_values(p, 2, -1, p, p) == -1
    assert lib.mpk_ritz_values(p, 1, 2, p, p) == -1                         # ldh < k
    assert lib.mpk_ritz_values(None, 2, 2, p, p) == -1
    assert lib.mpk_ritz_values(p, 600, 513, p, p) == -1
