"""Thin Python binding of libmpk.so (argument marshalling only).

Every step of the matrix power kernel runs in the library: the host planner
(C++) and the HIP kernels for gfx950.  PyTorch provides device memory and the
current stream.  There is no fallback: if the library is missing or fails to
load, importing this module raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpk.so")

MPK_IO_PERMUTED = 1
MPK_PLAIN = 2
MPK_STAGED = 4
MPK_LAST_POWER = 8  # server applies: return y_p only
MPK_RITZ_SHIFTS = 16  # s-step GMRES: Newton shifts from Ritz values
VALUE_TYPES = {"f64": 0, "f32": 1, "bf16": 2}  # bf16: BF16 values with a per-row FP32 scale
POLY_KINDS = {"monomial": 0, "newton": 1, "chebyshev": 2}
# operator kinds of mpk_block_powers
OPS = {"powers": 0, "poly_monomial": 1, "poly_newton": 2, "poly_chebyshev": 3, "newton_basis": 4,
       "jacobi_chain": 5, "gs2_chain": 6, "gs2_smooth": 7}
PRECONDS = {"chebyshev": 0, "none": 1, "jacobi": 2, "gs2": 3}  # right preconditioners of sstep_gmres
CALL_APPLY, CALL_POLY, CALL_SSTEP, CALL_SOLVE = 0, 1, 2, 3

STATUS = {0: "MPK_OK", -1: "MPK_ERR_ARG", -2: "MPK_ERR_CSR", -3: "MPK_ERR_NOMEM",
          -4: "MPK_ERR_HIP", -5: "MPK_ERR_UNSUPPORTED", -6: "MPK_ERR_STATE",
          -7: "MPK_ERR_DEVICE"}

# every entry point declared in include/mpk.h
EXPORTS = ["mpk_options_default", "mpk_version", "mpk_last_error", "mpk_build_levels",
           "mpk_get_levels", "mpk_get_partition", "mpk_get_deps", "mpk_min_workers",
           "mpk_upload", "mpk_work_bytes", "mpk_apply", "poly_apply", "sstep_basis", "mpk_refine_solve",
           "mpk_get_schedule",
           "mpk_permute", "mpk_check_device", "mpk_plan_info", "mpk_destroy",
           "mpk_server_create", "mpk_server_submit_apply", "mpk_server_submit_solve",
           "mpk_server_wait", "mpk_server_destroy", "mpk_sstep_gmres", "mpk_sstep_gmres_work_bytes",
           "mpk_server_submit_gmres", "mpk_jacobi_apply", "mpk_jacobi_work_bytes",
           "mpk_gs2_apply", "mpk_gs2_work_bytes", "mpk_sstep_gmres_ex",
           "mpk_set_block", "mpk_tune_block", "mpk_block_powers", "mpk_set_watchdog",
           "poly_apply_static", "mpk_update_values", "mpk_plan_cache_create", "mpk_plan_cache_get",
           "mpk_plan_cache_release", "mpk_plan_cache_stats", "mpk_plan_cache_destroy", "mpk_server_create_ex",
           "mpk_gs2_smooth", "mpk_gs2_smooth_work_bytes", "mpk_ritz_values", "mpk_min_workers_units",
           "mpk_block_shape"]


class MPKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("root_mode", ctypes.c_int32), ("root", ctypes.c_int32),
                ("p_block", ctypes.c_int32), ("workers_per_xcd", ctypes.c_int32),
                ("watchdog_polls", ctypes.c_int32), ("chunks_per_worker", ctypes.c_int32),
                ("value_type", ctypes.c_int32), ("max_reg_slots", ctypes.c_int32),
                ("cache_mib", ctypes.c_int32), ("min_group_rows", ctypes.c_int32),
                ("column_scaling", ctypes.c_int32), ("split_lower", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "or python paper_2309_02228_amd/build.py")
    # PyTorch's HIP libraries ask for "libamdhip64.so" while the runtime's
    # soname is "libamdhip64.so.7".  Loading libmpk.so first would map the
    # system runtime under that soname and make torch map a second HIP and HSA
    # runtime; only one of the two then sees the GPU.  Importing torch first
    # lets libmpk.so bind to torch's runtime: one runtime per process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ, U32, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                               ctypes.c_size_t, ctypes.c_uint32, ctypes.c_void_p)
    pI32, pI64, pSZ = (ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                       ctypes.POINTER(ctypes.c_size_t))
    sig = {
        "mpk_options_default": (None, [ctypes.POINTER(Options)]),
        "mpk_version": (ctypes.c_char_p, []),
        "mpk_last_error": (ctypes.c_char_p, []),
        "mpk_build_levels": (I32, [I32, P, P, P, ctypes.POINTER(Options), ctypes.POINTER(P), pSZ]),
        "mpk_get_levels": (I32, [P, pI32, P, P, P, P]),
        "mpk_get_partition": (I32, [P, pI32, pI32, pI32, P]),
        "mpk_get_deps": (I32, [P, pI64, P, P]),
        "mpk_min_workers": (I32, [P, I32, pI32]),
        "mpk_block_powers": (I32, [P, I32, pI32]),
        "mpk_min_workers_units": (I32, [P, I32, I32, pI32]),
        "mpk_block_shape": (I32, [P, I32, pI32, pI32, pI32]),
        "mpk_set_watchdog": (I32, [P, I32]),
        "poly_apply_static": (I32, [P, I32, I32, P, P, D, D, U32, P]),
        "mpk_update_values": (I32, [P, I32, P, P, P, P]),
        "mpk_plan_cache_create": (I32, [SZ, ctypes.POINTER(P)]),
        "mpk_plan_cache_get": (I32, [P, I32, P, P, P, P, P, ctypes.POINTER(P), pI32]),
        "mpk_plan_cache_release": (I32, [P, P]),
        "mpk_plan_cache_stats": (I32, [P, pI32, pSZ, pI64, pI64, pI64]),
        "mpk_plan_cache_destroy": (None, [P]),
        "mpk_server_create_ex": (I32, [I32, I32, SZ, ctypes.c_double, ctypes.POINTER(P)]),
        "mpk_upload": (I32, [P, P, SZ, P]),
        "mpk_work_bytes": (I32, [P, I32, I32, U32, pSZ]),
        "mpk_apply": (I32, [P, D, D, I64, I32, U32, P, SZ, P]),
        "poly_apply": (I32, [P, I32, I32, P, P, D, D, U32, P, SZ, P]),
        "sstep_basis": (I32, [P, I32, P, P, D, D, I64, U32, P, SZ, P]),
        "mpk_get_schedule": (I32, [P, I32, pI32, pI32, P]),
        "mpk_refine_solve": (I32, [P, P, I32, ctypes.c_double, ctypes.c_double, D, D, ctypes.c_double, I32,
                                   U32, P, SZ, pI32, ctypes.POINTER(ctypes.c_double), P]),
        "mpk_permute": (I32, [P, D, D, I32, P]),
        "mpk_check_device": (I32, [P, P]),
        "mpk_plan_info": (I32, [P, pI64, pI64, pI32, pI32, pI64, pI32, pI32, pI32]),
        "mpk_destroy": (None, [P]),
        "mpk_server_create": (I32, [I32, SZ, ctypes.POINTER(P)]),
        "mpk_server_submit_apply": (I32, [P, P, P, I32, P, U32, pI64]),
        "mpk_server_submit_solve": (I32, [P, P, P, P, P, I32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          I32, U32, pI64]),
        "mpk_server_wait": (I32, [P, I64, pI32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), pI32, ctypes.POINTER(ctypes.c_double)]),
        "mpk_server_destroy": (None, [P]),
        "mpk_sstep_gmres": (I32, [P, P, I32, I32, I32, ctypes.c_double, ctypes.c_double, P, P, ctypes.c_double,
                                  I32, U32, P, SZ, pI32, pI32, ctypes.POINTER(ctypes.c_double), P]),
        "mpk_sstep_gmres_work_bytes": (I32, [P, I32, I32, I32, U32, pSZ]),
        "mpk_sstep_gmres_ex": (I32, [P, P, I32, I32, I32, I32, ctypes.c_double, ctypes.c_double, P, P,
                                     ctypes.c_double, I32, U32, P, SZ, pI32, pI32, ctypes.POINTER(ctypes.c_double), P]),
        "mpk_jacobi_apply": (I32, [P, I32, P, P, I64, I32, U32, P, SZ, P]),
        "mpk_jacobi_work_bytes": (I32, [P, I32, I32, U32, pSZ]),
        "mpk_gs2_apply": (I32, [P, I32, P, P, I64, I32, U32, P, SZ, P]),
        "mpk_gs2_work_bytes": (I32, [P, I32, I32, U32, pSZ]),
        "mpk_gs2_smooth": (I32, [P, I32, I32, P, P, P, U32, P, SZ, P]),
        "mpk_gs2_smooth_work_bytes": (I32, [P, I32, U32, pSZ]),
        "mpk_ritz_values": (I32, [P, I64, I32, P, P]),
        "mpk_set_block": (I32, [P, I32]),
        "mpk_tune_block": (I32, [P, I32, P, P, I64, P, pI32, ctypes.POINTER(ctypes.c_double)]),
        "mpk_server_submit_gmres": (I32, [P, P, P, P, P, I32, I32, I32, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, I32, U32, pI64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def version():
    return _lib.mpk_version().decode()


def _check(code):
    if code != 0:
        raise MPKError(code, _lib.mpk_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Plan:
    """A matrix prepared for the blocked MPK (levels, permutation, layout, schedule).

    ``Plan(n, rowptr, col, val)`` runs the host planner (``mpk_build_levels``);
    ``upload()`` places it in device memory owned by a torch tensor.
    """

    def __init__(self, n, rowptr, col, val, root=None, p_block=0, workers_per_xcd=0,
                 watchdog_polls=0, chunks_per_worker=0, values="f64", max_reg_slots=0, cache_mib=0,
                 min_group_rows=0, column_scaling=None, split_lower=False):
        self._h = None
        self.n = int(n)
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        opt = Options()
        _lib.mpk_options_default(ctypes.byref(opt))
        if root is not None:
            opt.root_mode, opt.root = 1, int(root)
        opt.p_block = int(p_block)
        opt.workers_per_xcd = int(workers_per_xcd)
        opt.watchdog_polls = int(watchdog_polls)
        opt.chunks_per_worker = int(chunks_per_worker)
        if values not in VALUE_TYPES:
            raise ValueError(f"values must be one of {sorted(VALUE_TYPES)}")
        opt.value_type = VALUE_TYPES[values]
        opt.max_reg_slots = int(max_reg_slots)
        opt.cache_mib = int(cache_mib)
        opt.min_group_rows = int(min_group_rows)
        if column_scaling not in (None, "jacobi"):
            raise ValueError("column_scaling must be None or 'jacobi' (the plan then holds A D^-1)")
        opt.column_scaling = 1 if column_scaling == "jacobi" else 0
        opt.split_lower = 1 if split_lower else 0
        self.column_scaling = column_scaling
        self.values = values
        h = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        _check(_lib.mpk_build_levels(self.n, _ptr(rowptr), _ptr(col), _ptr(val), ctypes.byref(opt),
                                     ctypes.byref(h), ctypes.byref(nbytes)))
        self._h = h
        self.device_bytes = nbytes.value
        self.buffer = None

    @classmethod
    def from_csr(cls, A, **kw):
        return cls(A[0], A[1], A[2], A[3], **kw)

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mpk_destroy(self._h)
            self._h = None

    def update_values(self, A, stream=None):
        """New values of the same sparsity pattern (CSR tuple A): levels and layout are
        kept, the values refilled and, once uploaded, copied to the device."""
        n, rowptr, col, val = A
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        st = _stream(stream) if self.buffer is not None or stream is not None else None
        _check(_lib.mpk_update_values(self._h, int(n), _ptr(rowptr), _ptr(col), _ptr(val), st))
        return self

    # ---------------------------------------------------------- host tables
    def levels(self):
        nl = ctypes.c_int32()
        _check(_lib.mpk_get_levels(self._h, ctypes.byref(nl), None, None, None, None))
        lp = np.empty(nl.value + 1, np.int32)
        lv, perm, iperm = (np.empty(self.n, np.int32) for _ in range(3))
        _check(_lib.mpk_get_levels(self._h, ctypes.byref(nl), _ptr(lp), _ptr(lv), _ptr(perm), _ptr(iperm)))
        return {"nlevels": nl.value, "level_ptr": lp, "level_of_row": lv, "perm": perm, "iperm": iperm}

    def partition(self):
        nc, cr, npart = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.mpk_get_partition(self._h, ctypes.byref(nc), ctypes.byref(cr), ctypes.byref(npart), None))
        owner = np.empty(nc.value, np.int32)
        _check(_lib.mpk_get_partition(self._h, ctypes.byref(nc), ctypes.byref(cr), ctypes.byref(npart), _ptr(owner)))
        return {"nchunks": nc.value, "chunk_rows": cr.value, "nparts": npart.value, "owner": owner}

    def deps(self):
        nd = ctypes.c_int64()
        _check(_lib.mpk_get_deps(self._h, ctypes.byref(nd), None, None))
        nc = self.partition()["nchunks"]
        ptr = np.empty(nc + 1, np.int32)
        idx = np.empty(max(1, nd.value), np.int32)
        _check(_lib.mpk_get_deps(self._h, ctypes.byref(nd), _ptr(ptr), _ptr(idx)))
        return ptr, idx[:nd.value]

    def schedule(self, q):
        """Level-group wavefront of one block of q powers: (ngroups, tasks) with tasks an
        (ntasks, 4) array of {stage, k, row_begin, row_end} in permuted rows."""
        nt, ng = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.mpk_get_schedule(self._h, int(q), ctypes.byref(nt), ctypes.byref(ng), None))
        t = np.empty((max(1, nt.value), 4), np.int32)
        _check(_lib.mpk_get_schedule(self._h, int(q), ctypes.byref(nt), ctypes.byref(ng), _ptr(t)))
        return ng.value, t[:nt.value]

    def min_workers(self, q, chunks_per_worker=None):
        """Deadlock bound (waves per XCD) for blocks of q powers, for the plan's units or,
        given chunks_per_worker, for the units of that size the plan holds."""
        w = ctypes.c_int32()
        if chunks_per_worker is None:
            _check(_lib.mpk_min_workers(self._h, int(q), ctypes.byref(w)))
        else:
            _check(_lib.mpk_min_workers_units(self._h, int(chunks_per_worker), int(q), ctypes.byref(w)))
        return w.value

    def block_powers(self, op="powers"):
        """Powers per blocked launch for calls of operator kind ``op`` (see OPS); 1 means
        those calls run the plain kernel."""
        q = ctypes.c_int32()
        _check(_lib.mpk_block_powers(self._h, OPS[op], ctypes.byref(q)))
        return q.value

    def block_shape(self, op="powers"):
        """(waves per XCD, chunks per wave, register slots per row) of the blocked kernel
        that calls of operator kind ``op`` use."""
        w, g, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.mpk_block_shape(self._h, OPS[op], ctypes.byref(w), ctypes.byref(g), ctypes.byref(r)))
        return w.value, g.value, r.value

    def info(self):
        n, nnz, slots = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        nl, nc, reg, wk, pb = (ctypes.c_int32() for _ in range(5))
        _check(_lib.mpk_plan_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(nl),
                                  ctypes.byref(nc), ctypes.byref(slots), ctypes.byref(reg),
                                  ctypes.byref(wk), ctypes.byref(pb)))
        return {"n": n.value, "nnz": nnz.value, "nlevels": nl.value, "nchunks": nc.value,
                "sell_slots": slots.value, "reg_slots": reg.value, "workers_per_xcd": wk.value,
                "p_block": pb.value, "values": self.values}

    # --------------------------------------------------------------- device
    def upload(self, device="cuda", stream=None):
        import torch
        self.buffer = torch.empty(max(256, self.device_bytes), dtype=torch.uint8, device=device)
        _check(_lib.mpk_upload(self._h, _dptr(self.buffer), self.buffer.numel(), _stream(stream)))
        return self

    def work_bytes(self, call, p, flags):
        b = ctypes.c_size_t()
        _check(_lib.mpk_work_bytes(self._h, int(call), int(p), int(flags), ctypes.byref(b)))
        return b.value

    def _work(self, call, p, flags, device):
        import torch
        nb = self.work_bytes(call, p, flags)
        if nb == 0:
            return None, 0
        w = torch.empty(nb // 8 + 1, dtype=torch.float64, device=device)
        return w, nb

    @staticmethod
    def _flags(permuted, plain, staged=False):
        return (MPK_IO_PERMUTED if permuted else 0) | (MPK_PLAIN if plain else 0) | (MPK_STAGED if staged else 0)

    def apply(self, x, p, Y=None, permuted=True, plain=False, stream=None, staged=False):
        """Y[k-1] = A^k x for k = 1..p (a (p, n) float64 tensor)."""
        import torch
        if Y is None:
            Y = torch.empty((p, self.n), dtype=torch.float64, device=x.device)
        flags = self._flags(permuted, plain, staged)
        w, nb = self._work(CALL_APPLY, p, flags, x.device)
        ldy = Y.stride(0) if Y.dim() == 2 else self.n
        _check(_lib.mpk_apply(self._h, _dptr(x), _dptr(Y), ldy, int(p), flags, _dptr(w), nb,
                              _stream(stream)))
        return Y

    def poly(self, kind, c, x, params=None, out=None, permuted=True, plain=False, stream=None, staged=False):
        """out = sum_k c[k] phi_k(A) x (kind: monomial, newton, chebyshev)."""
        import torch
        c = np.ascontiguousarray(c, dtype=np.float64)
        pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=x.device)
        flags = self._flags(permuted, plain, staged)
        d = c.size - 1
        w, nb = self._work(CALL_POLY, d, flags, x.device)
        _check(_lib.poly_apply(self._h, POLY_KINDS[kind], d, _ptr(c), _ptr(pr), _dptr(x), _dptr(out),
                               flags, _dptr(w), nb, _stream(stream)))
        return out

    def poly_static(self, kind, c, x, params=None, out=None, permuted=True, plain=False, stream=None):
        """``poly`` through poly_apply_static: no work buffer, the library's per-device
        static scratch holds the intermediate vectors."""
        import torch
        c = np.ascontiguousarray(c, dtype=np.float64)
        pr = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=x.device)
        flags = self._flags(permuted, plain)
        _check(_lib.poly_apply_static(self._h, POLY_KINDS[kind], c.size - 1, _ptr(c), _ptr(pr), _dptr(x), _dptr(out),
                                      flags, _stream(stream)))
        return out

    def sstep(self, v, lambdas, sigmas=None, V=None, permuted=True, plain=False, stream=None, staged=False):
        """(s+1, n) Newton basis: V[0] = v, V[k] = (A - lambda_k I) V[k-1] / sigma_k."""
        import torch
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        sig = None if sigmas is None else np.ascontiguousarray(sigmas, dtype=np.float64)
        s = lam.size
        if V is None:
            V = torch.empty((s + 1, self.n), dtype=torch.float64, device=v.device)
        flags = self._flags(permuted, plain, staged)
        w, nb = self._work(CALL_SSTEP, s, flags, v.device)
        _check(_lib.sstep_basis(self._h, s, _ptr(lam), _ptr(sig), _dptr(v), _dptr(V), V.stride(0),
                                flags, _dptr(w), nb, _stream(stream)))
        return V

    def refine_solve(self, lo, b, degree, lmin, lmax, tol=1e-10, max_iter=1000, x=None, permuted=True,
                     plain=False, stream=None, staged=False):
        """Solve A x = b: FP64 residuals with this plan (FP64 values), corrections with
        the degree-``degree`` Chebyshev polynomial of ``lo`` (the same matrix, FP32 or FP64
        values).  Returns (x, corrections applied, final ||r|| / ||b||)."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        flags = self._flags(permuted, plain, staged)
        w, nb = lo._work(CALL_SOLVE, degree, flags, b.device)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        _check(_lib.mpk_refine_solve(self._h, lo._h, int(degree), float(lmin), float(lmax), _dptr(b), _dptr(x),
                                     float(tol), int(max_iter), flags, _dptr(w), nb, ctypes.byref(it),
                                     ctypes.byref(rel), _stream(stream)))
        return x, it.value, rel.value

    def jacobi_apply(self, x, p, k, Y=None, permuted=True, plain=False, staged=False, stream=None):
        """W[j-1] = (A P^{-1})^j x, j = 1..p, with P^{-1} k Jacobi sweeps from zero; the
        plan must hold A D^{-1} (column_scaling="jacobi").  Returns a (p, n) tensor."""
        import torch
        if Y is None:
            Y = torch.empty((p, self.n), dtype=torch.float64, device=x.device)
        flags = self._flags(permuted, plain, staged)
        nb = ctypes.c_size_t()
        _check(_lib.mpk_jacobi_work_bytes(self._h, int(k), int(p), flags, ctypes.byref(nb)))
        w = torch.empty(nb.value // 8 + 1, dtype=torch.float64, device=x.device) if nb.value else None
        _check(_lib.mpk_jacobi_apply(self._h, int(k), _dptr(x), _dptr(Y), Y.stride(0), int(p), flags,
                                     _dptr(w) if w is not None else None, nb.value, _stream(stream)))
        return Y

    def gs2_apply(self, x, p, gamma, Y=None, permuted=True, plain=False, staged=False, stream=None):
        """W[j-1] = (A P^{-1})^j x, j = 1..p, with P^{-1} one GS2 iteration from zero with
        ``gamma`` inner sweeps; the plan must be built with split_lower=True."""
        import torch
        if Y is None:
            Y = torch.empty((p, self.n), dtype=torch.float64, device=x.device)
        flags = self._flags(permuted, plain, staged)
        nb = ctypes.c_size_t()
        _check(_lib.mpk_gs2_work_bytes(self._h, int(gamma), int(p), flags, ctypes.byref(nb)))
        w = torch.empty(nb.value // 8 + 64, dtype=torch.float64, device=x.device)
        _check(_lib.mpk_gs2_apply(self._h, int(gamma), _dptr(x), _dptr(Y), Y.stride(0), int(p), flags, _dptr(w),
                                  w.numel() * 8, _stream(stream)))
        return Y

    def gs2_smooth(self, b, x, sweeps, gamma, r=None, permuted=True, plain=False, staged=False, stream=None):
        """AMG pre-smoothing fused with the residual: ``sweeps`` outer GS2 iterations
        (``gamma`` inner sweeps; 0 is Jacobi) on A x = b from x, which is overwritten with
        the result, then r = b - A x.  Returns (x, r); the plan must be built with
        split_lower=True."""
        import torch
        if r is None:
            r = torch.empty_like(b)
        flags = self._flags(permuted, plain, staged)
        nb = ctypes.c_size_t()
        _check(_lib.mpk_gs2_smooth_work_bytes(self._h, int(gamma), flags, ctypes.byref(nb)))
        w = torch.empty(nb.value // 8 + 64, dtype=torch.float64, device=b.device)
        _check(_lib.mpk_gs2_smooth(self._h, int(gamma), int(sweeps), _dptr(b), _dptr(x), _dptr(r), flags, _dptr(w),
                                   w.numel() * 8, _stream(stream)))
        return x, r

    def gmres_work_bytes(self, s, m, degree, permuted=True):
        nb = ctypes.c_size_t()
        _check(_lib.mpk_sstep_gmres_work_bytes(self._h, int(s), int(m), int(degree),
                                               MPK_IO_PERMUTED if permuted else 0, ctypes.byref(nb)))
        return nb.value

    def sstep_gmres(self, lo, b, s, m, degree, lmin, lmax, tol=1e-10, max_cycles=100, x=None, permuted=True,
                    plain=False, staged=False, stream=None, work=None, precond="chebyshev"):
        """Solve A x = b by restarted s-step GMRES (blocks of ``s``, restart ``m``) with the
        right degree-``degree`` Chebyshev polynomial preconditioner on [lmin, lmax] (or
        ``precond`` none / jacobi / gs2): FP64 residuals with this plan, basis and
        preconditioner with ``lo`` (the same matrix, FP32 or FP64 values).  With
        lmin = lmax = None (not for Chebyshev) the Newton shifts come from Ritz values of
        the first cycle's Arnoldi steps.  Returns (x, basis vectors built, cycles, final
        ||r|| / ||b||)."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        flags = self._flags(permuted, plain, staged)
        nb = lo.gmres_work_bytes(s, m, degree, permuted)
        if work is None:
            work = torch.empty(nb // 8 + 64, dtype=torch.float64, device=b.device)
        it, cy, rel = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        if precond not in PRECONDS:
            raise ValueError(f"precond must be one of {sorted(PRECONDS)}")
        if lmin is None and lmax is None:
            flags |= MPK_RITZ_SHIFTS
            lmin = lmax = 0.0
        _check(_lib.mpk_sstep_gmres_ex(self._h, lo._h, PRECONDS[precond], int(s), int(m), int(degree), float(lmin),
                                       float(lmax), _dptr(b), _dptr(x), float(tol), int(max_cycles), flags,
                                       _dptr(work), work.numel() * work.element_size(), ctypes.byref(it),
                                       ctypes.byref(cy), ctypes.byref(rel), _stream(stream)))
        return x, it.value, cy.value, rel.value

    def set_block(self, q):
        """Caps the powers per blocked launch at q (0 removes the cap)."""
        _check(_lib.mpk_set_block(self._h, int(q)))

    def tune_block(self, x, p, Y=None, stream=None):
        """Times the blocked MPK of p powers for each admissible block size on x (level
        order), keeps the fastest as the plan's cap; returns (q, seconds per call)."""
        import torch
        if Y is None:
            Y = torch.empty((p, self.n), dtype=torch.float64, device=x.device)
        q, t = ctypes.c_int32(), ctypes.c_double()
        _check(_lib.mpk_tune_block(self._h, int(p), _dptr(x), _dptr(Y), Y.stride(0), _stream(stream),
                                   ctypes.byref(q), ctypes.byref(t)))
        return q.value, t.value

    def permute(self, x, direction=0, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(x)
        _check(_lib.mpk_permute(self._h, _dptr(x), _dptr(out), int(direction), _stream(stream)))
        return out

    def set_watchdog(self, polls):
        """Polls of a pending entry before a blocked-kernel wave gives up (0: default,
        negative: at once)."""
        _check(_lib.mpk_set_watchdog(self._h, int(polls)))

    def check(self, stream=None):
        """Synchronises ``stream`` and raises MPKError if a blocked launch on it reported a
        failure."""
        _check(_lib.mpk_check_device(self._h, _stream(stream)))


class CachedPlan(Plan):
    """A plan held by a PlanCache (not destroyed by Python; released to the cache)."""

    def __init__(self, handle, n, cache, values):
        self._h = handle
        self.n = int(n)
        self.values = values
        self.column_scaling = None
        self.buffer = None
        self._cache = cache

    def __del__(self):
        pass  # the cache owns the plan

    def release(self):
        if self._h is not None:
            _check(_lib.mpk_plan_cache_release(self._cache._h, self._h))
            self._h = None


class PlanCache:
    """Plans keyed by sparsity pattern (mpk_plan_cache_*), on the current device,
    within ``device_bytes`` of plan buffers."""

    OUTCOMES = {0: "hit", 1: "new values", 2: "planned"}

    def __init__(self, device_bytes=8 << 30):
        h = ctypes.c_void_p()
        _check(_lib.mpk_plan_cache_create(int(device_bytes), ctypes.byref(h)))
        self._h = h

    def get(self, A, values="f64", p_block=0, stream=None):
        """(plan, outcome) for the CSR tuple A; release the plan when done with it."""
        n, rowptr, col, val = A
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        opt = Options()
        _lib.mpk_options_default(ctypes.byref(opt))
        opt.p_block = int(p_block)
        opt.value_type = VALUE_TYPES[values]
        h = ctypes.c_void_p()
        out = ctypes.c_int32()
        _check(_lib.mpk_plan_cache_get(self._h, int(n), _ptr(rowptr), _ptr(col), _ptr(val), ctypes.byref(opt),
                                       _stream(stream), ctypes.byref(h), ctypes.byref(out)))
        return CachedPlan(h, n, self, values), self.OUTCOMES[out.value]

    def stats(self):
        pl, used = ctypes.c_int32(), ctypes.c_size_t()
        hits, upd, miss = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.mpk_plan_cache_stats(self._h, ctypes.byref(pl), ctypes.byref(used), ctypes.byref(hits),
                                         ctypes.byref(upd), ctypes.byref(miss)))
        return {"plans": pl.value, "bytes_used": used.value, "hits": hits.value, "value_updates": upd.value,
                "misses": miss.value}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mpk_plan_cache_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Server:
    """Request server on the current device: host-memory MPK applications and
    refinement solves, run by ``workers`` threads with a stream each and
    admitted in arrival order against a device pool of ``device_bytes``."""

    def __init__(self, workers=4, device_bytes=1 << 30, apply_workers=0, max_wait_s=None):
        """``workers`` take any request, ``apply_workers`` matrix powers only; with
        ``max_wait_s`` (seconds) any waiting request that fits may start before older
        ones until the oldest has waited that long; None is strict arrival order."""
        h = ctypes.c_void_p()
        if apply_workers == 0 and max_wait_s is None:
            _check(_lib.mpk_server_create(int(workers), int(device_bytes), ctypes.byref(h)))
        else:
            _check(_lib.mpk_server_create_ex(int(workers), int(apply_workers), int(device_bytes),
                                             float(max_wait_s or 0.0), ctypes.byref(h)))
        self._h = h
        self._keep = {}  # ticket -> host arrays and plans the request uses

    def __del__(self):
        if _lib is not None:  # at interpreter exit the module's globals may already be gone
            self.close()

    def close(self):
        if getattr(self, "_h", None):
            _lib.mpk_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    @staticmethod
    def _host(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        return a

    def submit_apply(self, plan, x, p, permuted=True, plain=False, staged=False, last_only=False, Y=None):
        """Queues y_1..y_p of host vector x (y_p alone with ``last_only``) into
        ``Y`` (a new (p, n) or (n,) float64 array if None); returns the ticket."""
        x = self._host(x)
        shape = (x.shape[0],) if last_only else (p, x.shape[0])  # row k-1 holds y_k
        if Y is None:
            Y = np.empty(shape, dtype=np.float64)
        if Y.shape != shape or Y.dtype != np.float64 or not Y.flags.c_contiguous:
            raise ValueError(f"Y must be a C-contiguous float64 array of shape {shape}")
        flags = Plan._flags(permuted, plain, staged) | (MPK_LAST_POWER if last_only else 0)
        t = ctypes.c_int64()
        _check(_lib.mpk_server_submit_apply(self._h, plan._h, _ptr(x), int(p), _ptr(Y), flags, ctypes.byref(t)))
        self._keep[t.value] = (plan, x, Y)
        return t.value

    def submit_solve(self, hi, lo, b, degree, lmin, lmax, tol=1e-10, max_iter=1000, x0=None, permuted=True,
                     plain=False, staged=False):
        """Queues a refinement solve of A x = b (host vectors); ``x0`` (zeros if
        None) is the initial guess and receives the solution.  Returns the ticket."""
        b = self._host(b)
        x = np.zeros_like(b) if x0 is None else x0
        if x.shape != b.shape or x.dtype != np.float64 or not x.flags.c_contiguous:
            raise ValueError("x0 must be a C-contiguous float64 array shaped like b (overwritten by the solution)")
        t = ctypes.c_int64()
        _check(_lib.mpk_server_submit_solve(self._h, hi._h, lo._h, _ptr(b), _ptr(x), int(degree), float(lmin),
                                            float(lmax), float(tol), int(max_iter),
                                            Plan._flags(permuted, plain, staged), ctypes.byref(t)))
        self._keep[t.value] = (hi, lo, b, x)
        return t.value

    def submit_gmres(self, hi, lo, b, s, m, degree, lmin, lmax, tol=1e-10, max_cycles=100, x0=None,
                     permuted=True, plain=False, staged=False):
        """Queues an s-step GMRES solve of A x = b (host vectors); ``x0`` (zeros if None) is
        the initial guess and receives the solution.  Returns the ticket; the result's
        "iters" counts basis vectors."""
        b = self._host(b)
        x = np.zeros_like(b) if x0 is None else x0
        if x.shape != b.shape or x.dtype != np.float64 or not x.flags.c_contiguous:
            raise ValueError("x0 must be a C-contiguous float64 array shaped like b (overwritten by the solution)")
        t = ctypes.c_int64()
        _check(_lib.mpk_server_submit_gmres(self._h, hi._h, lo._h, _ptr(b), _ptr(x), int(s), int(m), int(degree),
                                            float(lmin), float(lmax), float(tol), int(max_cycles),
                                            Plan._flags(permuted, plain, staged), ctypes.byref(t)))
        self._keep[t.value] = (hi, lo, b, x)
        return t.value

    def wait(self, ticket):
        """Waits for a request.  Returns a dict with the result ("Y": p x n for an
        apply, "x" for a solve), "latency_s", "queue_s", "iters", "relres";
        raises MPKError if the request failed."""
        st = ctypes.c_int32()
        lat, qs, rel = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        it = ctypes.c_int32()
        _check(_lib.mpk_server_wait(self._h, int(ticket), ctypes.byref(st), ctypes.byref(lat), ctypes.byref(qs),
                                    ctypes.byref(it), ctypes.byref(rel)))
        keep = self._keep.pop(int(ticket))
        _check(st.value)
        out = {"latency_s": lat.value, "queue_s": qs.value, "iters": it.value, "relres": rel.value}
        if len(keep) == 3:
            out["Y"] = keep[2]
        else:
            out["x"] = keep[3]
        return out
