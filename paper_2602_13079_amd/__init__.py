"""Python binding of libhbgs (argument marshalling only).

Block Gauss-Seidel / SA-AMG preconditioned flexible GMRES for coupled
multiphysics systems on one AMD MI355X.  Every step of setup, apply, solve
and gradient runs in the HIP library ``libhbgs.so`` (C ABI in
``include/hbgs.h``); PyTorch provides device memory and streams.  There is no
CPU fallback: if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhbgs.so")
_lib = None

MAX_FIELDS = 16
MAX_LEVELS = 16
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESINGULAR", -5: "ESETUP"}


class HBGSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hbgs {STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("cheb_degree", ctypes.c_int32), ("cheb_ratio", ctypes.c_double),
        ("cheb_boost", ctypes.c_double), ("eig_iters", ctypes.c_int32), ("sa_damping", ctypes.c_double),
        ("coarse_max", ctypes.c_int32), ("max_levels", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("theta", ctypes.c_double * MAX_FIELDS), ("use_graphs", ctypes.c_int32),
        ("setup_concurrent", ctypes.c_int32), ("block_jacobi", ctypes.c_int32), ("nested", ctypes.c_int32),
        ("inner_restart", ctypes.c_int32), ("inner_max_iters", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
        ("field_cheb_degree", ctypes.c_int32 * MAX_FIELDS), ("field_leaf", ctypes.c_int32 * MAX_FIELDS),
        ("ilu_block", ctypes.c_int32), ("build_transpose", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_fields", ctypes.c_int32), ("nnz", ctypes.c_int64),
        ("levels", ctypes.c_int32 * MAX_FIELDS),
        ("rows", (ctypes.c_int32 * MAX_LEVELS) * MAX_FIELDS),
        ("nnz_a", (ctypes.c_int64 * MAX_LEVELS) * MAX_FIELDS),
        ("nnz_p", (ctypes.c_int64 * MAX_LEVELS) * MAX_FIELDS),
        ("vcycle_bytes", ctypes.c_double * 2), ("spmv_bytes", ctypes.c_double * 2),
        ("setup_seconds", ctypes.c_double), ("setup_field_seconds", ctypes.c_double * MAX_FIELDS),
        ("setup_stage_seconds", ctypes.c_double * 8),
    ]


EXPORTS = {
    "hbgs_default_options": (None, ["opt*"]),
    "hbgs_setup": ("i32", ["ctx**", "i32", "i64", "p", "p", "p", "i32", "p", "i32", "p", "opt*", "p"]),
    "hbgs_set_values": ("i32", ["p", "p", "i32", "p"]),
    "hbgs_set_precision": ("i32", ["p", "i32"]),
    "hbgs_set_tolerance": ("i32", ["p", "f64", "i32"]),
    "hbgs_apply": ("i32", ["p", "p", "p", "i32", "p"]),
    "hbgs_apply_noalloc": ("i32", ["p", "p", "p", "i32", "p"]),
    "hbgs_solve": ("i32", ["p", "p", "p", "i32", "i32", "i32*", "p", "i32", "i32*", "p"]),
    "hbgs_grad_values": ("i32", ["p", "p", "p", "p", "p"]),
    "hbgs_stats": ("i32", ["p", "stats*"]),
    "hbgs_get_level": ("i32", ["p", "i32", "i32", "i32", "i32*", "i32*", "i64*", "p", "p", "p"]),
    "hbgs_get_aggregates": ("i32", ["p", "i32", "i32", "p", "p"]),
    "hbgs_profile": ("i32", ["p", "i32"]),
    "hbgs_kernel_times": ("i32", ["p", "p", "p", "p", "p", "i32"]),
    "hbgs_set_allocator": ("i32", ["p", "p", "p"]),
    "hbgs_debug_spgemm_route": ("i32", ["i32"]),
    "hbgs_debug_spmv_tiles": ("i32", ["i32"]),
    "hbgs_destroy": (None, ["p"]),
    "hbgs_last_error": ("str", []),
}


def _ctype(t):
    return {
        "i32": ctypes.c_int32, "i64": ctypes.c_int64, "f64": ctypes.c_double, "p": ctypes.c_void_p,
        "str": ctypes.c_char_p,
        "ctx**": ctypes.POINTER(ctypes.c_void_p), "opt*": ctypes.POINTER(Options),
        "stats*": ctypes.POINTER(Stats), "i32*": ctypes.POINTER(ctypes.c_int32),
        "i64*": ctypes.POINTER(ctypes.c_int64), None: None,
    }[t]


def load(path: str = LIB_PATH):
    """Load libhbgs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_2602_13079_amd/build.py "
                              "(there is no CPU fallback)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = _ctype(res)
            fn.argtypes = [_ctype(a) for a in args]
        _lib = lib
    return _lib


def default_options(**kw) -> Options:
    o = Options()
    load().hbgs_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k in ("theta", "field_cheb_degree", "field_leaf"):
            arr = getattr(o, k)
            for i in range(MAX_FIELDS):
                arr[i] = 0
            for i, t in enumerate(v):
                arr[i] = t
        else:
            setattr(o, k, v)
    return o


def _check(code):
    if code < 0:
        raise HBGSError(code, load().hbgs_last_error().decode())
    return code


def _values_key(val):
    """Identity of a value tensor's current contents: storage address and
    in-place version counter."""
    return (val.data_ptr(), getattr(val, "_version", 0), val.numel())


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, torch):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.contiguous()


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_alloc_hooks = []  # every installed pair stays alive: live contexts free through the hook that allocated


def set_allocator(alloc=None, free=None):
    """Route the persistent device memory of Solvers created afterwards
    through alloc(nbytes) -> int pointer (0 on failure) and free(pointer);
    no arguments restores hipMalloc / hipFree."""
    lib = load()
    if alloc is None and free is None:
        _check(lib.hbgs_set_allocator(None, None, None))
        return

    def _a(nbytes, user):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:  # reported to the library as an allocation failure
            return None

    def _f(ptr, user):
        free(int(ptr))

    hooks = (_ALLOC_FN(_a), _FREE_FN(_f))
    _check(lib.hbgs_set_allocator(ctypes.cast(hooks[0], ctypes.c_void_p), ctypes.cast(hooks[1], ctypes.c_void_p),
                                  None))
    _alloc_hooks.append(hooks)


def debug_spgemm_route(route: int = 0):
    """Process-wide test knob: the kernel path of every sparse product row in
    the Galerkin products (0 by size, 1 wavefront, 2 block, 3 global tables)."""
    _check(load().hbgs_debug_spgemm_route(int(route)))


def debug_spmv_tiles(on: bool = True):
    """Process-wide test knob: SpMVs stage their operand tiles in LDS where
    the matrix has them (default), or always gather (bitwise the same)."""
    _check(load().hbgs_debug_spmv_tiles(1 if on else 0))


def use_torch_allocator(enable=True):
    """Serve Solver memory from torch's caching allocator (or stop doing so)."""
    if not enable:
        set_allocator()
        return
    import torch
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n), torch.cuda.caching_allocator_delete)


class Solver:
    """Preconditioner + GMRES context for one CSR pattern.

    rowptr/col: int32 device tensors; val: float64 device tensor;
    field_of_row: int32 device tensor; tree: bracket code (see hbgs.h).
    """

    def __init__(self, rowptr, col, val, field_of_row, n_fields, tree, **opts):
        import torch
        self._torch = torch
        self.lib = load()
        values_key = _values_key(val)
        rowptr = _dev(rowptr, torch.int32, torch)
        col = _dev(col, torch.int32, torch)
        val = _dev(val, torch.float64, torch)
        field_of_row = _dev(field_of_row, torch.int32, torch)
        self.n = rowptr.numel() - 1
        self.nnz = col.numel()
        self.n_fields = n_fields
        self.opts = default_options(**opts)
        tr = (ctypes.c_int32 * len(tree))(*tree)
        h = ctypes.c_void_p()
        _check(self.lib.hbgs_setup(ctypes.byref(h), self.n, self.nnz, rowptr.data_ptr(), col.data_ptr(),
                                   val.data_ptr(), n_fields, field_of_row.data_ptr(), len(tree), tr,
                                   ctypes.byref(self.opts), _stream(torch)))
        self.h = h
        self._values_key = values_key

    def __del__(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.hbgs_destroy(self.h)
            self.h = None

    def set_precision(self, p: int):
        _check(self.lib.hbgs_set_precision(self.h, p))

    def set_tolerance(self, rtol, max_iters=2000):
        _check(self.lib.hbgs_set_tolerance(self.h, float(rtol), int(max_iters)))
        self.opts.rtol, self.opts.max_iters = rtol, max_iters

    def set_values(self, val, rebuild=True):
        """New values on the same pattern; rebuild=False keeps the preconditioner."""
        key = _values_key(val)
        val = _dev(val, self._torch.float64, self._torch)
        _check(self.lib.hbgs_set_values(self.h, val.data_ptr(), int(rebuild), _stream(self._torch)))
        self._values_key = key

    def apply(self, r, transpose=False):
        torch = self._torch
        r = _dev(r, torch.float64, torch)
        z = torch.empty_like(r)
        _check(self.lib.hbgs_apply(self.h, r.data_ptr(), z.data_ptr(), int(transpose), _stream(torch)))
        return z

    def apply_noalloc(self, r, z, transpose=False):
        """z = M^-1 r (or M^-T r) into the caller's z through the entry point
        that allocates nothing; enqueued on the current stream, no sync."""
        torch = self._torch
        if not (r.is_cuda and z.is_cuda and r.dtype == z.dtype == torch.float64
                and r.is_contiguous() and z.is_contiguous() and r.numel() == z.numel() == self.n):
            raise ValueError("r and z must be contiguous float64 device tensors of n entries")
        _check(self.lib.hbgs_apply_noalloc(self.h, r.data_ptr(), z.data_ptr(), int(transpose), _stream(torch)))
        return z

    def solve(self, b, x0=None, transpose=False, hist_cap=4096):
        """Returns (x, status, iters, residual history as numpy)."""
        torch = self._torch
        b = _dev(b, torch.float64, torch)
        x = torch.zeros_like(b) if x0 is None else _dev(x0, torch.float64, torch).clone()
        it = ctypes.c_int32()
        hl = ctypes.c_int32()
        hist = np.zeros(hist_cap)
        st = _check(self.lib.hbgs_solve(self.h, b.data_ptr(), x.data_ptr(), int(x0 is not None), int(transpose),
                                        ctypes.byref(it), hist.ctypes.data_as(ctypes.c_void_p), hist_cap,
                                        ctypes.byref(hl), _stream(torch)))
        return x, st, it.value, hist[:min(hl.value, hist_cap)].copy()

    def grad_values(self, lam, x):
        torch = self._torch
        lam = _dev(lam, torch.float64, torch)  # kept alive until the kernel is enqueued
        x = _dev(x, torch.float64, torch)
        g = torch.empty(self.nnz, dtype=torch.float64, device=lam.device)
        _check(self.lib.hbgs_grad_values(self.h, lam.data_ptr(), x.data_ptr(), g.data_ptr(), _stream(torch)))
        return g

    def stats(self) -> dict:
        st = Stats()
        _check(self.lib.hbgs_stats(self.h, ctypes.byref(st)))
        nf = st.n_fields
        return dict(
            n=st.n, nnz=st.nnz, n_fields=nf,
            levels=[st.levels[f] for f in range(nf)],
            rows=[[st.rows[f][l] for l in range(st.levels[f])] for f in range(nf)],
            nnz_a=[[st.nnz_a[f][l] for l in range(st.levels[f])] for f in range(nf)],
            nnz_p=[[st.nnz_p[f][l] for l in range(st.levels[f])] for f in range(nf)],
            vcycle_bytes=list(st.vcycle_bytes), spmv_bytes=list(st.spmv_bytes),
            setup_seconds=st.setup_seconds,
            setup_field_seconds=[st.setup_field_seconds[f] for f in range(nf)],
            setup_stage_seconds=list(st.setup_stage_seconds))

    def get_level(self, field, level, which="A"):
        """Host copy (rowptr, col, val, ncols) of A_l / P_l / R_l / A_l^T."""
        w = {"A": 0, "P": 1, "R": 2, "AT": 3}[which]
        nr, nc, nz = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(self.lib.hbgs_get_level(self.h, field, level, w, ctypes.byref(nr), ctypes.byref(nc),
                                       ctypes.byref(nz), None, None, None))
        rp = np.empty(nr.value + 1, dtype=np.int32)
        ci = np.empty(nz.value, dtype=np.int32)
        v = np.empty(nz.value, dtype=np.float64)
        _check(self.lib.hbgs_get_level(self.h, field, level, w, None, None, None,
                                       rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p),
                                       v.ctypes.data_as(ctypes.c_void_p)))
        return rp, ci, v, nc.value

    def aggregates(self, field, level):
        nrows = self.get_level(field, level, "A")[0].shape[0] - 1
        agg = np.empty(nrows, dtype=np.int32)
        sc = np.empty(3)
        _check(self.lib.hbgs_get_aggregates(self.h, field, level, agg.ctypes.data_as(ctypes.c_void_p),
                                            sc.ctypes.data_as(ctypes.c_void_p)))
        return agg, dict(lam_cheb=sc[0], lam_p=sc[1], omega=sc[2])

    def level_scalars(self, field, level):
        sc = np.empty(3)
        _check(self.lib.hbgs_get_aggregates(self.h, field, level, None, sc.ctypes.data_as(ctypes.c_void_p)))
        return dict(lam_cheb=sc[0], lam_p=sc[1], omega=sc[2])

    def profile(self, on=True, kinds=None):
        """Enable event timing of all kernel classes, or only the named ones."""
        if not on:
            mask = 0
        elif kinds is None:
            mask = -1
        else:
            names = list(self.kernel_times())
            mask = 0
            for k in kinds:
                mask |= 1 << names.index(k)
        _check(self.lib.hbgs_profile(self.h, mask))

    def kernel_times(self) -> dict:
        cap = 64
        names = (ctypes.c_char * 48 * cap)()
        ms = np.zeros(cap)
        cnt = np.zeros(cap, dtype=np.int64)
        by = np.zeros(cap)
        k = self.lib.hbgs_kernel_times(self.h, names, ms.ctypes.data_as(ctypes.c_void_p),
                                       cnt.ctypes.data_as(ctypes.c_void_p), by.ctypes.data_as(ctypes.c_void_p), cap)
        if k < 0:
            raise HBGSError(-3, self.lib.hbgs_last_error().decode())
        out = {}
        for i in range(k):
            nm = bytes(names[i]).split(b"\0")[0].decode()
            out[nm] = dict(ms=float(ms[i]), launches=int(cnt[i]), bytes=float(by[i]))
        return out


def _autograd_function():
    import torch

    class HBGSSolve(torch.autograd.Function):
        """x = A(val)^-1 b with implicit differentiation.

        backward solves the adjoint system A^T lambda = dL/dx on the same
        hierarchy (transposed operators, reversed sweep) and returns
        dL/db = lambda and dL/dval[p] = -lambda[row p] * x[col p].
        The preconditioner is not differentiated (exact at convergence).
        """

        @staticmethod
        def forward(ctx, val, b, solver):
            if _values_key(val) != solver._values_key:  # new values: rebuild the preconditioner
                solver.set_values(val)
            x, st, it, _ = solver.solve(b)
            if st != 0:
                raise HBGSError(st, f"forward solve did not converge ({it} iterations)")
            ctx.solver = solver
            ctx.save_for_backward(x)
            return x

        @staticmethod
        def backward(ctx, g):
            (x,) = ctx.saved_tensors
            solver = ctx.solver
            lam, st, it, _ = solver.solve(g.contiguous(), transpose=True)
            if st != 0:
                raise HBGSError(st, f"adjoint solve did not converge ({it} iterations)")
            grad_val = solver.grad_values(lam, x) if ctx.needs_input_grad[0] else None
            return grad_val, lam, None

    return HBGSSolve


_HBGSSolve = None


def hbgs_solve(val, b, solver: Solver):
    """Differentiable solve x = A(val)^-1 b.  When val is not the tensor (or
    its version) the solver last saw, its values are loaded first (with a
    preconditioner rebuild)."""
    global _HBGSSolve
    if _HBGSSolve is None:
        _HBGSSolve = _autograd_function()
    return _HBGSSolve.apply(val, b, solver)
