"""CPU oracle (test infrastructure only).

Plain double-precision restatement of the block Gauss-Seidel / SA-AMG /
flexible GMRES method, compiled from ``hbgs_oracle.cpp`` with g++ and called
through ctypes.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("cheb_degree", ctypes.c_int32), ("cheb_ratio", ctypes.c_double),
        ("cheb_boost", ctypes.c_double), ("eig_iters", ctypes.c_int32), ("sa_damping", ctypes.c_double),
        ("omega_override", ctypes.c_double), ("coarse_max", ctypes.c_int32), ("max_levels", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("theta", ctypes.c_double * 16), ("exact_leaves", ctypes.c_int32),
        ("block_jacobi", ctypes.c_int32), ("nested", ctypes.c_int32), ("inner_restart", ctypes.c_int32),
        ("inner_max_iters", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
        ("field_cheb_degree", ctypes.c_int32 * 16), ("field_leaf", ctypes.c_int32 * 16),
        ("ilu_block", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "hbgs_oracle.cpp")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        P = ctypes.POINTER(Options)
        sig = {
            "or_default_options": (None, [P]),
            "or_last_error": (ctypes.c_char_p, []),
            "or_set_threads": (None, [i32]),
            "or_get_threads": (i32, []),
            "or_set_verbose": (None, [i32]),
            "or_amg_setup": (vp, [i32, vp, vp, vp, f64, P, u64]),
            "or_amg_destroy": (None, [vp]),
            "or_amg_levels": (i32, [vp]),
            "or_amg_smoothed_coarsest": (i32, [vp]),
            "or_amg_get": (i64, [vp, i32, i32, vp, vp, vp, vp, vp]),
            "or_amg_agg": (None, [vp, i32, vp]),
            "or_amg_scalars": (None, [vp, i32, vp]),
            "or_amg_vcycle": (None, [vp, P, i32, i32, vp, vp]),
            "or_amg_chebyshev": (None, [vp, P, i32, vp, vp, i32]),
            "or_strength": (None, [i32, vp, vp, vp, f64, vp]),
            "or_aggregate": (i32, [i32, vp, vp, vp, vp, u64, vp, vp]),
            "or_agg_key": (u64, [i32, u64]),
            "or_power_estimate": (f64, [i32, vp, vp, vp, vp, i32, u64]),
            "or_filter": (None, [i32, vp, vp, vp, vp, vp, vp, vp, vp]),
            "or_spgemm": (i64, [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
            "or_lu_solve": (i32, [i32, vp, vp, vp, vp, vp, i32]),
            "or_setup": (vp, [i32, vp, vp, vp, i32, vp, i32, vp, P]),
            "or_destroy": (None, [vp]),
            "or_set_precision": (None, [vp, i32]),
            "or_levels": (i32, [vp, i32]),
            "or_field_amg": (vp, [vp, i32]),
            "or_apply": (None, [vp, vp, vp, i32]),
            "or_apply_flat": (None, [vp, vp, vp, i32]),
            "or_solve": (i32, [vp, vp, vp, i32, i32, vp, vp, i32, vp]),
            "or_grad_values": (None, [vp, vp, vp, vp]),
            "or_permutation": (None, [vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results are bitwise the same
    for every count)."""
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return _load().or_get_threads()


def set_verbose(on: bool) -> None:
    """Progress lines on stderr while a system's fields are set up."""
    _load().or_set_verbose(int(bool(on)))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def options(**kw) -> Options:
    o = Options()
    _load().or_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "theta":
            for i in range(16):
                o.theta[i] = 0.0
            for i, t in enumerate(v):
                o.theta[i] = t
        elif k in ("field_cheb_degree", "field_leaf"):
            arr = getattr(o, k)
            for i in range(16):
                arr[i] = 0
            for i, t in enumerate(v):
                arr[i] = t
        else:
            setattr(o, k, v)
    return o


def _csr_args(rowptr, col, val):
    return _i32(rowptr), _i32(col), _f64(val)


# ------------------------------------------------------------ building blocks
def strength(rowptr, col, val, theta):
    rp, ci, v = _csr_args(rowptr, col, val)
    out = np.zeros(len(ci), dtype=np.int8)
    _load().or_strength(len(rp) - 1, _p(rp), _p(ci), _p(v), theta, _p(out))
    return out.astype(bool)


def aggregate(rowptr, col, val, strong, salt):
    rp, ci, v = _csr_args(rowptr, col, val)
    n = len(rp) - 1
    agg = np.empty(n, dtype=np.int32)
    root = np.empty(n, dtype=np.int8)
    s = np.ascontiguousarray(strong, dtype=np.int8)
    nagg = _load().or_aggregate(n, _p(rp), _p(ci), _p(v), _p(s), salt, _p(agg), _p(root))
    return agg, root.astype(bool), nagg


def agg_key(i, salt):
    return _load().or_agg_key(i, salt)


def filtered(rowptr, col, val, strong):
    rp, ci, v = _csr_args(rowptr, col, val)
    n = len(rp) - 1
    frp = np.empty(n + 1, dtype=np.int32)
    fci = np.empty(len(ci), dtype=np.int32)
    fv = np.empty(len(ci), dtype=np.float64)
    dabs = np.empty(n, dtype=np.float64)
    s = np.ascontiguousarray(strong, dtype=np.int8)
    _load().or_filter(n, _p(rp), _p(ci), _p(v), _p(s), _p(frp), _p(fci), _p(fv), _p(dabs))
    nnz = frp[-1]
    return frp, fci[:nnz].copy(), fv[:nnz].copy(), dabs


def power_estimate(rowptr, col, val, d, iters, salt):
    rp, ci, v = _csr_args(rowptr, col, val)
    return _load().or_power_estimate(len(rp) - 1, _p(rp), _p(ci), _p(v), _p(_f64(d)), iters, salt)


def spgemm(a, b):
    """a, b: (rowptr, col, val, ncols).  Returns (rowptr, col, val)."""
    arp, aci, av = _csr_args(*a[:3])
    brp, bci, bv = _csr_args(*b[:3])
    n, k, m = len(arp) - 1, a[3], b[3]
    lib = _load()
    nnz = lib.or_spgemm(n, k, m, _p(arp), _p(aci), _p(av), _p(brp), _p(bci), _p(bv), None, None, None)
    crp = np.empty(n + 1, dtype=np.int32)
    cci = np.empty(nnz, dtype=np.int32)
    cv = np.empty(nnz, dtype=np.float64)
    lib.or_spgemm(n, k, m, _p(arp), _p(aci), _p(av), _p(brp), _p(bci), _p(bv), _p(crp), _p(cci), _p(cv))
    return crp, cci, cv


def lu_solve(rowptr, col, val, b, transpose=False):
    rp, ci, v = _csr_args(rowptr, col, val)
    x = np.empty(len(rp) - 1)
    rc = _load().or_lu_solve(len(rp) - 1, _p(rp), _p(ci), _p(v), _p(_f64(b)), _p(x), int(transpose))
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return x


class Amg:
    """Single-block SA-AMG hierarchy (oracle)."""

    def __init__(self, rowptr, col, val, theta=0.0, salt=1, opts=None, _handle=None, _owner=None):
        self._lib = _load()
        self.opts = opts if opts is not None else options()
        if _handle is not None:
            self.h, self._owner = _handle, _owner
            return
        rp, ci, v = _csr_args(rowptr, col, val)
        self.h = self._lib.or_amg_setup(len(rp) - 1, _p(rp), _p(ci), _p(v), theta, ctypes.byref(self.opts), salt)
        self._owner = None
        if not self.h:
            raise RuntimeError(self._lib.or_last_error().decode())

    def __del__(self):
        if getattr(self, "h", None) and self._owner is None:
            self._lib.or_amg_destroy(self.h)
            self.h = None

    @property
    def levels(self):
        return self._lib.or_amg_levels(self.h)

    @property
    def smoothed_coarsest(self):
        """True when coarsening stopped above the dense-solve limit and the
        coarsest level is smoothed instead of solved."""
        return bool(self._lib.or_amg_smoothed_coarsest(self.h))

    def get(self, l, which="A"):
        w = {"A": 0, "P": 1, "R": 2, "AT": 3}[which]
        nr, nc = ctypes.c_int(), ctypes.c_int()
        nnz = self._lib.or_amg_get(self.h, l, w, ctypes.byref(nr), ctypes.byref(nc), None, None, None)
        rp = np.empty(nr.value + 1, dtype=np.int32)
        ci = np.empty(nnz, dtype=np.int32)
        v = np.empty(nnz, dtype=np.float64)
        self._lib.or_amg_get(self.h, l, w, None, None, _p(rp), _p(ci), _p(v))
        return rp, ci, v, nc.value

    def agg(self, l):
        n = self.get(l, "A")[0].shape[0] - 1
        out = np.empty(n, dtype=np.int32)
        self._lib.or_amg_agg(self.h, l, _p(out))
        return out

    def scalars(self, l):
        out = np.empty(3)
        self._lib.or_amg_scalars(self.h, l, _p(out))
        return dict(lam_cheb=out[0], lam_p=out[1], omega=out[2])

    def vcycle(self, b, transpose=False, precision=0):
        b = _f64(b)
        x = np.empty_like(b)
        self._lib.or_amg_vcycle(self.h, ctypes.byref(self.opts), int(transpose), precision, _p(b), _p(x))
        return x

    def chebyshev(self, l, b, x0=None):
        b = _f64(b)
        x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
        self._lib.or_amg_chebyshev(self.h, ctypes.byref(self.opts), l, _p(b), _p(x), int(x0 is None))
        return x


def field_salt_base(seed, f):
    """Salt of field f's hierarchy (level l adds l)."""
    def sm(x):
        x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
        x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
        return x ^ (x >> 31)
    return sm((seed + 0x1000 * (f + 1)) & 0xFFFFFFFFFFFFFFFF)


class Oracle:
    """Whole-system oracle: setup / apply / solve / gradient in the original ordering."""

    def __init__(self, rowptr, col, val, nf, field_of_row, tree, **opt):
        self._lib = _load()
        self.opts = options(**opt)
        rp, ci, v = _csr_args(rowptr, col, val)
        self.n = len(rp) - 1
        self.nnz = len(ci)
        fld = _i32(field_of_row)
        tr = _i32(tree)
        self.h = self._lib.or_setup(self.n, _p(rp), _p(ci), _p(v), nf, _p(fld), len(tr), _p(tr),
                                    ctypes.byref(self.opts))
        if not self.h:
            raise RuntimeError(self._lib.or_last_error().decode())
        self.nf = nf

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.or_destroy(self.h)
            self.h = None

    def set_precision(self, precision):
        """Precision mode of later applies and solves (0 double, 1 single-
        precision sweep); the hierarchy is the same for both."""
        self._lib.or_set_precision(self.h, int(precision))
        self.opts.precision = int(precision)

    def amg(self, f) -> Amg:
        return Amg(None, None, None, opts=self.opts, _handle=self._lib.or_field_amg(self.h, f), _owner=self)

    def levels(self, f):
        return self._lib.or_levels(self.h, f)

    def permutation(self):
        out = np.empty(self.n, dtype=np.int32)
        self._lib.or_permutation(self.h, _p(out))
        return out

    def apply(self, r, transpose=False, flat=False):
        r = _f64(r)
        z = np.empty_like(r)
        fn = self._lib.or_apply_flat if flat else self._lib.or_apply
        fn(self.h, _p(r), _p(z), int(transpose))
        return z

    def solve(self, b, x0=None, transpose=False, hist_cap=100000):
        b = _f64(b)
        x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
        it = ctypes.c_int()
        hl = ctypes.c_int()
        hist = np.empty(hist_cap)
        rc = self._lib.or_solve(self.h, _p(b), _p(x), int(x0 is not None), int(transpose), ctypes.byref(it),
                                _p(hist), hist_cap, ctypes.byref(hl))
        return dict(x=x, status=rc, iters=it.value, hist=hist[:min(hl.value, hist_cap)].copy())

    def grad_values(self, lam, x):
        out = np.empty(self.nnz)
        self._lib.or_grad_values(self.h, _p(_f64(lam)), _p(_f64(x)), _p(out))
        return out
