"""Seeded synthetic layered-battery systems (inputs only).

The paper's linear systems are finite-element snapshots of thermal-battery
simulations (Sec. 2: solid/liquid voltage, Butler-Volmer coupling, liquid
continuity, Stefan-Maxwell species) and are not public.  This module builds
finite-volume stand-ins with the same block structure; the assembly rules are
documented at the top of ``synth.c``.  It holds none of the solver's
arithmetic and is shared by the solver's tests/benchmark and the CPU oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

FIELD_NAMES_4 = ("phi_s", "phi_e", "p", "c")
FIELD_NAMES_6 = ("phi_s", "phi_e", "p", "c1", "c2", "c3")

# Named workloads: the five layered-battery configurations.
CONFIGS = {
    0: dict(nx=32, ny=32, nz=0, nspecies=1),      # 2D, 4 fields, 4,096 DOF
    1: dict(nx=64, ny=64, nz=64, nspecies=1),     # 3D, 4 fields, 1,048,576 DOF
    2: dict(nx=128, ny=128, nz=64, nspecies=1),   # 3D, 4 fields, 4,194,304 DOF
    3: dict(nx=96, ny=96, nz=96, nspecies=3),     # 3D, 6 fields, 5,308,416 DOF
    4: dict(nx=256, ny=256, nz=128, nspecies=3),  # 3D, 6 fields, 50,331,648 DOF
}


class SynthParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nspecies", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("diff", ctypes.c_double * 3), ("inv_dt", ctypes.c_double), ("mig", ctypes.c_double),
        ("perm_lo", ctypes.c_double), ("perm_hi", ctypes.c_double),
        ("j0_lo", ctypes.c_double), ("j0_hi", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile libsynth.so with gcc (no floating-point contraction)."""
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.synth_u01.restype = ctypes.c_double
        lib.synth_u01.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_layer.restype = ctypes.c_int32
        lib.synth_layer.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.synth_nrows.restype = ctypes.c_int64
        lib.synth_nrows.argtypes = [P(SynthParams)]
        lib.synth_rowptr.restype = ctypes.c_int64
        lib.synth_rowptr.argtypes = [P(SynthParams), ctypes.c_void_p]
        lib.synth_fill.restype = ctypes.c_int
        lib.synth_fill.argtypes = [P(SynthParams), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_cells.restype = ctypes.c_int
        lib.synth_cells.argtypes = [P(SynthParams)] + [ctypes.c_void_p] * 4
        lib.synth_uniform_pm1.restype = None
        lib.synth_uniform_pm1.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        lib.synth_matvec.restype = None
        lib.synth_matvec.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 5
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_seed(cfg: int) -> int:
    return 2602 * 16 + cfg


def make_params(nx, ny, nz=0, nspecies=1, seed=0, diff=None, inv_dt=100.0, mig=0.1) -> SynthParams:
    if diff is None:
        diff = (1e-3, 5e-4, 2e-3)
    p = SynthParams()
    p.nx, p.ny, p.nz, p.nspecies, p.seed = nx, ny, nz, nspecies, seed
    for i in range(3):
        p.diff[i] = diff[i]
    p.inv_dt, p.mig = inv_dt, mig
    p.perm_lo, p.perm_hi = 1e-3, 1e-1
    p.j0_lo, p.j0_hi = 0.1, 10.0
    return p


def u01(seed: int, stream: int, idx: int) -> float:
    return _load().synth_u01(seed, stream, idx)


def uniform_pm1(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_uniform_pm1(seed, stream, n, _ptr(out))
    return out


def matvec(rowptr, col, val, x) -> np.ndarray:
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    y = np.empty(len(rp) - 1, dtype=np.float64)
    _load().synth_matvec(len(rp) - 1, _ptr(rp), _ptr(np.ascontiguousarray(col, dtype=np.int32)),
                         _ptr(np.ascontiguousarray(val, dtype=np.float64)),
                         _ptr(np.ascontiguousarray(x, dtype=np.float64)), _ptr(y))
    return y


class System(dict):
    """CSR system plus seeded vectors; keys documented in :func:`make_system`."""

    def __getattr__(self, k):
        try:
            return self[k]
        except KeyError as e:
            raise AttributeError(k) from e


def make_system(nx=None, ny=None, nz=0, nspecies=1, seed=None, cfg=None, j0=None,
                with_dj0=True) -> System:
    """Assemble one layered-battery system.

    Returns a System with: n, nnz, nf, rowptr (int32), col (int32), val (f64),
    field_of_row (int32), x_star, b = A x_star, x_t (targets), j0 (per cell),
    layer (per cell), dcell/dcoef (per nnz: the cell whose j0 the entry is
    linear in, and d val / d j0), dims, field_names, tree (group bracket code).
    """
    if cfg is not None:
        c = CONFIGS[cfg]
        nx, ny, nz, nspecies = c["nx"], c["ny"], c["nz"], c["nspecies"]
        if seed is None:
            seed = default_seed(cfg)
    if seed is None:
        seed = 0
    lib = _load()
    p = make_params(nx, ny, nz, nspecies, seed)
    n = lib.synth_nrows(ctypes.byref(p))
    rowptr = np.empty(n + 1, dtype=np.int64)
    nnz = lib.synth_rowptr(ctypes.byref(p), _ptr(rowptr))
    if nnz < 0:
        raise MemoryError("synth_rowptr failed")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    dcell = np.empty(nnz, dtype=np.int32) if with_dj0 else None
    dcoef = np.empty(nnz, dtype=np.float64) if with_dj0 else None
    fld = np.empty(n, dtype=np.int32)
    j0o = None if j0 is None else np.ascontiguousarray(j0, dtype=np.float64)
    rc = lib.synth_fill(ctypes.byref(p), _ptr(j0o), _ptr(rowptr), _ptr(col), _ptr(val),
                        _ptr(dcell), _ptr(dcoef), _ptr(fld))
    if rc != 0:
        raise RuntimeError(f"synth_fill failed ({rc})")
    ncell = n // (3 + nspecies)
    layer = np.empty(ncell, dtype=np.int32)
    j0s = np.empty(ncell, dtype=np.float64)
    lib.synth_cells(ctypes.byref(p), _ptr(layer), _ptr(j0s), None, None)
    x_star = uniform_pm1(seed, 2, n)
    b = np.empty(n, dtype=np.float64)
    lib.synth_matvec(n, _ptr(rowptr), _ptr(col), _ptr(val), _ptr(x_star), _ptr(b))
    x_t = uniform_pm1(seed, 4, n)
    nf = 3 + nspecies
    if nspecies == 1:
        tree = [-1, -1, 0, 1, -2, -1, 2, -2, -1, 3, -2, -2]
        names = FIELD_NAMES_4
    else:
        tree = [-1, -1, 0, 1, -2, -1, 2, -2, -1, 3, 4, 5, -2, -2]
        names = FIELD_NAMES_6
    return System(n=int(n), nnz=int(nnz), nf=nf, rowptr=rowptr.astype(np.int32), col=col, val=val,
                  field_of_row=fld, x_star=x_star, b=b, x_t=x_t, j0=j0s if j0 is None else j0o,
                  layer=layer, dcell=dcell, dcoef=dcoef, seed=seed,
                  dims=(nx, ny, nz), field_names=names, tree=tree)


def fd_cells(seed: int, layer: np.ndarray, count: int = 8) -> np.ndarray:
    """Seeded electrode cells (stream 5) for finite-difference gradient checks."""
    elec = np.flatnonzero((layer == 1) | (layer == 3))
    out = []
    i = 0
    while len(out) < count:
        c = int(elec[int(u01(seed, 5, i) * len(elec))])
        if c not in out:
            out.append(c)
        i += 1
    return np.array(out, dtype=np.int64)
