"""FP64 CPU oracle for dictionary learning with Jacobi atom updates.

TEST INFRASTRUCTURE ONLY: the plain, slow statement of what the GPU path
computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import it.  The product package never imports it and
shares no code with it; both sides only receive the same inputs from the
seeded generator module.

The heavy parts (OMP, the group atom update, the error) are plain C with
OpenMP in ``dlo.c``; this module loads that library with ctypes and adds
thin numpy wrappers.  Numpy-only pieces live in sibling modules.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dlo.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RULE_AKSVD = 0
RULE_SGK = 1
RULE_NSGK = 2

# Stop thresholds shared with the GPU path's documented reading of the
# paper's silent points (see the module docstring of dlo.c).
TOL_CORR = 1e-5
TOL_PIVOT = 1e-10

_lib = None


def build(force: bool = True) -> str:
    """Compile ``dlo.c`` into ``liboracle.so`` with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        c_int, c_double, c_long = ctypes.c_int, ctypes.c_double, ctypes.c_long
        lib.dlo_omp.argtypes = [c_int, c_int, c_int, c_int, dp, dp, c_double, c_double, ip, dp]
        lib.dlo_omp.restype = c_long
        lib.dlo_omp_signal.argtypes = [c_int, c_int, c_int, dp, dp, c_double, c_double, ip, dp]
        lib.dlo_omp_signal.restype = c_int
        lib.dlo_residual.argtypes = [c_int, c_int, c_int, dp, dp, ip, dp, dp]
        lib.dlo_residual.restype = None
        lib.dlo_rmse.argtypes = [c_int, c_int, c_int, dp, dp, ip, dp]
        lib.dlo_rmse.restype = c_double
        lib.dlo_jau_update.argtypes = [c_int, c_int, c_int, c_int, dp, dp, ip, dp, c_int, c_int]
        lib.dlo_jau_update.restype = c_long
        lib.dlo_jau_update_range.argtypes = [c_int, c_int, c_int, c_int, dp, dp, ip, dp, c_int,
                                             c_int, c_int, c_int]
        lib.dlo_jau_update_range.restype = c_long
        lib.dlo_nsgk_update_range.argtypes = [c_int, c_int, c_int, c_int, dp, dp, ip, dp, ip,
                                              dp, c_int, c_int, c_int]
        lib.dlo_nsgk_update_range.restype = c_long
        lib.dlo_normalize.argtypes = [c_int, c_int, dp]
        lib.dlo_normalize.restype = None
        lib.dlo_iterate.argtypes = [c_int, c_int, c_int, c_int, dp, dp, c_int, c_int, c_int,
                                    c_double, c_double, ip, dp, dp]
        lib.dlo_iterate.restype = None
        lib.dlo_max_threads.argtypes = []
        lib.dlo_max_threads.restype = c_int
        lib.dlo_set_threads.argtypes = [c_int]
        lib.dlo_set_threads.restype = None
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def omp(D, Y, s, tol_corr=TOL_CORR, tol_pivot=TOL_PIVOT):
    """Plain OMP of every row of ``Y`` [m][p] against the atoms (rows) of ``D`` [n][p].

    Returns ``(idx [m][s] int32, val [m][s] float64, early_stops)``.
    """
    lib = _load()
    D = _f64(D)
    Y = _f64(Y)
    n, p = D.shape
    m = Y.shape[0]
    idx = np.empty((m, s), dtype=np.int32)
    val = np.empty((m, s), dtype=np.float64)
    early = lib.dlo_omp(p, n, m, s, _dp(D), _dp(Y), tol_corr, tol_pivot, _ip(idx), _dp(val))
    return idx, val, int(early)


def residual(Y, D, idx, val):
    """E = Y - D X, one row per signal."""
    lib = _load()
    Y, D, idx, val = _f64(Y), _f64(D), _i32(idx), _f64(val)
    m, p = Y.shape
    s = idx.shape[1]
    E = np.empty((m, p), dtype=np.float64)
    lib.dlo_residual(p, m, s, _dp(Y), _dp(D), _ip(idx), _dp(val), _dp(E))
    return E


def rmse(Y, D, idx, val):
    """||Y - D X||_F / sqrt(p m)."""
    lib = _load()
    Y, D, idx, val = _f64(Y), _f64(D), _i32(idx), _f64(val)
    m, p = Y.shape
    return float(lib.dlo_rmse(p, m, idx.shape[1], _dp(Y), _dp(D), _ip(idx), _dp(val)))


def jau_update(Y, D, idx, val, group_size, rule=RULE_AKSVD, atoms=None):
    """Group-wise Jacobi atom update; returns ``(D_new, val_new, unused_atoms)``.

    ``atoms=(first, end)`` restricts the sweep to atoms [first, end).
    """
    lib = _load()
    Y, idx = _f64(Y), _i32(idx)
    D = _f64(D).copy()
    val = _f64(val).copy()
    n, p = D.shape
    m, s = idx.shape
    a0, a1 = (0, n) if atoms is None else atoms
    unused = lib.dlo_jau_update_range(p, n, m, s, _dp(Y), _dp(D), _ip(idx), _dp(val),
                                      int(group_size), int(rule), int(a0), int(a1))
    return D, val, int(unused)


def nsgk_update(Y, D, idx, val, idx_prev, val_prev, group_size, atoms=None):
    """P-NSGK atom update (eq. 7 with the P-SGK group loop) of ``D`` = D^(k),
    given this iteration's representations X^(k) (``idx``/``val``) and the
    previous ones X^(k-1) (``idx_prev``/``val_prev``); returns
    ``(D_new, unused_atoms)``.  The representations are not changed."""
    lib = _load()
    Y, idx, idx_prev = _f64(Y), _i32(idx), _i32(idx_prev)
    val, val_prev = _f64(val), _f64(val_prev)
    D = _f64(D).copy()
    n, p = D.shape
    m, s = idx.shape
    a0, a1 = (0, n) if atoms is None else atoms
    unused = lib.dlo_nsgk_update_range(p, n, m, s, _dp(Y), _dp(D), _ip(idx), _dp(val),
                                       _ip(idx_prev), _dp(val_prev), int(group_size), int(a0),
                                       int(a1))
    return D, int(unused)


def max_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().dlo_max_threads())


def set_threads(threads: int) -> None:
    """Number of OpenMP threads of the oracle's later calls (timing only)."""
    _load().dlo_set_threads(int(threads))


def normalize(D):
    lib = _load()
    D = _f64(D).copy()
    n, p = D.shape
    lib.dlo_normalize(p, n, _dp(D))
    return D


def iterate(Y, D0, s, iters, group_size, rule=RULE_AKSVD, tol_corr=TOL_CORR, tol_pivot=TOL_PIVOT):
    """``iters`` DL iterations; returns ``(D, idx, val, rmse[iters])``."""
    lib = _load()
    Y = _f64(Y)
    D = _f64(D0).copy()
    n, p = D.shape
    m = Y.shape[0]
    idx = np.empty((m, s), dtype=np.int32)
    val = np.empty((m, s), dtype=np.float64)
    r = np.empty(iters, dtype=np.float64)
    lib.dlo_iterate(p, n, m, s, _dp(Y), _dp(D), int(iters), int(group_size), int(rule),
                    tol_corr, tol_pivot, _ip(idx), _dp(val), _dp(r))
    return D, idx, val, r


def iterate_bf16(Y, D0, s, iters, group_size, rule=RULE_AKSVD, tol_corr=TOL_CORR,
                 tol_pivot=TOL_PIVOT):
    """The precision variant with its quantisation emulated: every OMP sees D
    and Y rounded to BF16 (its correlations and Gram entries are formed from
    those values), the atom update and the error use the FP32 inputs.
    Returns ``(D, idx, val, rmse[iters])``."""
    from .bf16 import round_bf16
    Y32 = np.ascontiguousarray(Y, dtype=np.float32)
    Yb = round_bf16(Y32)
    D = normalize(D0)
    r = np.empty(iters)
    idx = val = None
    for k in range(iters):
        idx, val, _ = omp(round_bf16(D.astype(np.float32)), Yb, s, tol_corr, tol_pivot)
        D, val, _ = jau_update(Y32, D, idx, val, group_size, rule)
        r[k] = rmse(Y32, D, idx, val)
    return D, idx, val, r
