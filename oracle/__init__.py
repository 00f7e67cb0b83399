"""ctypes wrapper of the plain FP64 CPU revised-simplex oracle (simplex_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the CPU
baseline leg of bench.py, never by the product package.  It shares no code with
the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "simplex_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with -fopenmp: loops over independent columns and rows run on
# several threads, with bit-identical results (each dot product keeps its order).
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OPTIMAL, UNBOUNDED, ITER_LIMIT, NUMERICAL, INFEASIBLE = 1, 2, 3, 4, 5
STATUS_NAMES = {0: "RUNNING", 1: "OPTIMAL", 2: "UNBOUNDED", 3: "ITER_LIMIT", 4: "NUMERICAL", 5: "INFEASIBLE"}
FLAG_DEGENERATE, FLAG_TIE, FLAG_ASPIRATION, FLAG_LCLEAR, FLAG_DRIVEOUT = 1, 2, 4, 8, 16
ROW_LE, ROW_GE, ROW_EQ = 0, 1, 2

# -ffp-contract=off: only the explicit fma() calls fuse.  x86-64-v3 has hardware FMA,
# so fma() is one correctly rounded instruction instead of a libm emulation.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-march=x86-64-v3", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Builds the sequential library and the -fopenmp one; returns the sequential one's path."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB


def omp_lib(threads: int = 0) -> str:
    """Path of the -fopenmp build (built if missing), with its thread count set (0: the
    OpenMP default, normally every core)."""
    if not os.path.exists(_LIB_OMP):
        build(force=False)
    L = lib(_LIB_OMP)
    L.oracle_set_threads(int(threads))
    return _LIB_OMP


def threads(lib_path: str | None = None) -> int:
    """Threads the given build runs on (1 for the sequential build)."""
    return int(lib(lib_path).oracle_set_threads(0))


_libs = {}


def lib(path: str | None = None):
    """Load the oracle library (or, for mutation tests, another build of the same source)."""
    key = path or _LIB
    if key not in _libs:
        if path is None and not os.path.exists(_LIB):
            build()
        L = C.CDLL(key)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.oracle_create.restype = P
        L.oracle_create.argtypes = [I32, I32, dp, dp, dp, I32, I32, I32, D, D, D, D]
        L.oracle_create_general.restype = P
        L.oracle_create_general.argtypes = [I32, I32, dp, dp, dp, ip, I32, I32, I32, D, D, D, D]
        L.oracle_phase.restype = I32
        L.oracle_phase.argtypes = [P]
        L.oracle_columns.restype = I32
        L.oracle_columns.argtypes = [P]
        L.oracle_destroy.argtypes = [P]
        L.oracle_run.restype = I32
        L.oracle_run.argtypes = [P, I64]
        L.oracle_iterations.restype = I64
        L.oracle_iterations.argtypes = [P]
        L.oracle_status.restype = I32
        L.oracle_status.argtypes = [P]
        L.oracle_ray.restype = I32
        L.oracle_ray.argtypes = [P]
        L.oracle_objective.restype = D
        L.oracle_objective.argtypes = [P]
        L.oracle_solution.argtypes = [P, dp, dp, ip]
        L.oracle_state.argtypes = [P, dp, dp, dp, dp]
        L.oracle_pivots.restype = I64
        L.oracle_pivots.argtypes = [P, ip, ip, ip, ip, I64]
        L.oracle_margins.restype = I64
        L.oracle_margins.argtypes = [P, dp, I64]
        L.oracle_counts.argtypes = [P, C.POINTER(C.c_int64)]
        L.oracle_set_threads.restype = I32
        L.oracle_set_threads.argtypes = [I32]
        L.oracle_basis_inverse.restype = I32
        L.oracle_basis_inverse.argtypes = [I32, I32, dp, ip, dp]
        _libs[key] = L
    return _libs[key]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


@dataclass
class Result:
    status: int
    iterations: int
    objective: float
    x: np.ndarray
    y: np.ndarray
    basis: np.ndarray
    enter: np.ndarray
    row: np.ndarray
    leave: np.ndarray
    flags: np.ndarray
    counts: dict = field(default_factory=dict)
    ray: int = -1
    # per pivot: the distance of its closest decision from its threshold or rival value
    # (a report, never used in a decision; inf for drive-out pivots)
    margin: np.ndarray = None

    @property
    def status_name(self):
        return STATUS_NAMES.get(self.status, str(self.status))


class Oracle:
    """One LP held by the oracle; run() may be called repeatedly (resume).

    With row_type (ROW_LE / ROW_GE / ROW_EQ per row) the LP may have >= and = rows and b of
    any sign, and is solved by the two-phase method; its handle then has extra surplus
    columns after the caller's n (self.ncols in all), which pivot logs and bases use."""

    def __init__(self, A, b, c, sense="max", tenure=5, leaving_list=True, eps_d=1e-9, eps_p=1e-9,
                 eps_z=1e-9, eps_t=1e-9, lib_path=None, row_type=None):
        self._L = lib(lib_path)
        A = np.asarray(A, dtype=np.float64)
        m, n = A.shape
        self.m, self.n = m, n
        self._A = np.asfortranarray(A)
        self._b = np.ascontiguousarray(b, dtype=np.float64)
        self._c = np.ascontiguousarray(c, dtype=np.float64)
        assert self._b.shape == (m,) and self._c.shape == (n,)
        s = {"min": 0, "max": 1}[sense]
        if row_type is None:
            self._h = self._L.oracle_create(m, n, _dp(self._A), _dp(self._b), _dp(self._c), s, int(tenure),
                                          int(bool(leaving_list)), eps_d, eps_p, eps_z, eps_t)
        else:
            self._rt = np.ascontiguousarray(row_type, dtype=np.int32)
            assert self._rt.shape == (m,)
            self._h = self._L.oracle_create_general(m, n, _dp(self._A), _dp(self._b), _dp(self._c),
                                                  _ip(self._rt), s, int(tenure), int(bool(leaving_list)),
                                                  eps_d, eps_p, eps_z, eps_t)
        if not self._h:
            raise ValueError("oracle_create rejected the LP (m<=0, negative or non-finite b, bad row type, "
                             "or no memory)")
        self.ncols = self._L.oracle_columns(self._h)

    @property
    def phase(self):
        return self._L.oracle_phase(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.oracle_destroy(h)
            self._h = None

    def run(self, max_iter=None):
        if max_iter is None:
            max_iter = 10 * (self.m + self.ncols)
        st = self._L.oracle_run(self._h, int(max_iter))
        if st < 0:
            raise MemoryError("oracle ran out of memory")
        return st

    @property
    def iterations(self):
        return self._L.oracle_iterations(self._h)

    def state(self):
        m = self.m
        Binv = np.empty((m, m))
        xB = np.empty(m)
        W = np.empty(m)
        z = C.c_double()
        self._L.oracle_state(self._h, _dp(Binv), _dp(xB), _dp(W), C.byref(z))
        return Binv, xB, W, z.value

    def result(self) -> Result:
        L = self._L
        m, n = self.m, self.n
        x = np.empty(self.ncols)
        y = np.empty(m)
        basis = np.empty(m, dtype=np.int32)
        L.oracle_solution(self._h, _dp(x), _dp(y), _ip(basis))
        x = x[:n].copy()
        cnt = L.oracle_pivots(self._h, None, None, None, None, 0)
        e = np.empty(cnt, dtype=np.int32)
        r = np.empty(cnt, dtype=np.int32)
        lv = np.empty(cnt, dtype=np.int32)
        f = np.empty(cnt, dtype=np.int32)
        L.oracle_pivots(self._h, _ip(e), _ip(r), _ip(lv), _ip(f), cnt)
        mg = np.empty(cnt)
        L.oracle_margins(self._h, _dp(mg), cnt)
        counts = (C.c_int64 * 4)()
        L.oracle_counts(self._h, counts)
        return Result(status=L.oracle_status(self._h), iterations=L.oracle_iterations(self._h),
                      objective=L.oracle_objective(self._h), x=x, y=y, basis=basis, enter=e, row=r,
                      leave=lv, flags=f,
                      counts=dict(degenerate=counts[0], tie=counts[1], aspiration=counts[2], lclear=counts[3]),
                      ray=L.oracle_ray(self._h), margin=mg)


def solve(A, b, c, sense="max", max_iter=None, **kw) -> Result:
    o = Oracle(A, b, c, sense=sense, **kw)
    o.run(max_iter)
    return o.result()


def basis_inverse(A, basis, lib_path=None):
    """B^-1 (m x m) of the basis list `basis` of (A', I), by Gauss-Jordan elimination with
    partial pivoting; None if B is singular."""
    A = np.asfortranarray(np.asarray(A, dtype=np.float64))
    m, n = A.shape
    basis = np.ascontiguousarray(basis, dtype=np.int32)
    if basis.shape != (m,):
        raise ValueError("basis must have m entries")
    out = np.empty((m, m))
    rc = lib(lib_path).oracle_basis_inverse(m, n, _dp(A), _ip(basis), _dp(out))
    return out if rc == 0 else None
