"""ctypes binding of liblpgpu.so: the C ABI of include/lpgpu.h, argument marshalling only.

Every step of the simplex iteration runs in the library's HIP kernels.  The library is
loaded from this package directory; if it is missing, importing raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblpgpu.so")

LP_OK, LP_ERR_ARG, LP_ERR_NEG_RHS, LP_ERR_NOMEM, LP_ERR_DEVICE, LP_ERR_STATE = 0, -1, -2, -3, -4, -5
LP_RUNNING, LP_OPTIMAL, LP_UNBOUNDED, LP_ITER_LIMIT, LP_NUMERICAL, LP_INFEASIBLE = 0, 1, 2, 3, 4, 5
LP_PIVOT_DEGENERATE, LP_PIVOT_TIE, LP_PIVOT_ASPIRATION, LP_PIVOT_LCLEAR, LP_PIVOT_DRIVEOUT = 1, 2, 4, 8, 16
LP_ROW_LE, LP_ROW_GE, LP_ROW_EQ = 0, 1, 2
LP_MIN, LP_MAX = 0, 1
LP_FP64, LP_MIXED = 0, 1
LP_MAX_ROWS = 9792
STATUS_NAMES = {0: "RUNNING", 1: "OPTIMAL", 2: "UNBOUNDED", 3: "ITER_LIMIT", 4: "NUMERICAL", 5: "INFEASIBLE"}


class lp_options(C.Structure):
    _fields_ = [
        ("sense", C.c_int32),
        ("tabu_tenure", C.c_int32),
        ("leaving_list", C.c_int32),
        ("iters_per_sync", C.c_int32),
        ("max_iter", C.c_int64),
        ("eps_d", C.c_double),
        ("eps_p", C.c_double),
        ("eps_z", C.c_double),
        ("eps_t", C.c_double),
        ("record_pivots", C.c_int32),
        ("profile", C.c_int32),
        ("batch_small_m", C.c_int32),
        ("stream", C.c_void_p),
        ("precision", C.c_int32),
        ("shortlist_k", C.c_int32),
        ("reinv_period", C.c_int32),
        ("batch_binv_lds_m", C.c_int32),
        ("device_budget", C.c_int64),
    ]


class lp_stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int64),
        ("degenerate", C.c_int64),
        ("ties", C.c_int64),
        ("aspirations", C.c_int64),
        ("list_clears", C.c_int64),
        ("syncs", C.c_int64),
        ("solve_ms", C.c_double),
        ("price_launches", C.c_int64),
        ("price_ms", C.c_double),
        ("update_launches", C.c_int64),
        ("update_ms", C.c_double),
        ("price_bytes", C.c_double),
        ("update_bytes", C.c_double),
        ("finish_launches", C.c_int64),
        ("finish_ms", C.c_double),
        ("ray", C.c_int64),
        ("price32_launches", C.c_int64),
        ("full_prices", C.c_int64),
        ("reinversions", C.c_int64),
        ("reinv_failed", C.c_int64),
        ("reinv_ms", C.c_double),
        ("price32_ms", C.c_double),
        ("shortlist_ms", C.c_double),
        ("price32_bytes", C.c_double),
        ("phase1_iterations", C.c_int64),
        ("drive_outs", C.c_int64),
        ("phase_switch_ms", C.c_double),
        ("memory_case", C.c_int64),
        ("panel_rows", C.c_int64),
        ("panels", C.c_int64),
        ("price_fin_launches", C.c_int64),
        ("price_fin_ms", C.c_double),
    ]


class lp_batch_stats(C.Structure):
    _fields_ = [
        ("count", C.c_int64),
        ("narrow_lps", C.c_int64),
        ("wide_lps", C.c_int64),
        ("work_items", C.c_int64),
        ("workgroups", C.c_int64),
        ("lds_bytes", C.c_int64),
        ("narrow_bucket_mask", C.c_int64),
        ("solve_ms", C.c_double),
        ("tune_ms", C.c_double),
        ("binv_lds_lps", C.c_int64),
        ("binv_lds_m", C.c_int64),
        ("tuned_from_table", C.c_int64),
    ]


class LPError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().lp_error_string(code).decode()} (code {code})")


_lib = None

# Every function include/lpgpu.h declares, with (restype, argtypes).
_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)
_LP = C.POINTER(C.c_int64)
SIGNATURES = {
    "lp_default_options": (C.c_int, [C.POINTER(lp_options)]),
    "lp_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, _DP, _DP, _DP, C.POINTER(lp_options)]),
    "lp_create_device": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, _P, _P, _P, C.POINTER(lp_options)]),
    "lp_create_general": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, _DP, _DP, _DP, _IP,
                                    C.POINTER(lp_options)]),
    "lp_solve": (C.c_int, [_P, _IP]),
    "lp_solve_until": (C.c_int, [_P, C.c_int64, _IP]),
    "lp_iterate": (C.c_int, [_P, C.c_int64, _IP]),
    "lp_solve_device_noalloc": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.POINTER(lp_options), C.c_void_p, C.c_void_p, C.c_void_p, _IP,
                                          C.POINTER(C.c_int64)]),
    "lp_reset": (C.c_int, [_P]),
    "lp_get_solution": (C.c_int, [_P, _DP, _DP, _DP, _IP, _LP]),
    "lp_get_pivots": (C.c_int, [_P, _IP, _IP, _IP, _IP, C.c_int64, _LP]),
    "lp_get_tableau": (C.c_int, [_P, _DP, _DP, _DP, _DP]),
    "lp_get_stats": (C.c_int, [_P, C.POINTER(lp_stats)]),
    "lp_reinvert": (C.c_int, [_P]),
    "lp_destroy": (None, [_P]),
    "lp_error_string": (C.c_char_p, [C.c_int]),
    "lp_batch_create": (C.c_int, [C.POINTER(_P), C.c_int32, _IP, _IP, C.POINTER(_DP), C.POINTER(_DP),
                                  C.POINTER(_DP), C.POINTER(lp_options)]),
    "lp_batch_create_dense": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_uint64, C.c_int32, C.c_int32,
                                        C.POINTER(lp_options)]),
    "lp_batch_get_sizes": (C.c_int, [_P, _IP, _IP]),
    "lp_batch_solve": (C.c_int, [_P]),
    "lp_batch_results": (C.c_int, [_P, _IP, _DP, _LP]),
    "lp_batch_get": (C.c_int, [_P, C.c_int32, _DP, _IP, _IP, _IP, _IP, C.c_int64, _LP]),
    "lp_batch_get_stats": (C.c_int, [_P, C.POINTER(lp_batch_stats)]),
    "lp_batch_destroy": (None, [_P]),
    "lp_batch_tune_load": (C.c_int, [_P, C.c_char_p]),
    "lp_batch_tune_save": (C.c_int, [_P, C.c_char_p]),
    "lp_solve_batch": (C.c_int, [C.c_int32, _IP, _IP, C.POINTER(_DP), C.POINTER(_DP), C.POINTER(_DP),
                                 C.POINTER(lp_options), _IP, _DP, _LP]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is not built; run python paper_1803_04378_amd/build.py")
        L = C.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code, where):
    if code != LP_OK:
        raise LPError(code, where)


def default_options(**kw) -> lp_options:
    o = lp_options()
    _check(lib().lp_default_options(C.byref(o)), "lp_default_options")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _dptr(a):
    return a.ctypes.data_as(_DP)


class LP:
    """One LP held on the GPU (an lp_problem handle).  With row_type (LP_ROW_LE / LP_ROW_GE /
    LP_ROW_EQ per row) the rows may be >= or = and b may have any sign (lp_create_general,
    two-phase start)."""

    def __init__(self, A=None, b=None, c=None, *, device_tensors=None, sense="max", precision="fp64",
                 row_type=None, **opts):
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        o = default_options(sense=LP_MAX if sense == "max" else LP_MIN,
                            precision=LP_MIXED if precision == "mixed" else LP_FP64, **opts)
        h = _P()
        if device_tensors is not None:
            dA, db, dc, m, n = device_tensors
            rc = lib().lp_create_device(C.byref(h), m, n, dA, db, dc, C.byref(o))
        else:
            A = np.asfortranarray(np.asarray(A, dtype=np.float64))
            b = np.ascontiguousarray(b, dtype=np.float64)
            c = np.ascontiguousarray(c, dtype=np.float64)
            m, n = A.shape
            if b.shape != (m,) or c.shape != (n,):
                raise ValueError("shapes of A, b, c do not match")
            self._keep = (A, b, c)
            if row_type is None:
                rc = lib().lp_create(C.byref(h), m, n, _dptr(A), _dptr(b), _dptr(c), C.byref(o))
            else:
                rt = np.ascontiguousarray(row_type, dtype=np.int32)
                if rt.shape != (m,):
                    raise ValueError("row_type must have m entries")
                self._keep += (rt,)
                rc = lib().lp_create_general(C.byref(h), m, n, _dptr(A), _dptr(b), _dptr(c),
                                             rt.ctypes.data_as(_IP), C.byref(o))
        _check(rc, "lp_create")
        self._h = h
        self.m, self.n = m, n
        self.options = o

    @classmethod
    def from_torch(cls, A, b, c, **kw):
        """A, b, c: float64 CUDA tensors; A of shape (m, n) in column-major memory order
        (A.t().contiguous().t(), i.e. stride (1, m))."""
        m, n = A.shape
        if A.dtype != b.dtype or A.dtype != c.dtype or str(A.dtype) != "torch.float64":
            raise TypeError("tensors must be float64")
        if not (A.is_cuda and b.is_cuda and c.is_cuda):
            raise TypeError("tensors must be on the GPU")
        if n > 1 and A.stride() != (1, m):
            raise ValueError("A must be column-major: stride (1, m)")
        return cls(device_tensors=(A.data_ptr(), b.data_ptr(), c.data_ptr(), m, n), **kw)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lp_destroy(h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, max_iter=None) -> int:
        st = C.c_int32()
        if max_iter is None:
            _check(lib().lp_solve(self._h, C.byref(st)), "lp_solve")
        else:
            _check(lib().lp_solve_until(self._h, int(max_iter), C.byref(st)), "lp_solve_until")
        return st.value

    def iterate(self, count) -> int:
        """Exactly `count` more pivots (fewer if the solve ends first); LP_RUNNING if it has not."""
        st = C.c_int32()
        _check(lib().lp_iterate(self._h, int(count), C.byref(st)), "lp_iterate")
        return st.value

    def reset(self):
        _check(lib().lp_reset(self._h), "lp_reset")

    def reinvert(self):
        _check(lib().lp_reinvert(self._h), "lp_reinvert")

    def solution(self):
        obj = C.c_double()
        x = np.empty(self.n)
        y = np.empty(self.m)
        basis = np.empty(self.m, dtype=np.int32)
        it = C.c_int64()
        _check(lib().lp_get_solution(self._h, C.byref(obj), _dptr(x), _dptr(y), basis.ctypes.data_as(_IP),
                                     C.byref(it)), "lp_get_solution")
        return dict(objective=obj.value, x=x, y=y, basis=basis, iterations=it.value)

    def pivots(self):
        cnt = C.c_int64()
        _check(lib().lp_get_pivots(self._h, None, None, None, None, 0, C.byref(cnt)), "lp_get_pivots")
        k = cnt.value
        arrs = [np.empty(k, dtype=np.int32) for _ in range(4)]
        _check(lib().lp_get_pivots(self._h, *[a.ctypes.data_as(_IP) for a in arrs], k, C.byref(cnt)),
               "lp_get_pivots")
        return dict(enter=arrs[0], row=arrs[1], leave=arrs[2], flags=arrs[3])

    def tableau(self):
        m = self.m
        Binv = np.empty((m, m))
        xB = np.empty(m)
        W = np.empty(m)
        z = C.c_double()
        _check(lib().lp_get_tableau(self._h, _dptr(Binv), _dptr(xB), _dptr(W), C.byref(z)), "lp_get_tableau")
        return Binv, xB, W, z.value

    def stats(self) -> dict:
        s = lp_stats()
        _check(lib().lp_get_stats(self._h, C.byref(s)), "lp_get_stats")
        return {f: getattr(s, f) for f, _ in lp_stats._fields_}


def solve_device_noalloc(A, b, c, x=None, y=None, objective=None, sense="max", **opts):
    """lp_solve_device_noalloc on torch CUDA tensors (A float64 of shape (m, n) with stride
    (1, m), b and c float64); x (n), y (m), objective (1): float64 CUDA tensors or None.
    Returns (status, iterations)."""
    m, n = A.shape
    for t in (A, b, c):
        if str(t.dtype) != "torch.float64" or not t.is_cuda:
            raise TypeError("A, b, c must be float64 CUDA tensors")
    if n > 1 and A.stride() != (1, m):
        raise ValueError("A must be column-major: stride (1, m)")
    for t, k in ((x, n), (y, m), (objective, 1)):
        if t is not None and (str(t.dtype) != "torch.float64" or not t.is_cuda or t.numel() != k
                              or not t.is_contiguous()):
            raise ValueError("outputs must be contiguous float64 CUDA tensors of n, m and 1 entries")
    o = default_options(sense=LP_MAX if sense == "max" else LP_MIN, **opts)
    st = C.c_int32()
    it = C.c_int64()
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    _check(lib().lp_solve_device_noalloc(m, n, A.data_ptr(), b.data_ptr(), c.data_ptr(), C.byref(o), ptr(x), ptr(y),
                                         ptr(objective), C.byref(st), C.byref(it)), "lp_solve_device_noalloc")
    return st.value, it.value


class Batch:
    """A batch of independent LPs (an lp_batch handle), solved in one persistent launch."""

    def __init__(self, lps, sense="max", **opts):
        """lps: sequence of (A, b, c) host arrays, A of shape (m_i, n_i)."""
        o = default_options(sense=LP_MAX if sense == "max" else LP_MIN, **opts)
        cnt = len(lps)
        As, bs, cs = [], [], []
        ms = np.empty(cnt, dtype=np.int32)
        ns = np.empty(cnt, dtype=np.int32)
        for i, (A, b, c) in enumerate(lps):
            A = np.asfortranarray(np.asarray(A, dtype=np.float64))
            As.append(A)
            bs.append(np.ascontiguousarray(b, dtype=np.float64))
            cs.append(np.ascontiguousarray(c, dtype=np.float64))
            ms[i], ns[i] = A.shape
            if bs[-1].shape != (ms[i],) or cs[-1].shape != (ns[i],):
                raise ValueError(f"LP {i}: shapes of A, b, c do not match")
        self._keep = (As, bs, cs, ms, ns)
        pa = (_DP * cnt)(*[_dptr(a) for a in As])
        pb = (_DP * cnt)(*[_dptr(a) for a in bs])
        pc = (_DP * cnt)(*[_dptr(a) for a in cs])
        h = _P()
        _check(lib().lp_batch_create(C.byref(h), cnt, ms.ctypes.data_as(_IP), ns.ctypes.data_as(_IP), pa, pb, pc,
                                     C.byref(o)), "lp_batch_create")
        self._h = h
        self.count, self.m, self.n = cnt, ms, ns

    @classmethod
    def dense(cls, count, seed, m_lo=16, m_hi=256, sense="max", **opts):
        """A batch of seeded dense LPs generated in device memory (lp_batch_create_dense)."""
        o = default_options(sense=LP_MAX if sense == "max" else LP_MIN, **opts)
        self = cls.__new__(cls)
        h = _P()
        _check(lib().lp_batch_create_dense(C.byref(h), int(count), int(seed) & ((1 << 64) - 1), int(m_lo), int(m_hi),
                                           C.byref(o)), "lp_batch_create_dense")
        self._h = h
        ms = np.empty(count, dtype=np.int32)
        ns = np.empty(count, dtype=np.int32)
        _check(lib().lp_batch_get_sizes(h, ms.ctypes.data_as(_IP), ns.ctypes.data_as(_IP)), "lp_batch_get_sizes")
        self._keep = None
        self.count, self.m, self.n = int(count), ms, ns
        return self

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lp_batch_destroy(h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self):
        _check(lib().lp_batch_solve(self._h), "lp_batch_solve")

    def tune_load(self, path):
        """Takes this device's records of a tune table file (before the first solve)."""
        _check(lib().lp_batch_tune_load(self._h, os.fsencode(path)), "lp_batch_tune_load")

    def tune_save(self, path):
        """Merges the tuned modes and threshold into a tune table file."""
        _check(lib().lp_batch_tune_save(self._h, os.fsencode(path)), "lp_batch_tune_save")

    def results(self):
        st = np.empty(self.count, dtype=np.int32)
        obj = np.empty(self.count)
        it = np.empty(self.count, dtype=np.int64)
        _check(lib().lp_batch_results(self._h, st.ctypes.data_as(_IP), _dptr(obj), it.ctypes.data_as(_LP)),
               "lp_batch_results")
        return dict(status=st, objective=obj, iterations=it)

    def get(self, i):
        m, n = int(self.m[i]), int(self.n[i])
        x = np.empty(n)
        basis = np.empty(m, dtype=np.int32)
        cnt = C.c_int64()
        _check(lib().lp_batch_get(self._h, i, _dptr(x), basis.ctypes.data_as(_IP), None, None, None, 0,
                                  C.byref(cnt)), "lp_batch_get")
        k = cnt.value
        arrs = [np.empty(k, dtype=np.int32) for _ in range(3)]
        _check(lib().lp_batch_get(self._h, i, None, None, *[a.ctypes.data_as(_IP) for a in arrs], k, C.byref(cnt)),
               "lp_batch_get")
        return dict(x=x, basis=basis, enter=arrs[0], row=arrs[1], flags=arrs[2])

    def stats(self) -> dict:
        s = lp_batch_stats()
        _check(lib().lp_batch_get_stats(self._h, C.byref(s)), "lp_batch_get_stats")
        return {f: getattr(s, f) for f, _ in lp_batch_stats._fields_}
