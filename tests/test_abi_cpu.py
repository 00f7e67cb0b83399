"""The C-ABI library loads and exports every symbol its header declares; host-side argument
checks run without a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1803_04378_amd as lpg
from paper_1803_04378_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lpgpu.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    names = _declared()
    assert {"lp_create", "lp_solve", "lp_get_solution", "lp_destroy"} <= set(names)
    L = lpg.lib()
    for name in names:
        assert hasattr(L, name), name
        assert name in binding.SIGNATURES, f"binding lacks {name}"
    assert set(binding.SIGNATURES) == set(names)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define (LP_[A-Z_]+) \(?(-?\d+)\)?", text))
    for k, v in consts.items():
        if hasattr(binding, k):
            assert getattr(binding, k) == int(v), k


def test_struct_layouts():
    assert C.sizeof(binding.lp_options) == 104
    assert C.sizeof(binding.lp_batch_stats) == 96
    assert C.sizeof(binding.lp_stats) == 256


def test_default_options():
    o = lpg.default_options()
    assert o.sense == binding.LP_MAX and o.tabu_tenure == 5 and o.leaving_list == 1
    assert o.eps_d == 1e-9 and o.eps_p == 1e-9 and o.eps_z == 1e-9 and o.eps_t == 1e-9 and o.max_iter == 0 and o.batch_small_m == -1
    assert o.batch_binv_lds_m == -1
    assert o.precision == binding.LP_FP64 and o.shortlist_k == 16 and o.reinv_period == -1
    assert lpg.lib().lp_default_options(None) == binding.LP_ERR_ARG


def _create(m, n, A, b, c, opt=None):
    h = C.c_void_p()
    rc = lpg.lib().lp_create(C.byref(h), m, n, A, b, c, opt)
    return rc, h


def test_argument_errors_need_no_gpu():
    L = lpg.lib()
    A = np.ones((3, 2), order="F")
    b = np.ones(3)
    c = np.ones(2)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    assert _create(0, 2, dp(A), dp(b), dp(c))[0] == binding.LP_ERR_ARG
    assert _create(3, -1, dp(A), dp(b), dp(c))[0] == binding.LP_ERR_ARG
    assert _create(3, 2, None, dp(b), dp(c))[0] == binding.LP_ERR_ARG
    assert _create(binding.LP_MAX_ROWS + 1, 2, dp(A), dp(b), dp(c))[0] == binding.LP_ERR_ARG
    bn = b.copy()
    bn[1] = -1.0
    rc, h = _create(3, 2, dp(A), dp(bn), dp(c))
    assert rc == binding.LP_ERR_NEG_RHS and not h.value
    assert "negative" in L.lp_error_string(rc).decode()
    An = A.copy(order="F")
    An[2, 1] = np.inf
    assert _create(3, 2, dp(An), dp(b), dp(c))[0] == binding.LP_ERR_ARG
    o = lpg.default_options(iters_per_sync=0)
    assert _create(3, 2, dp(A), dp(b), dp(c), C.byref(o))[0] == binding.LP_ERR_ARG
    o = lpg.default_options(sense=7)
    assert _create(3, 2, dp(A), dp(b), dp(c), C.byref(o))[0] == binding.LP_ERR_ARG
    for bad in (dict(precision=2), dict(shortlist_k=0), dict(shortlist_k=17), dict(reinv_period=-2)):
        o = lpg.default_options(**bad)
        assert _create(3, 2, dp(A), dp(b), dp(c), C.byref(o))[0] == binding.LP_ERR_ARG, bad
    with pytest.raises(ValueError):
        lpg.LP(A, b, c, precision="fp16")
    assert L.lp_solve(None, None) == binding.LP_ERR_ARG
    L.lp_destroy(None)  # NULL-safe
    with pytest.raises(lpg.LPError):
        lpg.LP(A, bn, c)


def test_general_create_argument_errors_need_no_gpu():
    L = lpg.lib()
    A = np.ones((3, 2), order="F")
    b = np.array([1.0, -2.0, 0.5])
    c = np.ones(2)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))

    def create(m, n, A_, b_, c_, rt, o=None):
        h = C.c_void_p()
        return L.lp_create_general(C.byref(h), m, n, A_, b_, c_, rt, o), h

    rt = np.array([binding.LP_ROW_LE, binding.LP_ROW_GE, binding.LP_ROW_EQ], dtype=np.int32)
    assert L.lp_create_general(None, 3, 2, dp(A), dp(b), dp(c), ip(rt), None) == binding.LP_ERR_ARG
    assert create(0, 2, dp(A), dp(b), dp(c), ip(rt))[0] == binding.LP_ERR_ARG
    assert create(3, 2, None, dp(b), dp(c), ip(rt))[0] == binding.LP_ERR_ARG
    bad = rt.copy()
    bad[1] = 3
    rc, h = create(3, 2, dp(A), dp(b), dp(c), ip(bad))
    assert rc == binding.LP_ERR_ARG and not h.value
    assert "row type" in L.lp_error_string(rc).decode()
    bi = b.copy()
    bi[0] = np.nan
    assert create(3, 2, dp(A), dp(bi), dp(c), ip(rt))[0] == binding.LP_ERR_ARG
    An = A.copy(order="F")
    An[1, 0] = np.inf
    assert create(3, 2, dp(An), dp(b), dp(c), ip(rt))[0] == binding.LP_ERR_ARG
    o = lpg.default_options(iters_per_sync=0)
    assert create(3, 2, dp(A), dp(b), dp(c), ip(rt), C.byref(o))[0] == binding.LP_ERR_ARG
    with pytest.raises(ValueError):
        lpg.LP(A, b, c, row_type=[0, 1])


def test_error_strings():
    L = lpg.lib()
    for code in (0, -1, -2, -3, -4, -5, 99):
        assert isinstance(L.lp_error_string(code), bytes)


def test_batch_argument_errors_need_no_gpu():
    L = lpg.lib()
    A = np.ones((3, 2), order="F")
    b = np.ones(3)
    c = np.ones(2)
    dp = C.POINTER(C.c_double)
    ms = (C.c_int32 * 2)(3, 3)
    ns = (C.c_int32 * 2)(2, 2)
    pa = (dp * 2)(A.ctypes.data_as(dp), A.ctypes.data_as(dp))
    pb = (dp * 2)(b.ctypes.data_as(dp), b.ctypes.data_as(dp))
    pc = (dp * 2)(c.ctypes.data_as(dp), c.ctypes.data_as(dp))
    h = C.c_void_p()
    assert L.lp_batch_create(C.byref(h), 0, ms, ns, pa, pb, pc, None) == binding.LP_ERR_ARG
    bn = -b
    pbn = (dp * 2)(b.ctypes.data_as(dp), bn.ctypes.data_as(dp))
    assert L.lp_batch_create(C.byref(h), 2, ms, ns, pa, pbn, pc, None) == binding.LP_ERR_NEG_RHS
    big = (C.c_int32 * 2)(3, 5000)
    Abig = np.ones((5000, 2), order="F")
    bbig = np.ones(5000)
    pa2 = (dp * 2)(A.ctypes.data_as(dp), Abig.ctypes.data_as(dp))
    pb2 = (dp * 2)(b.ctypes.data_as(dp), bbig.ctypes.data_as(dp))
    assert L.lp_batch_create(C.byref(h), 2, big, ns, pa2, pb2, pc, None) == binding.LP_ERR_ARG
    o = lpg.default_options(precision=binding.LP_MIXED)
    assert L.lp_batch_create(C.byref(h), 2, ms, ns, pa, pb, pc, C.byref(o)) == binding.LP_ERR_ARG
    assert L.lp_batch_solve(None) == binding.LP_ERR_ARG
    assert L.lp_reinvert(None) == binding.LP_ERR_ARG
    L.lp_batch_destroy(None)


_HUGE_CREATE = r"""
import ctypes as C, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_1803_04378_amd import binding
L = binding.lib()
m, n = binding.LP_MAX_ROWS, 500_000_000  # the normal form alone needs m * n doubles (39 TB)
b, A, c = np.ones(m), np.ones(4), np.ones(4)
dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
h = C.c_void_p()
rc = L.lp_create_general(C.byref(h), m, n, dp(A), dp(b), dp(c), None, None)
print(rc, bool(h.value), L.lp_error_string(rc).decode())
"""


def test_host_allocation_failure_is_an_error_code():
    """A host allocation that fails inside an entry point comes back as LP_ERR_NOMEM, not as
    an exception unwinding through the C ABI (which aborts the process).  Run in a child
    process so that a regression cannot take the test runner down."""
    import subprocess
    import sys
    try:
        mode = open("/proc/sys/vm/overcommit_memory").read().strip()
    except OSError:
        mode = "?"
    if mode not in ("0", "2"):
        pytest.skip("the kernel may grant a 39 TB allocation (overcommit_memory = %s)" % mode)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", _HUGE_CREATE, root], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    rc, handed, msg = out.stdout.strip().split(" ", 2)
    assert int(rc) == binding.LP_ERR_NOMEM and handed == "False"
    assert "host allocation failed" in msg
