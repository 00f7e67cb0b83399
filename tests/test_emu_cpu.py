"""The library's own kernels run on the CPU (tests/emu: every GPU thread a fiber, device
allocations between guard pages), against the oracle: the launch sequence with the
ratio-test finish fused into pricing, ties and the leaving-side tabu list, the mixed form
with reinversion, the two-phase start, the batched solver and the entry point that
allocates nothing.  An out-of-bounds access ends the run with the kernel named, so these
also check bounds on the host.  Each case runs in its own process (the binding holds one
library per process)."""
import os
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "emu"))
import build as emu_build  # noqa: E402

pytestmark = pytest.mark.skipif(not os.path.exists(emu_build.CXX), reason="no clang++ for the emulation build")


@pytest.fixture(scope="module")
def emu_lib():
    return emu_build.build()


def _run(lib, body, timeout=600):
    code = textwrap.dedent(f"""
        import sys
        sys.path[:0] = [{ROOT!r}, {os.path.join(ROOT, "tests")!r}]
        import numpy as np
        import paper_1803_04378_amd.binding as binding
        binding._LIB_PATH = {lib!r}
        import lpgen, oracle
        import paper_1803_04378_amd as lpg
        def same_log(piv, ref):
            return all(np.array_equal(piv[k], getattr(ref, k)) for k in ("enter", "row", "leave", "flags"))
    """) + textwrap.dedent(body)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=timeout)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    return res.stdout


def test_fused_sequence_follows_oracle(emu_lib):
    """Dense and degenerate (ties, tabu list) LPs: pivot logs equal the oracle's, with
    launch sequences of 1, 3 and 16 iterations (every kernel of the FP64 sequence)."""
    out = _run(emu_lib, """
        for A, b, c in (lpgen.dense_lp(0, 64, 128), lpgen.degenerate_lp(0, 60, 120, budget_row=True)):
            ref = oracle.solve(A, b, c)
            for ips in (1, 3, 16):
                with lpg.LP(A, b, c, iters_per_sync=ips) as p:
                    st = p.solve(); piv = p.pivots(); sol = p.solution(); s = p.stats()
                assert st == ref.status and same_log(piv, ref), (ips, st, ref.status)
                assert s["ties"] == ref.counts["tie"] and s["list_clears"] == ref.counts["lclear"]
                assert abs(sol["objective"] - ref.objective) <= 1e-9 * max(1.0, abs(ref.objective))
        print("ok", ref.counts)
    """)
    assert "ok" in out


def test_mixed_form_and_two_phase(emu_lib):
    out = _run(emu_lib, """
        A, b, c = lpgen.dense_lp(1, 64, 128)
        ref = oracle.solve(A, b, c)
        with lpg.LP(A, b, c, precision="mixed", reinv_period=8) as p:
            st = p.solve(); sol = p.solution(); s = p.stats()
        assert st == ref.status and s["reinversions"] > 0 and s["reinv_failed"] == 0
        assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)
        A, b, c, rt = lpgen.general_lp(0, 40, 80)
        ref = oracle.solve(A, b, c, row_type=rt)
        with lpg.LP(A, b, c, row_type=rt) as p:
            st = p.solve(); piv = p.pivots()
        assert st == ref.status and same_log(piv, ref)
        print("ok")
    """)
    assert "ok" in out


def test_batch_and_noalloc_equal_the_handle_path(emu_lib):
    out = _run(emu_lib, """
        import ctypes as C
        lps = [lpgen.dense_lp(lpgen.instance_seed(5, i), 16 + 9 * i, 32 + 18 * i) for i in range(6)]
        with lpg.Batch(lps) as bt:
            bt.solve(); res = bt.results()
        L = lpg.lib()
        dp = lambda a: a.ctypes.data_as(C.c_void_p)
        for i, (A, b, c) in enumerate(lps):
            with lpg.LP(A, b, c) as p:
                st = p.solve(); sol = p.solution()
            assert res["status"][i] == st and res["objective"][i] == sol["objective"]
            # the allocation-free entry point (host pointers stand in for device ones here)
            m, n = A.shape
            Af = np.asfortranarray(A); x = np.full(n, np.nan); y = np.full(m, np.nan); obj = np.full(1, np.nan)
            s2 = C.c_int32(); it = C.c_int64(); o = binding.default_options()
            rc = L.lp_solve_device_noalloc(m, n, dp(Af), dp(b), dp(c), C.byref(o), dp(x), dp(y), dp(obj),
                                           C.byref(s2), C.byref(it))
            assert rc == 0 and s2.value == st and it.value == sol["iterations"]
            assert np.array_equal(x, sol["x"]) and np.array_equal(y, sol["y"]) and obj[0] == sol["objective"]
        print("ok")
    """)
    assert "ok" in out
