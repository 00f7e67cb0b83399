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


def _run(lib, body, timeout=600, env=None):
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
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=timeout,
                         env=dict(os.environ, **(env or {})))
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


def test_compact_columns_follow_oracle(emu_lib):
    """Rows of 1024 and more: the FP64 form keeps B^-1 as compact columns over the list D
    (k_update_c, and rho formed from them by the pricing kernels).  Pivot logs equal the
    oracle's on the nearly diagonal law (|D| grows by one per pivot, past the 512 entries a
    lane holds in registers and far past ld/8), on ties with the leaving-side list, and on a
    two-phase LP with a drive-out and a redundant row (the switch writes B^-1 out and
    compacts it again); the tableau read-back is B^-1 to rounding; an FP64 reinversion (B^-1 written
    out, reinverted, compacted) keeps the oracle's objective."""
    out = _run(emu_lib, """
        def check_inverse(p, A, basis):
            Binv = p.tableau()[0]
            m = A.shape[0]
            B = np.hstack([A, np.eye(m)])[:, basis]
            err = np.abs(Binv @ B - np.eye(m)).max()
            assert err < 1e-9, err
        A, b, c = lpgen.diagonal_lp(0, 1032, 520)
        ref = oracle.solve(A, b, c)
        with lpg.LP(A, b, c, iters_per_sync=64) as p:
            st = p.solve(); piv = p.pivots(); sol = p.solution()
            assert st == ref.status and same_log(piv, ref)
            assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)
            check_inverse(p, A, sol["basis"])
        A, b, c = lpgen.degenerate_lp(4, 1030, 100, budget_row=True)
        ref = oracle.solve(A, b, c)
        with lpg.LP(A, b, c, iters_per_sync=3) as p:
            st = p.solve(); piv = p.pivots(); s = p.stats()
        assert st == ref.status and same_log(piv, ref) and s["ties"] == ref.counts["tie"] > 0
        # plus an empty >= row and an empty = row, both with b = 0: phase 1 ends with their
        # artificial variables basic at zero; the first is driven out by its surplus
        # column, the second row is redundant
        A, b, c, rt = lpgen.general_lp(0, 1022, 60)
        A = np.vstack([A, np.zeros((2, 60))])
        b = np.concatenate([b, [0.0, 0.0]])
        rt = np.concatenate([rt, [1, 2]]).astype(np.int32)
        ref = oracle.solve(A, b, c, row_type=rt)
        with lpg.LP(A, b, c, row_type=rt) as p:
            st = p.solve(); piv = p.pivots(); s = p.stats()
        assert st == ref.status and same_log(piv, ref)
        assert s["drive_outs"] == int(np.count_nonzero(ref.flags & oracle.FLAG_DRIVEOUT)) > 0
        A, b, c = lpgen.diagonal_lp(1, 1032, 200)
        ref = oracle.solve(A, b, c)
        with lpg.LP(A, b, c, reinv_period=16) as p:
            st = p.solve(); sol = p.solution(); s = p.stats()
            assert st == ref.status and s["reinversions"] > 0 and s["reinv_failed"] == 0
            assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)
            check_inverse(p, A, sol["basis"])
        print("ok")
    """, timeout=900)
    assert "ok" in out


def test_compact_columns_batch_and_noalloc(emu_lib):
    """The batched solver sums over D in D order at any |D| on rows of 1024 and more, as the
    FP64 form does: its results equal lp_solve's bit for bit; so do the allocation-free
    entry point's."""
    out = _run(emu_lib, """
        import ctypes as C
        lps = [lpgen.diagonal_lp(1, 1032, 200), lpgen.dense_lp(7, 1024, 40),
               lpgen.degenerate_lp(5, 1030, 60, budget_row=True)]
        with lpg.Batch(lps) as bt:
            bt.solve(); res = bt.results()
            for i, (A, b, c) in enumerate(lps):
                with lpg.LP(A, b, c) as p:
                    st = p.solve(); sol = p.solution(); piv = p.pivots()
                g = bt.get(i)
                assert res["status"][i] == st and res["iterations"][i] == sol["iterations"]
                assert res["objective"][i] == sol["objective"]
                for k in ("enter", "row", "flags"):
                    assert np.array_equal(g[k], piv[k]), (i, k)
                assert np.array_equal(g["x"], sol["x"]) and np.array_equal(g["basis"], sol["basis"])
        L = lpg.lib()
        dp = lambda a: a.ctypes.data_as(C.c_void_p)
        A, b, c = lps[1]
        with lpg.LP(A, b, c) as p:
            st = p.solve(); sol = p.solution()
        m, n = A.shape
        Af = np.asfortranarray(A); x = np.full(n, np.nan); y = np.full(m, np.nan); obj = np.full(1, np.nan)
        s2 = C.c_int32(); it = C.c_int64(); o = binding.default_options()
        rc = L.lp_solve_device_noalloc(m, n, dp(Af), dp(b), dp(c), C.byref(o), dp(x), dp(y), dp(obj),
                                       C.byref(s2), C.byref(it))
        assert rc == 0 and s2.value == st and it.value == sol["iterations"]
        assert np.array_equal(x, sol["x"]) and np.array_equal(y, sol["y"]) and obj[0] == sol["objective"]
        print("ok")
    """, timeout=900)
    assert "ok" in out


def test_front_guards_after_a_stop(emu_lib):
    """Every allocation starts at a guard page (EMU_GUARD_FRONT), so an access one element
    before an array faults.  A solve that stops inside a launch sequence (phase 1 priced
    out optimal) leaves the deferred bookkeeping of its last fused pivot behind with no
    pivot pending (r = -1); after the phase switch, and when a solve resumes past its pivot
    limit or after a reinversion, the next update must not apply it."""
    out = _run(emu_lib, """
        A, b, c, rt = lpgen.general_lp(0, 40, 80)
        ref = oracle.solve(A, b, c, row_type=rt)
        for ips in (3, 16):
            with lpg.LP(A, b, c, row_type=rt, iters_per_sync=ips) as p:
                st = p.solve(); piv = p.pivots()
            assert st == ref.status and same_log(piv, ref), ips
        A, b, c = lpgen.dense_lp(2, 64, 128)
        ref = oracle.solve(A, b, c)
        with lpg.LP(A, b, c, iters_per_sync=4) as p:
            assert p.solve(7) == lpg.LP_ITER_LIMIT
            st = p.solve(); piv = p.pivots()
        assert st == ref.status and same_log(piv, ref)
        with lpg.LP(A, b, c, reinv_period=5, iters_per_sync=4) as p:
            st = p.solve(); sol = p.solution(); s = p.stats()
        assert st == ref.status and s["reinversions"] > 0
        assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)
        print("ok")
    """, env={"EMU_GUARD_FRONT": "1"})
    assert "ok" in out


def test_compact_columns_mixed_form(emu_lib):
    """The mixed form on compact columns (rows of 1024 and more): FP32 screening forms W_new
    from row r of Bc; without reinversion the pivots are the oracle's, with reinversion
    (B^-1 written out, reinverted, compacted) the objective is the oracle's and the tableau
    read-back is B^-1 to rounding."""
    out = _run(emu_lib, """
        A, b, c = lpgen.dense_lp(3, 1024, 200)
        ref = oracle.solve(A, b, c)
        with lpg.LP(A, b, c, precision="mixed", reinv_period=0, iters_per_sync=8) as p:
            st = p.solve(); piv = p.pivots()
        assert st == ref.status and same_log(piv, ref)
        A, b, c = lpgen.diagonal_lp(1, 1032, 300)
        ref = oracle.solve(A, b, c)
        with lpg.LP(A, b, c, precision="mixed", reinv_period=16, iters_per_sync=4) as p:
            st = p.solve(); sol = p.solution(); s = p.stats()
            assert st == ref.status and s["reinversions"] > 0 and s["reinv_failed"] == 0
            assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)
            Binv = p.tableau()[0]
        B = np.hstack([A, np.eye(A.shape[0])])[:, sol["basis"]]
        assert np.abs(Binv @ B - np.eye(A.shape[0])).max() < 1e-9
        print("ok")
    """, timeout=900)
    assert "ok" in out


def test_device_generated_batch_equals_host_arrays(emu_lib):
    """lp_batch_create_dense writes the batch law's LPs in device memory; a batch made from
    host arrays of the same law (tests' generator) solves to the same bits."""
    out = _run(emu_lib, """
        with lpg.Batch.dense(6, 11, 16, 64) as g:
            g.solve(); rg = g.results()
            lps = lpgen.batch_lps(11, 6, 16, 64)
            assert [A.shape for A, _, _ in lps] == list(zip(g.m.tolist(), g.n.tolist()))
            with lpg.Batch(lps) as h:
                h.solve(); rh = h.results()
                for k in ("status", "objective", "iterations"):
                    assert np.array_equal(rg[k], rh[k]), k
                for i in range(6):
                    assert np.array_equal(g.get(i)["x"], h.get(i)["x"])
        print("ok")
    """)
    assert "ok" in out
