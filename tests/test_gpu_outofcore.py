"""The out-of-core mode of Section 3 (Case 2, Figures 2 and 4): with a device-memory budget
below the tableau's size, B^-1 lives in pinned host memory in panels of consecutive rows
that every iteration streams through the device, the last panel staying resident.  The
pivots must still be the oracle's, and every result must equal the in-memory path's
(Case 1) bit for bit: the arithmetic of every row is the same."""
import sys

import numpy as np
import pytest

import lpgen
import oracle

# Case 2 is switched off in the library (an LP beyond the budget gets LP_ERR_NOMEM): a GPU run
# that exercised it, among other paths new at the time, faulted the device with no output to
# name the failing kernel, and the CPU emulation of the kernels found no out-of-bounds access.
pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="out-of-core panel mode switched off until it is validated "
                                                       "on the device (unexplained device fault in the run that "
                                                       "first exercised it)")]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lpg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_04378_amd as mod
    mod.lib()
    return mod


def _budget(m, n, panel_rows):
    """Device bytes for A', the vectors, the pivot log and three panels of panel_rows rows
    (the library reserves a little more for its partial results)."""
    ld = (m + 7) // 8 * 8
    max_iter = 10 * (m + n)
    return 8 * ld * n + 64 * (n + m) + 64 * ld + 64 * max_iter + 3 * 8 * ld * panel_rows + 300_000


@pytest.mark.parametrize("m,n,seed,rows", [(1000, 2000, 0, 120), (2000, 4000, 1, 300), (1500, 700, 2, 100)])
def test_panels_follow_the_oracle(lpg, m, n, seed, rows):
    A, b, c = lpgen.dense_lp(seed, m, n)
    _say(f"case: out-of-core panels, dense m={m} n={n} seed {seed}, ~{rows} rows per panel")
    ref = oracle.solve(A, b, c)
    with lpg.LP(A, b, c, device_budget=_budget(m, n, rows)) as p:
        st = p.solve()
        piv = p.pivots()
        sol = p.solution()
        stats = p.stats()
        tab = p.tableau()
    _say(f"  case {stats['memory_case']}: {stats['panels']} panels of {stats['panel_rows']} rows; "
         f"{sol['iterations']} pivots in {stats['solve_ms']:.1f} ms")
    assert stats["memory_case"] == 2 and stats["panels"] >= 3
    assert st == ref.status == oracle.OPTIMAL
    for k in ("enter", "row", "leave", "flags"):
        np.testing.assert_array_equal(piv[k], getattr(ref, k), err_msg=k)
    assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)
    with lpg.LP(A, b, c) as p1:
        assert p1.solve() == st
        assert p1.stats()["memory_case"] == 1
        sol1 = p1.solution()
        tab1 = p1.tableau()
    assert sol1["objective"] == sol["objective"]
    np.testing.assert_array_equal(sol1["x"], sol["x"])
    for t0, t1 in zip(tab, tab1):
        np.testing.assert_array_equal(t0, t1)


def test_panels_step_reset_and_degenerate_law(lpg):
    """Stepping with lp_iterate, a reset, and ties on the degenerate law (every decision of
    the ratio test reduces partials from every panel)."""
    A, b, c = lpgen.degenerate_lp(9, 150, 300)
    ref = oracle.solve(A, b, c)
    m, n = A.shape
    with lpg.LP(A, b, c, device_budget=_budget(m, n, 16)) as p:
        assert p.stats()["panels"] >= 8
        for k in (1, 7, 30):
            assert p.iterate(k) == lpg.LP_RUNNING
        st = p.solve()
        piv = p.pivots()
        np.testing.assert_array_equal(piv["row"], ref.row)
        np.testing.assert_array_equal(piv["flags"], ref.flags)
        assert st == ref.status
        p.reset()
        assert p.solve() == st
        np.testing.assert_array_equal(p.pivots()["enter"], ref.enter)


def test_panel_mode_limits(lpg):
    A, b, c = lpgen.dense_lp(3, 600, 900)
    m, n = A.shape
    with pytest.raises(lpg.LPError):  # the mixed form reinverts: it needs B^-1 in device memory
        lpg.LP(A, b, c, precision="mixed", device_budget=_budget(m, n, 50))
    with pytest.raises(lpg.LPError) as e:  # not even A' fits
        lpg.LP(A, b, c, device_budget=8 * 600 * 900 // 2)
    assert e.value.code == lpg.binding.LP_ERR_NOMEM
    rt = np.zeros(m, dtype=np.int32)
    rt[0] = 1
    with pytest.raises(lpg.LPError):
        lpg.LP(A, b, c, row_type=rt, device_budget=_budget(m, n, 50))
