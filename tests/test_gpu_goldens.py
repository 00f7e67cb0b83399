"""Whole-solve parity at the benchmark's sizes: the GPU path's pivot log against the oracle's,
stored by tests/golden/make_goldens.py (oracle and seeded generators only).

Each case regenerates the LP from its law and seed, solves it on the GPU in the
benchmark's launch configuration (16 iterations per status read-back) up to the stored
pivot count, and compares every pivot (entering variable, leaving row, leaving variable,
flags) element by element, then the status, the pivot count, the final basis and the
objective (relative 1e-9; the two sides sum their dot products in different orders)."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_goldens  # noqa: E402

pytestmark = pytest.mark.gpu

OBJ_RTOL = 1e-9


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def lpg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_04378_amd as mod
    mod.lib()
    return mod


def _compare(name, g, piv, st, sol, lpg):
    k = g["iterations"]
    assert len(piv["enter"]) == k, f"{name}: {len(piv['enter'])} pivots, oracle {k}"
    for key in ("enter", "row", "leave", "flags"):
        got, want = piv[key], np.asarray(g[key], dtype=np.int32)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, f"{name}: {key} differs first at pivot {bad[0]}: {got[bad[0]]} vs {want[bad[0]]}"
    assert lpg.STATUS_NAMES[st] == g["status"], (lpg.STATUS_NAMES[st], g["status"])
    np.testing.assert_array_equal(sol["basis"], np.asarray(g["basis"], dtype=np.int32))
    if g["status"] == "OPTIMAL":
        rel = abs(sol["objective"] - g["objective"]) / max(1.0, abs(g["objective"]))
        _say(f"  objective {sol['objective']!r} vs oracle {g['objective']!r}: relative {rel:.2e}")
        assert rel <= OBJ_RTOL


# Cases whose kernels are switched off in the library: rows above LP_MAX_ROWS (the chunked
# update kernel) and, near the row limit, sparse-column mode with more than 2B entries of D.
# A GPU run that first exercised these paths (with others new at the time) faulted the
# device without output naming the kernel; the CPU emulation of the kernels found no
# out-of-bounds access, so they stay off until they are validated on the device.
SWITCHED_OFF = {"dense_m12000_n150_s0", "diagonal_m12000_n1600_s0", "diagonal_m9700_n1300_s0"}


@pytest.mark.parametrize("name", [pytest.param(n, marks=pytest.mark.skip(reason="kernel path switched off until "
                                                                            "validated on the device"))
                                  if n in SWITCHED_OFF else n for n in make_goldens.GOLDENS])
def test_gpu_follows_oracle_log(lpg, name):
    g = make_goldens.load(name)
    law, seed, m, n, cap, what = make_goldens.GOLDENS[name]
    _say(f"case: {name} ({what}), {g['iterations']} oracle pivots, status {g['status']}")
    A, b, c = make_goldens.make(law, seed, m, n)
    with lpg.LP(A, b, c, iters_per_sync=16) as p:
        st = p.solve(g["iterations"] if g["pivot_cap"] else None)
        piv = p.pivots()
        sol = p.solution()
        stats = p.stats()
    _say(f"  GPU: status {lpg.STATUS_NAMES[st]} after {sol['iterations']} pivots, {stats['solve_ms']:.1f} ms")
    _compare(name, g, piv, st, sol, lpg)
