"""Whole-solve parity at the benchmark's sizes: the GPU path's pivot log against the oracle's,
stored by tests/golden/make_goldens.py (oracle and seeded generators only).

Each case regenerates the LP from its law and seed, solves it on the GPU in the
benchmark's launch configuration (16 iterations per status read-back) up to the stored
pivot count, and compares every pivot (entering variable, leaving row, leaving variable,
flags) element by element, then the status, the pivot count, the final basis and the
objective (relative 1e-9; the two sides sum their dot products in different orders).

The two sides sum in different orders, so a decision whose value lies within rounding
noise of its threshold can fall either way.  The oracle records each pivot's decision
margin (the distance of its closest threshold test or comparison).  Where the logs part,
the pivot must be one whose margin is below RISKY (half the thresholds' size, 5e-10): a
decision that close depends on the noise the basis inverse carries, and from there on
the two paths are different, equally valid, pivot sequences.  Every pivot before it must
match exactly; the test reports how many did and the smallest margin among them."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_goldens  # noqa: E402

pytestmark = pytest.mark.gpu

OBJ_RTOL = 1e-9
RISKY = 5e-10  # decision margin below which rounding may decide a pivot


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
    margin = np.array([np.inf if v is None else v for v in g["margin"]])
    first = k
    for key in ("enter", "row", "leave", "flags"):
        bad = np.flatnonzero(piv[key] != np.asarray(g[key], dtype=np.int32))
        if bad.size:
            first = min(first, int(bad[0]))
    matched_min = margin[:first].min() if first else np.inf
    if first < k:
        # The paths part at pivot `first`: allowed only where the oracle's decision was
        # within rounding reach of its threshold (the pivots before it are equal).
        _say(f"  logs equal for the first {first} of {k} pivots (smallest margin among them {matched_min:.3g}); "
             f"pivot {first} has margin {margin[first]:.3g}")
        assert margin[first] < RISKY, f"{name}: logs differ at pivot {first}, whose decision margin is {margin[first]}"
        assert lpg.STATUS_NAMES[st] == g["status"] or g["pivot_cap"], (lpg.STATUS_NAMES[st], g["status"])
        return
    _say(f"  logs equal for all {k} pivots; smallest decision margin {matched_min:.3g}")
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
