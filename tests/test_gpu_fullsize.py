"""Full-size instances in the benchmark's launch configuration (iters_per_sync = 16).

The oracle cannot afford whole solves at these sizes (0.1-0.6 s per pivot on one CPU core),
so each case checks (a) the GPU's first pivots against the oracle's, pivot by pivot, and
(b) a certificate of the final answer that holds at any size and is recomputed on the
host from the GPU's final basis with dense linear algebra: KKT conditions for OPTIMAL, an
improving ray (d_q < 0 and B^-1 a_q <= 0) for UNBOUNDED."""
import sys

import numpy as np
import pytest

import lpgen
import oracle
from lputil import assert_kkt

pytestmark = pytest.mark.gpu


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


def _prefix_parity(A, b, c, piv, k):
    o = oracle.Oracle(A, b, c)
    o.run(k)
    ref = o.result()
    k = min(k, len(ref.enter))
    np.testing.assert_array_equal(piv["enter"][:k], ref.enter[:k])
    np.testing.assert_array_equal(piv["row"][:k], ref.row[:k])
    np.testing.assert_array_equal(piv["flags"][:k], ref.flags[:k])
    return ref


def _ray_certificate(A, c, basis, q):
    """d_q < 0 and B^-1 a_q has no entry above the pivot tolerance: x_q can grow forever."""
    m, n = A.shape
    M = np.hstack([A, np.eye(m)])
    chat = np.concatenate([-c, np.zeros(m)])
    B = M[:, basis]
    alpha = np.linalg.solve(B, M[:, q])
    pi = np.linalg.solve(B.T, chat[basis])
    dq = chat[q] - pi @ M[:, q]
    assert dq < -1e-9, dq
    assert alpha.max() <= 1e-7, alpha.max()


def _no_repeated_basis(n, m, enter, row):
    """Anti-cycling check over a whole pivot log: the basis (as a set) never repeats.  The set
    is tracked by an incremental XOR hash of per-variable random keys, verified exactly on
    any hash collision."""
    rng = np.random.default_rng(12345)
    keys = rng.integers(0, 2**63, size=n + m, dtype=np.int64)
    basis = list(range(n, n + m))
    h = int(np.bitwise_xor.reduce(keys[n:]))
    seen = {h: [0]}
    snapshots = {0: frozenset(basis)}
    for t, (q, r) in enumerate(zip(enter.tolist(), row.tolist()), start=1):
        h ^= int(keys[basis[r]]) ^ int(keys[q])
        basis[r] = q
        if h in seen:
            cur = frozenset(basis)
            for t0 in seen[h]:
                if snapshots.get(t0) == cur:
                    raise AssertionError(f"basis at pivot {t} repeats pivot {t0}")
            seen[h].append(t)
            snapshots[t] = cur
        else:
            seen[h] = [t]
    return True


def _feasible_state(A, b, c, p, basis):
    _, xB, W, _ = p.tableau()
    m = A.shape[0]
    M = np.hstack([A, np.eye(m)])
    B = M[:, basis]
    xt = np.linalg.solve(B, b)
    assert xB.min() >= 0.0
    assert np.abs(xB - xt).max() <= 1e-6 * (1.0 + np.abs(xt).max())
    chat = np.concatenate([-c, np.zeros(m)])
    Wt = np.linalg.solve(B.T, chat[basis])
    assert np.abs(W - Wt).max() <= 1e-6 * (1.0 + np.abs(Wt).max())


def test_degenerate_5000x10000(lpg):
    """The degenerate law at full size opens with a long run of degenerate pivots (1500 rows
    with b_i = 0), so it runs to a pivot budget: the tabu rule must keep every basis new,
    and at the stop the basis must be primal feasible with x_B = B^-1 b."""
    _say("case: degenerate law m=5000 n=10000 seed 0, up to 40000 pivots")
    A, b, c = lpgen.degenerate_lp(0, 5000, 10000)
    with lpg.LP(A, b, c, iters_per_sync=16) as p:
        st = p.solve(40000)
        sol = p.solution()
        piv = p.pivots()
        stats = p.stats()
        _say(f"  status {st} after {sol['iterations']} pivots; degenerate {stats['degenerate']} ties {stats['ties']}")
        _prefix_parity(A, b, c, piv, 25)
        assert stats["degenerate"] > 0 and stats["ties"] > 0
        assert _no_repeated_basis(A.shape[1], A.shape[0], piv["enter"], piv["row"])
        if st == oracle.UNBOUNDED:
            _ray_certificate(A, c, sol["basis"], stats["ray"])
        else:
            assert st in (oracle.ITER_LIMIT, oracle.OPTIMAL)
            _feasible_state(A, b, c, p, sol["basis"])


def test_degenerate_500x1000_full_parity(lpg):
    """The literal degenerate law at a size the oracle finishes: whole pivot sequence, then
    the unboundedness certificate."""
    _say("case: degenerate law m=500 n=1000 seed 0, full parity")
    A, b, c = lpgen.degenerate_lp(0, 500, 1000)
    ref = oracle.solve(A, b, c)
    with lpg.LP(A, b, c, iters_per_sync=16) as p:
        st = p.solve()
        sol = p.solution()
        piv = p.pivots()
        stats = p.stats()
    np.testing.assert_array_equal(piv["enter"], ref.enter)
    np.testing.assert_array_equal(piv["row"], ref.row)
    np.testing.assert_array_equal(piv["flags"], ref.flags)
    assert st == ref.status == oracle.UNBOUNDED and stats["ray"] == ref.ray
    _ray_certificate(A, c, sol["basis"], stats["ray"])


def test_degenerate_budget_5001x10000_budgeted(lpg):
    """The bounded companion stalls for long stretches under Dantzig + tabu (pivot counts grow
    steeply with m on this law), so it runs to a fixed pivot budget; at the stop the basis
    must still be primal feasible and x_B must equal B^-1 b."""
    _say("case: degenerate law + budget row, m=5001 n=10000 seed 0, 20000 pivots")
    A, b, c = lpgen.degenerate_lp(0, 5000, 10000, budget_row=True)
    with lpg.LP(A, b, c, iters_per_sync=16) as p:
        st = p.solve(20000)
        sol = p.solution()
        piv = p.pivots()
        stats = p.stats()
        _say(f"  status {st} after {sol['iterations']} pivots; degenerate {stats['degenerate']} ties {stats['ties']}")
        _prefix_parity(A, b, c, piv, 25)
        assert st in (oracle.ITER_LIMIT, oracle.OPTIMAL)
        assert stats["degenerate"] > 0 and stats["ties"] > 0
        assert _no_repeated_basis(A.shape[1], A.shape[0], piv["enter"], piv["row"])
        _feasible_state(A, b, c, p, sol["basis"])


def test_dense_8000x16000_optimal(lpg):
    _say("case: dense law m=8000 n=16000 seed 0")
    A, b, c = lpgen.dense_lp(0, 8000, 16000)
    with lpg.LP(A, b, c, iters_per_sync=16) as p:
        st = p.solve()
        sol = p.solution()
        piv = p.pivots()
    _say(f"  status {st} after {sol['iterations']} pivots, objective {sol['objective']}")
    _prefix_parity(A, b, c, piv, 12)
    assert st == oracle.OPTIMAL
    assert_kkt(A, b, c, sol["x"], sol["y"])


def test_degenerate_budget_500_full_parity(lpg):
    """A mid-size degenerate LP the oracle can finish: the whole pivot sequence."""
    _say("case: degenerate law + budget row, m=501 n=1000 seed 0, full parity")
    A, b, c = lpgen.degenerate_lp(0, 500, 1000, budget_row=True)
    ref = oracle.solve(A, b, c)
    with lpg.LP(A, b, c, iters_per_sync=16) as p:
        st = p.solve()
        sol = p.solution()
        piv = p.pivots()
    np.testing.assert_array_equal(piv["enter"], ref.enter)
    np.testing.assert_array_equal(piv["row"], ref.row)
    np.testing.assert_array_equal(piv["flags"], ref.flags)
    assert st == ref.status == oracle.OPTIMAL
    assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)


def test_max_rows(lpg):
    """m = LP_MAX_ROWS (the largest m whose pricing kernel stages W in the LDS of one CU; the
    update kernel stages its vectors in chunks there): the solve runs and takes the
    oracle's pivots; one row more is rejected."""
    m, n = lpg.binding.LP_MAX_ROWS, 24
    _say(f"case: dense law m={m} n={n} seed 0 (LP_MAX_ROWS)")
    A, b, c = lpgen.dense_lp(0, m, n)
    ref = oracle.solve(A, b, c, lib_path=oracle.omp_lib())
    with lpg.LP(A, b, c) as p:
        st = p.solve()
        piv = p.pivots()
        sol = p.solution()
    assert st == ref.status == lpg.LP_OPTIMAL
    for k in ("enter", "row", "leave", "flags"):
        assert np.array_equal(piv[k], getattr(ref, k)), k
    assert abs(sol["objective"] - ref.objective) <= 1e-9 * abs(ref.objective)
    A1, b1, c1 = lpgen.dense_lp(0, m + 1, 2)
    with pytest.raises(lpg.LPError):
        lpg.LP(A1, b1, c1)
