"""Parity of the HIP path (through the C ABI) with the CPU oracle.

The FP64 GPU path must take the oracle's pivots exactly (entering variable, leaving row,
leaving variable, flags), reach the same status, and match the oracle's objective to
1e-9 relative.  Both sides take every pivot decision in FP64; their dot products sum in
different orders, so values agree to rounding, not bit for bit, and the tolerances
below are stated per quantity."""
import json
import os
import sys

import numpy as np
import pytest

import lpgen
import oracle
from lputil import assert_kkt

pytestmark = pytest.mark.gpu

OBJ_RTOL = 1e-9


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


def _gpu(lpg, A, b, c, max_iter=None, **opts):
    sense = opts.pop("sense", "max")
    with lpg.LP(A, b, c, sense=sense, **opts) as p:
        st = p.solve(max_iter)
        sol = p.solution()
        piv = p.pivots()
        stats = p.stats()
    return st, sol, piv, stats


def assert_parity(lpg, A, b, c, max_iter=None, tenure=5, leaving_list=True, sense="max", **gpu_opts):
    m, n = A.shape
    _say(f"parity case m={m} n={n} tenure={tenure} list={leaving_list} sense={sense} {gpu_opts}")
    ref = oracle.solve(A, b, c, sense=sense, max_iter=max_iter, tenure=tenure, leaving_list=leaving_list)
    st, sol, piv, stats = _gpu(lpg, A, b, c, max_iter=max_iter, tabu_tenure=tenure, leaving_list=int(leaving_list),
                               sense=sense, **gpu_opts)
    k = min(len(ref.enter), len(piv["enter"]))
    for name, a, g in (("enter", ref.enter, piv["enter"]), ("row", ref.row, piv["row"]),
                       ("leave", ref.leave, piv["leave"]), ("flags", ref.flags, piv["flags"])):
        diff = np.nonzero(a[:k] != g[:k])[0]
        assert diff.size == 0, f"first {name} divergence at pivot {diff[0]}: oracle {a[diff[0]]} gpu {g[diff[0]]}"
    assert len(ref.enter) == len(piv["enter"]) == sol["iterations"], (len(ref.enter), len(piv["enter"]))
    assert st == ref.status, (st, ref.status)
    assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * max(1.0, abs(ref.objective))
    np.testing.assert_array_equal(sol["basis"], ref.basis)
    scale = 1.0 + np.abs(ref.x).max(initial=0.0)
    assert np.abs(sol["x"] - ref.x).max(initial=0.0) <= 1e-9 * scale
    assert np.abs(sol["y"] - ref.y).max(initial=0.0) <= 1e-9 * (1.0 + np.abs(ref.y).max(initial=0.0))
    assert stats["degenerate"] == ref.counts["degenerate"] and stats["ties"] == ref.counts["tie"]
    assert stats["aspirations"] == ref.counts["aspiration"] and stats["list_clears"] == ref.counts["lclear"]
    if len(ref.margin):
        # how close the closest decision of the run came to its threshold (oracle's values)
        _say(f"  exact over {len(ref.enter)} pivots; smallest decision margin {ref.margin.min():.3g} "
             f"(pivot {int(np.argmin(ref.margin))})")
    return ref, (st, sol, piv, stats)


@pytest.mark.parametrize("seed", range(10))
def test_dense_64x128(lpg, seed):
    A, b, c = lpgen.dense_lp(seed, 64, 128)
    ref, (st, sol, _, _) = assert_parity(lpg, A, b, c)
    assert st == oracle.OPTIMAL
    assert_kkt(A, b, c, sol["x"], sol["y"])


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (2, 3), (7, 9), (9, 7), (63, 65), (65, 63), (100, 130),
                                 (130, 257), (257, 130), (300, 601)])
def test_dense_ragged_shapes(lpg, m, n):
    A, b, c = lpgen.dense_lp(m * 1000 + n, m, n)
    assert_parity(lpg, A, b, c)


NUMERICAL_LPS = [
    # the only ratio is 1e301 / 1e-8 = inf
    (np.array([[1e-8]]), np.array([1e301]), np.array([1.0])),
    # a degenerate pivot on alpha_r = 1e-8 drives B^-1[1,0] to -inf; the next FTRAN gives NaN
    (np.array([[1e-8, 0.0], [1e301, 1.0]]), np.array([0.0, 1.0]), np.array([1.0, 1.0])),
]


@pytest.mark.parametrize("case", range(len(NUMERICAL_LPS)))
@pytest.mark.parametrize("ips", [1, 16])
def test_numerical_status_matches_oracle(lpg, case, ips):
    """Overflow stops the solve with NUMERICAL at the same pivot as the oracle; a second
    solve call on the stopped handle reports it again without pivoting."""
    A, b, c = NUMERICAL_LPS[case]
    ref, (st, sol, piv, _) = assert_parity(lpg, A, b, c, iters_per_sync=ips)
    assert st == oracle.NUMERICAL == lpg.LP_NUMERICAL
    with lpg.LP(A, b, c, iters_per_sync=ips) as p:
        assert p.solve() == lpg.LP_NUMERICAL
        assert p.solve() == lpg.LP_NUMERICAL
        assert p.solution()["iterations"] == len(ref.enter)


@pytest.mark.parametrize("m,seed", [(60, 0), (100, 1), (150, 2), (200, 3)])
def test_degenerate_budget_law(lpg, m, seed):
    """Ties, degenerate pivots, the leaving-side tabu list and aspiration all occur here."""
    A, b, c = lpgen.degenerate_lp(seed, m, 2 * m, budget_row=True)
    ref, _ = assert_parity(lpg, A, b, c)
    assert ref.counts["degenerate"] > 0 and ref.counts["tie"] > 0


@pytest.mark.parametrize("m,seed", [(100, 0), (250, 0), (250, 1)])
def test_degenerate_law_status(lpg, m, seed):
    A, b, c = lpgen.degenerate_lp(seed, m, 2 * m)
    assert_parity(lpg, A, b, c)


def _cyc(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", "cycling_lps.json")) as f:
        d = json.load(f)[name]
    return np.array(d["A"], float), np.array(d["b"], float), np.array(d["c"], float), d["optimum"]


@pytest.mark.parametrize("name", ["chvatal", "beale"])
def test_cycling_lps(lpg, name):
    A, b, c, opt = _cyc(name)
    ref, (st, sol, _, _) = assert_parity(lpg, A, b, c)
    assert st == oracle.OPTIMAL and abs(sol["objective"] - opt) < 1e-12
    # plain Dantzig cycles on the GPU exactly as in the oracle
    assert_parity(lpg, A, b, c, max_iter=40, tenure=0, leaving_list=False)


@pytest.mark.parametrize("name", ["chvatal", "beale"])
def test_embedded_cycling_lp(lpg, name):
    from test_oracle_pins import _embedded
    A, b, c = _embedded(name)
    assert_parity(lpg, A, b, c)
    assert_parity(lpg, A, b, c, max_iter=300, tenure=0, leaving_list=False)


def test_unbounded_and_trivial(lpg):
    A, b, c = lpgen.dense_lp(2, 20, 30)
    A[:, 5] = -np.abs(A[:, 5])
    c[5] = 100.0
    ref, (st, _, _, stats) = assert_parity(lpg, A, b, c)
    assert st == oracle.UNBOUNDED and stats["ray"] == ref.ray == 5
    A, b, c = lpgen.dense_lp(3, 20, 30)
    _, (st, sol, _, _) = assert_parity(lpg, A, b, -c)
    assert st == oracle.OPTIMAL and sol["iterations"] == 0
    A, b, c = lpgen.dense_lp(4, 40, 70)
    assert_parity(lpg, A, b, -c, sense="min")
    b[:5] = 0.0
    assert_parity(lpg, A, b, c)


@pytest.mark.parametrize("k", [1, 3, 16, 64])
def test_iters_per_sync_does_not_change_results(lpg, k):
    A, b, c = lpgen.degenerate_lp(6, 120, 240, budget_row=True)
    assert_parity(lpg, A, b, c, iters_per_sync=k)


def test_resume_after_iter_limit(lpg):
    A, b, c = lpgen.degenerate_lp(5, 80, 160, budget_row=True)
    full = oracle.solve(A, b, c)
    with lpg.LP(A, b, c) as p:
        for cap in (1, 7, 8, 30):
            assert p.solve(cap) == oracle.ITER_LIMIT
            assert p.solution()["iterations"] == cap
        st = p.solve()
        piv = p.pivots()
        sol = p.solution()
    assert st == full.status
    np.testing.assert_array_equal(piv["enter"], full.enter)
    np.testing.assert_array_equal(piv["row"], full.row)
    assert abs(sol["objective"] - full.objective) <= OBJ_RTOL * abs(full.objective)


def test_reset_and_repeat_is_deterministic(lpg):
    A, b, c = lpgen.dense_lp(11, 300, 600)
    with lpg.LP(A, b, c) as p:
        p.solve()
        s1 = p.solution()
        l1 = p.pivots()
        p.reset()
        assert p.solution()["iterations"] == 0
        p.solve()
        s2 = p.solution()
        l2 = p.pivots()
    assert s1["objective"] == s2["objective"]
    np.testing.assert_array_equal(s1["x"], s2["x"])
    np.testing.assert_array_equal(l1["enter"], l2["enter"])


def test_tableau_matches_oracle(lpg):
    A, b, c = lpgen.degenerate_lp(8, 90, 180, budget_row=True)
    o = oracle.Oracle(A, b, c)
    with lpg.LP(A, b, c) as p:
        for cap in (1, 2, 10, 25):
            o.run(cap)
            p.solve(cap)
            Bo, xo, Wo, zo = o.state()
            Bg, xg, Wg, zg = p.tableau()
            assert np.abs(Bg - Bo).max() <= 1e-12 * (1 + np.abs(Bo).max())
            assert np.abs(xg - xo).max() <= 1e-12 * (1 + np.abs(xo).max())
            assert np.abs(Wg - Wo).max() <= 1e-12 * (1 + np.abs(Wo).max())
            assert abs(zg - zo) <= 1e-12 * (1 + abs(zo))


def test_create_from_torch_tensors(lpg):
    import torch
    A, b, c = lpgen.dense_lp(12, 150, 280)
    ref = oracle.solve(A, b, c)
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()  # column-major, stride (1, m)
    db = torch.from_numpy(b).cuda()
    dc = torch.from_numpy(c).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    with lpg.LP.from_torch(dA, db, dc, stream=stream) as p:
        st = p.solve()
        sol = p.solution()
        piv = p.pivots()
    assert st == ref.status
    np.testing.assert_array_equal(piv["enter"], ref.enter)
    assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * abs(ref.objective)
    bad = db.clone()
    bad[3] = -1.0
    torch.cuda.synchronize()
    with pytest.raises(lpg.LPError):
        lpg.LP.from_torch(dA, bad, dc)


def test_dense_2000x4000_full_parity(lpg):
    """Mid-size dense LP: the full pivot sequence and the objective against the oracle."""
    A, b, c = lpgen.dense_lp(0, 2000, 4000)
    ref, (st, sol, _, _) = assert_parity(lpg, A, b, c)
    assert st == oracle.OPTIMAL
    assert_kkt(A, b, c, sol["x"], sol["y"])


def test_dense_4000x8000_bench_configuration(lpg):
    """The benchmarked instance, in the bench's launch configuration: the first pivots
    equal the oracle's, and the final basis carries a KKT certificate of optimality."""
    A, b, c = lpgen.dense_lp(0, 4000, 8000)
    prefix = 40
    o = oracle.Oracle(A, b, c)
    o.run(prefix)
    ref = o.result()
    with lpg.LP(A, b, c, iters_per_sync=16) as p:
        st = p.solve()
        sol = p.solution()
        piv = p.pivots()
    np.testing.assert_array_equal(piv["enter"][:prefix], ref.enter)
    np.testing.assert_array_equal(piv["row"][:prefix], ref.row)
    assert st == oracle.OPTIMAL
    assert_kkt(A, b, c, sol["x"], sol["y"])
    assert abs(sol["objective"] - float(c @ sol["x"])) <= 1e-12 * abs(sol["objective"])


@pytest.mark.parametrize("profile", [1, 2])
def test_profiling_modes_time_kernels_without_changing_results(lpg, profile):
    A, b, c = lpgen.dense_lp(13, 500, 1000)
    ref, (st, sol, piv, stats) = assert_parity(lpg, A, b, c, profile=profile, iters_per_sync=4)
    assert stats["price_launches"] > 0 and stats["update_launches"] == stats["price_launches"]
    assert stats["price_ms"] > 0 and stats["update_ms"] > 0
    # every update reads B^-1 (8 m^2) and writes back only the element pairs the pivot
    # changed (16 B each): between a read-only and a full read + write pass
    L = stats["update_launches"]
    written = stats["update_bytes"] - 8.0 * 500 * 500 * L
    assert 0 < written <= 8.0 * 500 * 500 * L and written % 16 == 0


def test_no_structural_columns(lpg):
    """n = 0: the slack basis is the only basis; OPTIMAL at once with objective 0."""
    _say("case: m=3 n=0")
    A, b, c = np.zeros((3, 0)), np.array([1.0, 2.0, 3.0]), np.zeros(0)
    ref, (st, sol, _, _) = assert_parity(lpg, A, b, c)
    assert st == oracle.OPTIMAL and sol["iterations"] == 0 and sol["objective"] == 0.0
