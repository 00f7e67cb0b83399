"""Parity of the HIP two-phase start (lp_create_general) with the CPU oracle.

The GPU path must take the oracle's pivots exactly, phase 1, drive-outs and phase 2
alike (entering variable, leaving row, leaving variable, flags), reach the same status
(OPTIMAL, INFEASIBLE, UNBOUNDED), and match the oracle's objective to 1e-9 relative;
optimal results must also carry a KKT certificate for the given rows.  As in the
single-phase parity tests, dot products sum in different orders on the two sides, so
values agree to rounding; the phase-switch sums use the same order on both."""
import sys

import numpy as np
import pytest

import lpgen
import oracle
from lputil import assert_kkt_general, small_general_lps

pytestmark = pytest.mark.gpu

OBJ_RTOL = 1e-9
LE, GE, EQ = 0, 1, 2
# a heavier share of >= / = / negated rows than the generator's default, for small LPs
HEAVY = dict(ge_frac=0.2, eq_frac=0.1, neg_frac=0.1)


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


def _gpu(lpg, A, b, c, rt, max_iter=None, **opts):
    with lpg.LP(A, b, c, row_type=rt, **opts) as p:
        st = p.solve(max_iter)
        return st, p.solution(), p.pivots(), p.stats()


def assert_parity(lpg, A, b, c, rt, max_iter=None, kkt=True, **opts):
    ref = oracle.solve(A, b, c, row_type=rt, max_iter=max_iter, sense=opts.get("sense", "max"))
    st, sol, piv, stats = _gpu(lpg, A, b, c, rt, max_iter=max_iter, **opts)
    k = min(len(ref.enter), len(piv["enter"]))
    for name, a, g in (("enter", ref.enter, piv["enter"]), ("row", ref.row, piv["row"]),
                       ("leave", ref.leave, piv["leave"]), ("flags", ref.flags, piv["flags"])):
        diff = np.nonzero(a[:k] != g[:k])[0]
        assert diff.size == 0, f"first {name} divergence at pivot {diff[0]}: oracle {a[diff[0]]} gpu {g[diff[0]]}"
    assert len(ref.enter) == len(piv["enter"]) == sol["iterations"]
    assert st == ref.status, (lpg.STATUS_NAMES[st], ref.status_name)
    assert stats["drive_outs"] == int(np.count_nonzero(ref.flags & oracle.FLAG_DRIVEOUT))
    if st == lpg.LP_OPTIMAL:
        assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * (1 + abs(ref.objective))
        np.testing.assert_allclose(sol["x"], ref.x, rtol=0, atol=1e-9 * (1 + np.abs(ref.x).max(initial=0.0)))
        if kkt:
            assert_kkt_general(A, b, c, sol["x"], sol["y"], rt, sense=opts.get("sense", "max"))
    return st, sol, piv, stats


@pytest.mark.parametrize("m,n,seed,ips", [(60, 120, 0, 16), (60, 120, 1, 1), (60, 120, 2, 16), (300, 600, 0, 16),
                                          (1000, 2000, 0, 16)])
def test_general_law_parity(lpg, m, n, seed, ips):
    _say(f"case: general law m={m} n={n} seed={seed} iters_per_sync={ips}")
    A, b, c, rt = lpgen.general_lp(seed, m, n, **(HEAVY if m <= 300 else {}))
    st, sol, piv, stats = assert_parity(lpg, A, b, c, rt, iters_per_sync=ips)
    assert st == lpg.LP_OPTIMAL
    assert 0 < stats["phase1_iterations"] < sol["iterations"]


def test_small_degenerate_lps_parity(lpg):
    """Tiny degenerate LPs: every status of the phase switch, and drive-outs."""
    _say("case: 150 tiny degenerate LPs with row types")
    seen = set()
    for k, (A, b, c, rt) in enumerate(small_general_lps(3, 150)):
        st, sol, piv, stats = assert_parity(lpg, A, b, c, rt, max_iter=500)
        seen.add(st)
        if stats["drive_outs"]:
            seen.add("drive_out")
    assert {lpg.LP_OPTIMAL, lpg.LP_INFEASIBLE, lpg.LP_UNBOUNDED, "drive_out"} <= seen, seen


@pytest.mark.parametrize("sense", ["max", "min"])
def test_hand_derived_lp(lpg, sense):
    """min 4x1 + x2 (or max -4x1 - x2) s.t. 3x1 + x2 = 3, 4x1 + 3x2 >= 6, x1 + 2x2 <= 4:
    x = (0.4, 1.8), derived by eliminating x2 with the equality."""
    _say(f"case: hand-derived equality LP, sense {sense}")
    A = np.array([[3.0, 1.0], [4.0, 3.0], [1.0, 2.0]])
    b = np.array([3.0, 6.0, 4.0])
    c = np.array([4.0, 1.0]) * (1.0 if sense == "min" else -1.0)
    st, sol, _, _ = assert_parity(lpg, A, b, c, [EQ, GE, LE], sense=sense)
    assert st == lpg.LP_OPTIMAL
    np.testing.assert_allclose(sol["x"], [0.4, 1.8], rtol=0, atol=1e-14)


def test_infeasible_lps(lpg):
    _say("case: infeasible LPs (row contradiction, negative equality, general law + impossible row)")
    cases = [(np.array([[1.0, 1.0], [1.0, 1.0]]), np.array([1.0, 2.0]), np.array([1.0, 1.0]), [LE, GE]),
             (np.array([[1.0, 2.0], [1.0, 0.0]]), np.array([-1.0, 3.0]), np.array([1.0, 1.0]), [EQ, LE])]
    A, b, c, rt = lpgen.general_lp(3, 80, 160, **HEAVY)
    cases.append((np.vstack([A, np.ones((1, 160))]), np.concatenate([b, [-1.0]]), c,
                  np.concatenate([rt, [EQ]]).astype(np.int32)))
    for A, b, c, rt in cases:
        st, _, _, stats = assert_parity(lpg, A, b, c, rt)
        assert st == lpg.LP_INFEASIBLE and stats["phase1_iterations"] >= 0


def test_redundant_rows(lpg):
    _say("case: general law m=40 n=80 seed 4 plus two redundant = rows")
    A, b, c, rt = lpgen.general_lp(4, 40, 80, **HEAVY)
    eq = np.flatnonzero(rt == EQ)
    A2 = np.vstack([A, A[eq[0]], A[eq[0]] + A[eq[1]]])
    b2 = np.concatenate([b, [b[eq[0]], b[eq[0]] + b[eq[1]]]])
    rt2 = np.concatenate([rt, [EQ, EQ]]).astype(np.int32)
    st, sol, _, _ = assert_parity(lpg, A2, b2, c, rt2)
    assert st == lpg.LP_OPTIMAL


def test_unbounded_in_phase_two(lpg):
    _say("case: x1 + x2 >= 1, x1 - x3 <= 2, max x1 + x3")
    A = np.array([[1.0, 1.0, 0.0], [1.0, 0.0, -1.0]])
    st, _, _, stats = assert_parity(lpg, A, np.array([1.0, 2.0]), np.array([1.0, 0.0, 1.0]), [GE, LE])
    assert st == lpg.LP_UNBOUNDED and stats["phase1_iterations"] >= 0


def test_reset_and_resume_across_the_switch(lpg):
    _say("case: general law m=120 n=240 seed 5: reset, resume in steps of 7 pivots")
    A, b, c, rt = lpgen.general_lp(5, 120, 240, **HEAVY)
    with lpg.LP(A, b, c, row_type=rt) as p:
        assert p.solve() == lpg.LP_OPTIMAL
        first = p.pivots()
        p.reset()
        cap = 0
        while True:
            cap += 7
            if p.solve(cap) != lpg.LP_ITER_LIMIT:
                break
        again = p.pivots()
    for k in ("enter", "row", "leave", "flags"):
        assert np.array_equal(first[k], again[k]), k


@pytest.mark.parametrize("m,n", [(300, 600), (1000, 2000)])
def test_mixed_form_general(lpg, m, n):
    """The mixed form runs phase 1 without reinversions and phase 2 with them; its optimum
    must match the FP64 oracle's to 1e-9 and carry a KKT certificate."""
    _say(f"case: mixed form, general law m={m} n={n} seed 0")
    A, b, c, rt = lpgen.general_lp(0, m, n, **(HEAVY if m <= 300 else {}))
    ref = oracle.solve(A, b, c, row_type=rt)
    st, sol, _, stats = _gpu(lpg, A, b, c, rt, precision="mixed")
    assert st == ref.status == lpg.LP_OPTIMAL
    assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * abs(ref.objective)
    assert_kkt_general(A, b, c, sol["x"], sol["y"], rt)
    assert stats["phase1_iterations"] > 0


def test_general_full_size_4000x8000(lpg):
    """At the headline size: the first 150 pivots (all of phase 1 so far) equal the oracle's,
    and the GPU's optimum carries a KKT certificate for the given rows."""
    _say("case: general law m=4000 n=8000 seed 0 (oracle: first 150 pivots)")
    A, b, c, rt = lpgen.general_lp(0, 4000, 8000)
    o = oracle.Oracle(A, b, c, row_type=rt)
    o.run(150)
    ref = o.result()
    st, sol, piv, stats = _gpu(lpg, A, b, c, rt)
    assert st == lpg.LP_OPTIMAL
    k = len(ref.enter)
    assert k == 150
    for name in ("enter", "row", "leave", "flags"):
        assert np.array_equal(getattr(ref, name), piv[name][:k]), name
    assert_kkt_general(A, b, c, sol["x"], sol["y"], rt)
    _say(f"  {sol['iterations']} pivots, phase 1 {stats['phase1_iterations']}, drive-outs {stats['drive_outs']}, "
         f"switch {stats['phase_switch_ms']:.2f} ms")


@pytest.mark.parametrize("S,D,seed", [(6, 9, 1), (12, 15, 2), (30, 40, 3)])
def test_transportation_problem(lpg, S, D, seed):
    """All rows =, phase 1 from artificial variables only, one redundant row."""
    from lputil import transportation_lp
    _say(f"case: transportation problem {S} x {D} seed {seed}")
    A, b, c, rt = transportation_lp(seed, S, D)
    st, sol, _, _ = assert_parity(lpg, A, b, c, rt, sense="min")
    assert st == lpg.LP_OPTIMAL
    assert np.all(np.abs(sol["x"] - np.round(sol["x"])) < 1e-9)


@pytest.mark.parametrize("opts", [dict(tabu_tenure=0), dict(leaving_list=0), dict(iters_per_sync=64),
                                  dict(sense="min")])
def test_general_law_rule_variants(lpg, opts):
    _say(f"case: general law m=150 n=300 seed 6, options {opts}")
    A, b, c, rt = lpgen.general_lp(6, 150, 300, **HEAVY)
    if opts.get("sense") == "min":
        c = -c  # min of -c^T x: the same optimum as max c^T x
    ref_kw = {k: v for k, v in opts.items() if k in ("sense",)}
    ref = oracle.solve(A, b, c, row_type=rt, tenure=opts.get("tabu_tenure", 5),
                       leaving_list=bool(opts.get("leaving_list", 1)), **ref_kw)
    st, sol, piv, _ = _gpu(lpg, A, b, c, rt, **opts)
    assert st == ref.status == lpg.LP_OPTIMAL
    for k in ("enter", "row", "leave", "flags"):
        assert np.array_equal(getattr(ref, k), piv[k]), k
    assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * (1 + abs(ref.objective))
    assert_kkt_general(A, b, c, sol["x"], sol["y"], rt, sense=opts.get("sense", "max"))


def test_one_equality_row_and_zero_rhs(lpg):
    """sum a_j x_j = 4 alone (closed form 4 max c_j/a_j), and the same LP with an extra
    = row x_0 - x_1 = 0 whose artificial variable starts at zero."""
    _say("case: one = row; one = row plus a zero right-hand side")
    rng = np.random.default_rng(9)
    a = rng.uniform(0.5, 2.0, 7)
    c = rng.uniform(1.0, 3.0, 7)
    st, sol, _, _ = assert_parity(lpg, a[None, :], np.array([4.0]), c, [EQ])
    assert st == lpg.LP_OPTIMAL and abs(sol["objective"] - 4.0 * np.max(c / a)) <= 1e-12 * sol["objective"]
    A2 = np.vstack([a, np.eye(7)[0] - np.eye(7)[1]])
    st, sol, _, _ = assert_parity(lpg, A2, np.array([4.0, 0.0]), c, [EQ, EQ])
    assert st == lpg.LP_OPTIMAL and abs(sol["x"][0] - sol["x"][1]) < 1e-12


def test_no_given_columns(lpg):
    """n = 0 with = and >= rows: feasible only when every such b_i is 0 (then the >= row's
    surplus column drives its artificial variable out and the = row is redundant);
    a nonzero b_i on an = row, or b_i < 0 on a <= row, is infeasible."""
    _say("case: n=0 with = / >= / <= rows")
    Z = np.zeros((2, 0))
    st, sol, _, stats = assert_parity(lpg, Z, np.array([0.0, 0.0]), np.zeros(0), [EQ, GE])
    assert st == lpg.LP_OPTIMAL and stats["drive_outs"] == 1
    st, _, _, _ = assert_parity(lpg, Z, np.array([1.0, 0.0]), np.zeros(0), [EQ, LE])
    assert st == lpg.LP_INFEASIBLE
    st, _, _, _ = assert_parity(lpg, Z, np.array([-1.0, 0.0]), np.zeros(0), [LE, LE])
    assert st == lpg.LP_INFEASIBLE


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reinversion_during_phase_one(lpg, precision):
    """lp_reinvert in the middle of phase 1: W and z are recomputed with the phase-1 costs,
    and the solve still ends at the oracle's optimum with a KKT certificate."""
    _say(f"case: general law m=300 n=600 seed 1, reinversion after 40 pivots, {precision}")
    A, b, c, rt = lpgen.general_lp(1, 300, 600, **HEAVY)
    ref = oracle.solve(A, b, c, row_type=rt)
    with lpg.LP(A, b, c, row_type=rt, precision=precision, iters_per_sync=8) as p:
        assert p.solve(40) == lpg.LP_ITER_LIMIT
        assert p.stats()["phase1_iterations"] == -1  # still in phase 1
        p.reinvert()
        st = p.solve()
        sol = p.solution()
        stats = p.stats()
    assert st == ref.status == lpg.LP_OPTIMAL
    assert stats["reinversions"] >= 1 and stats["phase1_iterations"] > 40
    assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * abs(ref.objective)
    assert_kkt_general(A, b, c, sol["x"], sol["y"], rt)
