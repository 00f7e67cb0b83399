"""Pins of the CPU oracle against what the paper and the mathematics fix, not against itself.

- optimum value: brute-force vertex enumeration (tiny LPs), HiGHS via scipy (larger LPs),
  closed forms (one row, diagonal A');
- optimality certificate: KKT conditions of the returned primal/dual pair;
- the pivot rule of Steps 3-6: every logged pivot replayed with dense linear algebra;
- the tableau of Figure 1 after every pivot: B^-1, W, x_B and z recomputed from the basis;
- anti-cycling (Sections 2.2, 3.4): two textbook LPs that cycle under plain Dantzig;
- the tie rules: hand-derived pivots for equal reduced costs, and a replay that simulates
  the leaving-side tabu list on its own and checks every entering and leaving choice,
  ties and list clears included, on degenerate LPs where those rules decide the pivots;
- special cases: unbounded column (Step 5), already optimal (Step 4), rejected input.
"""
import json
import os

import numpy as np
import pytest

import lpgen
import oracle
from lputil import assert_kkt, basis_sets, brute_force, full_matrix, replay_check, replay_strict

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cycling_lps.json")


def _cyc():
    with open(GOLDEN) as f:
        d = json.load(f)
    return {k: v for k, v in d.items() if not k.startswith("_")}


def _tiny_lp(rng, m, n, degenerate):
    vals = np.array([-2.0, -1.0, 0.0, 0.0, 1.0, 1.0, 2.0, 3.0, 0.5, 1.5])
    A = rng.choice(vals, size=(m, n)) + (rng.random((m, n)) < 0.3) * rng.random((m, n))
    A[0, :] = 0.5 + rng.random(n)  # one strictly positive row keeps the LP bounded
    b = rng.integers(0, 5, size=m).astype(float) if degenerate else rng.random(m) * 5 + 0.5
    b[0] = 4.0
    c = rng.choice(np.array([-1.0, 0.0, 1.0, 2.0, 3.0]), size=n) + rng.random(n) * 0.1
    return A, b, c


@pytest.mark.parametrize("seed", range(60))
def test_brute_force_vertices(seed):
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(1, 5))
    n = int(rng.integers(1, 6))
    A, b, c = _tiny_lp(rng, m, n, degenerate=seed % 2 == 0)
    r = oracle.solve(A, b, c, sense="max")
    assert r.status == oracle.OPTIMAL
    best, _ = brute_force(A, b, c, "max")
    assert abs(r.objective - best) <= 1e-12 * (1 + abs(best)) + 1e-12
    assert_kkt(A, b, c, r.x, r.y, "max")


@pytest.mark.parametrize("seed", range(20))
def test_brute_force_min_sense(seed):
    rng = np.random.default_rng(5000 + seed)
    m = int(rng.integers(1, 5))
    n = int(rng.integers(1, 6))
    A, b, c = _tiny_lp(rng, m, n, degenerate=True)
    r = oracle.solve(A, b, -c, sense="min")  # min (-c)^T x == -(max c^T x)
    best, _ = brute_force(A, b, c, "max")
    assert r.status == oracle.OPTIMAL
    assert abs(r.objective + best) <= 1e-12 * (1 + abs(best)) + 1e-12
    assert_kkt(A, b, -c, r.x, r.y, "min")


@pytest.mark.parametrize("seed", range(10))
def test_dense_law_vs_highs_m64(seed):
    from scipy.optimize import linprog
    A, b, c = lpgen.dense_lp(seed, 64, 128)
    r = oracle.solve(A, b, c)
    ref = linprog(-c, A_ub=A, b_ub=b, method="highs")
    assert ref.status == 0 and r.status == oracle.OPTIMAL
    assert abs(r.objective - (-ref.fun)) <= 1e-9 * abs(ref.fun)
    assert_kkt(A, b, c, r.x, r.y)
    replay_check(A, b, c, r.enter, r.row)


@pytest.mark.parametrize("m,seed", [(128, 0), (256, 1), (300, 2)])
def test_dense_law_vs_highs_larger(m, seed):
    from scipy.optimize import linprog
    A, b, c = lpgen.dense_lp(seed, m, 2 * m)
    r = oracle.solve(A, b, c)
    ref = linprog(-c, A_ub=A, b_ub=b, method="highs")
    assert r.status == oracle.OPTIMAL
    assert abs(r.objective - (-ref.fun)) <= 1e-9 * abs(ref.fun)
    assert_kkt(A, b, c, r.x, r.y)


@pytest.mark.parametrize("m,seed", [(60, 0), (100, 1), (100, 2), (150, 3)])
def test_degenerate_law_status_vs_highs(m, seed):
    """Degenerate sparse-structured law: UNBOUNDED or OPTIMAL must agree with HiGHS."""
    from scipy.optimize import linprog
    A, b, c = lpgen.degenerate_lp(seed, m, 2 * m)
    r = oracle.solve(A, b, c)
    ref = linprog(-c, A_ub=A, b_ub=b, method="highs")
    assert ref.status in (0, 3)
    if ref.status == 3:
        assert r.status == oracle.UNBOUNDED
        # the recorded ray column gives an improving direction with no blocking row
        assert r.ray >= 0
    else:
        assert r.status == oracle.OPTIMAL
        assert abs(r.objective - (-ref.fun)) <= 1e-9 * (1 + abs(ref.fun))
        assert_kkt(A, b, c, r.x, r.y)


@pytest.mark.parametrize("m,seed", [(60, 0), (100, 1), (150, 2)])
def test_degenerate_budget_law_vs_highs(m, seed):
    """Bounded companion (one dense budget row): optimum agrees with HiGHS; ties occur."""
    from scipy.optimize import linprog
    A, b, c = lpgen.degenerate_lp(seed, m, 2 * m, budget_row=True)
    r = oracle.solve(A, b, c)
    ref = linprog(-c, A_ub=A, b_ub=b, method="highs")
    assert ref.status == 0 and r.status == oracle.OPTIMAL
    assert abs(r.objective - (-ref.fun)) <= 1e-9 * (1 + abs(ref.fun))
    assert_kkt(A, b, c, r.x, r.y)
    assert r.counts["degenerate"] > 0
    replay_check(A, b, c, r.enter, r.row)


def test_tableau_invariants_every_pivot():
    """Figure 1's tableau after each pivot equals its definition from the basis."""
    for A, b, c in [lpgen.dense_lp(3, 40, 80), lpgen.degenerate_lp(4, 50, 100, budget_row=True)]:
        m, n = A.shape
        M = full_matrix(A)
        chat = np.concatenate([-c, np.zeros(m)])
        o = oracle.Oracle(A, b, c)
        zprev = 0.0
        for k in range(1, 400):
            st = o.run(k)
            res = o.result()
            Binv, xB, W, z = o.state()
            B = M[:, res.basis]
            assert np.abs(Binv @ B - np.eye(m)).max() < 1e-9
            assert np.abs(xB - np.linalg.solve(B, b)).max() < 1e-9 * (1 + np.abs(b).max())
            assert np.abs(W - np.linalg.solve(B.T, chat[res.basis])).max() < 1e-9
            assert abs(z - chat[res.basis] @ xB) < 1e-9 * (1 + abs(z))
            assert xB.min() >= 0.0
            assert z <= zprev + 1e-12  # min form: z never increases
            assert abs(res.objective + z) < 1e-9 * (1 + abs(z))  # user objective = -z for max
            zprev = z
            if st != oracle.ITER_LIMIT:
                break
        assert st == oracle.OPTIMAL


def test_resume_equals_uninterrupted():
    A, b, c = lpgen.degenerate_lp(5, 80, 160, budget_row=True)
    full = oracle.solve(A, b, c)
    o = oracle.Oracle(A, b, c)
    for k in (1, 7, 8, 30, 31):
        assert o.run(k) == oracle.ITER_LIMIT
        assert o.iterations == k
    o.run()
    part = o.result()
    assert part.status == full.status
    assert np.array_equal(part.enter, full.enter) and np.array_equal(part.row, full.row)
    assert part.objective == full.objective


@pytest.mark.parametrize("name", ["chvatal", "beale"])
def test_plain_dantzig_cycles(name):
    """With no tabu rule and lowest-row ties the textbook LPs revisit the starting basis."""
    d = _cyc()[name]
    A, b, c = np.array(d["A"], float), np.array(d["b"], float), np.array(d["c"], float)
    r = oracle.solve(A, b, c, tenure=0, leaving_list=False, max_iter=50)
    assert r.status == oracle.ITER_LIMIT
    sets = basis_sets(A.shape[1], A.shape[0], r.enter, r.row)
    k = d["cycle_length"]
    assert sets[k] == sets[0]
    assert len(set(sets[:k])) == k
    assert r.objective == 0.0


@pytest.mark.parametrize("name", ["chvatal", "beale"])
def test_tabu_rule_terminates(name):
    d = _cyc()[name]
    A, b, c = np.array(d["A"], float), np.array(d["b"], float), np.array(d["c"], float)
    r = oracle.solve(A, b, c, tenure=5, leaving_list=True, max_iter=200)
    assert r.status == oracle.OPTIMAL
    assert abs(r.objective - d["optimum"]) < 1e-12
    assert r.counts["tie"] > 0
    assert_kkt(A, b, c, r.x, r.y)
    best, _ = brute_force(A, b, c)
    assert abs(best - d["optimum"]) < 1e-12


@pytest.mark.parametrize("name", ["chvatal", "beale"])
def test_entering_mask_alone_does_not_terminate(name):
    """The entering mask without the leaving-side list still cycles (aspiration overrides it)."""
    d = _cyc()[name]
    A, b, c = np.array(d["A"], float), np.array(d["b"], float), np.array(d["c"], float)
    r = oracle.solve(A, b, c, tenure=5, leaving_list=False, max_iter=300)
    assert r.status == oracle.ITER_LIMIT


def _embedded(name, seed=7):
    """A cycling LP embedded block-diagonally in a dense random LP (64 rows in total)."""
    d = _cyc()[name]
    Ac = np.array(d["A"], float)
    A0, b0, c0 = lpgen.dense_lp(seed, 61, 124)
    m, n = 64, 128
    A = np.zeros((m, n))
    A[:3, :4] = Ac
    A[3:, 4:] = A0
    b = np.concatenate([d["b"], b0])
    c = np.concatenate([d["c"], c0])
    return A, b, c


@pytest.mark.parametrize("name", ["chvatal", "beale"])
def test_embedded_cycling_lp(name):
    from scipy.optimize import linprog
    A, b, c = _embedded(name)
    plain = oracle.solve(A, b, c, tenure=0, leaving_list=False, max_iter=2000)
    r = oracle.solve(A, b, c)
    ref = linprog(-c, A_ub=A, b_ub=b, method="highs")
    assert r.status == oracle.OPTIMAL
    assert abs(r.objective + ref.fun) <= 1e-9 * abs(ref.fun)
    assert_kkt(A, b, c, r.x, r.y)
    assert plain.status == oracle.ITER_LIMIT


def test_one_row_closed_form():
    """m = 1: max sum c_j x_j s.t. sum a_j x_j <= beta, a > 0  has optimum beta*max_j(c_j/a_j)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = int(rng.integers(1, 30))
        a = rng.random(n) + 0.1
        c = rng.random(n) * 4 - 1
        beta = float(rng.random() * 10)
        r = oracle.solve(a[None, :], np.array([beta]), c)
        want = beta * max(0.0, float(np.max(c / a)))
        assert r.status == oracle.OPTIMAL
        assert abs(r.objective - want) <= 1e-12 * (1 + want)


def test_diagonal_closed_form():
    rng = np.random.default_rng(4)
    n = 25
    a = rng.random(n) + 0.5
    c = rng.random(n) * 2 - 0.5
    b = rng.random(n) * 3
    b[3] = 0.0
    r = oracle.solve(np.diag(a), b, c)
    want = float(np.sum(np.where(c > 0, c * b / a, 0.0)))
    assert r.status == oracle.OPTIMAL
    assert abs(r.objective - want) <= 1e-12 * (1 + want)
    # Dantzig with one pivot per improving column
    assert r.iterations == int(np.sum(c > 1e-9))


def test_unbounded_column():
    A, b, c = lpgen.dense_lp(2, 20, 30)
    A[:, 5] = -np.abs(A[:, 5])
    c[5] = 100.0
    r = oracle.solve(A, b, c)
    assert r.status == oracle.UNBOUNDED and r.ray == 5 and r.iterations == 0


def test_numerical_status_on_overflow():
    """Non-finite arithmetic stops the solve with NUMERICAL before the pivot.

    (i) The step overflows: one row, a_11 = 1e-8, b = 1e301, so the only ratio is 1e309.
    (ii) Y_k overflows: x_1 enters on row 0 with alpha = (1e-8, 1e301) at the step 0
    (b_0 = 0), which sets B^-1[1,0] = -1e301/1e-8 = -inf; x_2 (reduced cost -1) is then
    improving and its FTRAN gives alpha_1 = -inf * 0 + 1 = NaN."""
    r = oracle.solve(np.array([[1e-8]]), np.array([1e301]), np.array([1.0]))
    assert r.status == oracle.NUMERICAL and r.iterations == 0
    A = np.array([[1e-8, 0.0], [1e301, 1.0]])
    r = oracle.solve(A, np.array([0.0, 1.0]), np.array([1.0, 1.0]))
    assert r.status == oracle.NUMERICAL and r.iterations == 1
    assert list(r.enter) == [0] and list(r.row) == [0]
    # the same LP with a finite second column entry in row 1 solves normally
    A2 = np.array([[1e-8, 0.0], [1.0, 1.0]])
    r = oracle.solve(A2, np.array([0.0, 1.0]), np.array([1.0, 1.0]))
    assert r.status == oracle.OPTIMAL


def test_already_optimal():
    A, b, c = lpgen.dense_lp(2, 20, 30)
    r = oracle.solve(A, b, -c)
    assert r.status == oracle.OPTIMAL and r.iterations == 0 and r.objective == 0.0
    r = oracle.solve(A, b, c, sense="min")
    assert r.status == oracle.OPTIMAL and r.iterations == 0


def test_rejects_bad_input():
    A, b, c = lpgen.dense_lp(2, 5, 5)
    with pytest.raises(ValueError):
        oracle.Oracle(A, -b, c)
    with pytest.raises(ValueError):
        oracle.Oracle(np.zeros((0, 3)), np.zeros(0), np.zeros(3))
    bad = b.copy()
    bad[1] = np.nan
    with pytest.raises(ValueError):
        oracle.Oracle(A, bad, c)


def test_rounding_split_tie_is_a_tie():
    """Two rows that reach zero at the same step in exact arithmetic, but whose FP64 ratios
    differ by an ulp, form a tie (Sections 2.2/3.4: no unique leaving element): the lowest
    row leaves and the step is the minimum ratio."""
    b = np.array([0.1 * 3, 0.1])  # 0.30000000000000004 / 3 != 0.1 in FP64
    assert b[0] / 3.0 != b[1]
    A = np.array([[3.0], [1.0]])
    r = oracle.solve(A, b, np.array([1.0]))
    assert r.row[0] == 0 and r.flags[0] & oracle.FLAG_TIE
    assert r.objective == min(b[0] / 3.0, b[1])  # x = theta_min
    # a row that stays above zero by more than the tolerance is not tied: the smaller ratio leaves
    b2 = np.array([0.3 * (1 + 1e-6), 0.1])
    r2 = oracle.solve(A, b2, np.array([1.0]))
    assert r2.row[0] == 1 and not (r2.flags[0] & oracle.FLAG_TIE)


def test_tie_tolerance_is_in_x_units():
    """A huge alpha must not turn a ratio-sized tolerance into a large infeasibility: with
    theta_min = 0 a row with a tiny positive ratio but a large value is not tied."""
    A = np.array([[1.0, 1.0], [1e12, 1.0], [0.0, 1.0]])
    b = np.array([0.0, 1.0, 5.0])  # row 0 degenerate (ratio 0), row 1 ratio 1e-12 but x = 1
    r = oracle.solve(A, b, np.array([1.0, 0.0]), max_iter=1)
    assert r.row[0] == 0 and not (r.flags[0] & oracle.FLAG_TIE)
    o = oracle.Oracle(A, b, np.array([1.0, 0.0]))
    o.run(1)
    _, xB, _, _ = o.state()
    assert xB.min() >= 0.0


def test_entering_tie_goes_to_lowest_index():
    """Equal reduced costs: the lowest variable index enters (reading of Step 4).

    max 3x0 + 3x1 s.t. x0 + x1 <= 2 from the slack basis: W = 0, so d = (-3, -3), bit for
    bit equal.  x0 enters, its only row (alpha = 1, ratio 2) leaves with slack variable 2,
    and then W = -3 gives d_1 = -3 - (-3)(1) = 0 and d_2 = 0 - (-3) = 3: optimal at
    x = (2, 0), objective 6.  Taking the higher index would end at x = (0, 2) instead."""
    r = oracle.solve(np.array([[1.0, 1.0]]), np.array([2.0]), np.array([3.0, 3.0]))
    assert r.status == oracle.OPTIMAL
    assert list(r.enter) == [0] and list(r.row) == [0] and list(r.leave) == [2]
    assert np.array_equal(r.x, [2.0, 0.0]) and r.objective == 6.0
    # A dense LP whose 20 columns appear twice (j and j + 20 identical, equal costs): the two
    # copies always have equal reduced costs, so only the lower copy (or a slack, >= 40) enters.
    A0, b0, c0 = lpgen.dense_lp(3, 30, 20)
    A, c = np.hstack([A0, A0]), np.concatenate([c0, c0])
    r = oracle.solve(A, b0, c)
    assert r.status == oracle.OPTIMAL and r.iterations > 0
    assert all(q < 20 or q >= 40 for q in r.enter)
    replay_strict(A, b0, c, r.enter, r.row, r.flags)


# Degenerate LPs on which the leaving-side tabu list decides pivots: each has a tie whose
# tied rows' leaving variables are all in the entering variable's list (a list clear), and
# a later tie that the cleared list decides (keeping the stale entries picks another row).
TIE_LPS = [(150, 9, False), (150, 8, False), (200, 15, True)]


@pytest.mark.parametrize("m,seed,budget", TIE_LPS)
def test_tie_rules_replayed_on_degenerate_lps(m, seed, budget):
    A, b, c = lpgen.degenerate_lp(seed, m, 2 * m, budget_row=budget)
    r = oracle.solve(A, b, c)
    assert r.status == oracle.OPTIMAL
    assert r.counts["lclear"] >= 1 and r.counts["tie"] >= 20
    _, judged = replay_strict(A, b, c, r.enter, r.row, r.flags)
    assert judged >= 2 * r.iterations - 4  # nearly every decision is far from a threshold


@pytest.mark.parametrize("case", ["dense0", "dense1", "beale", "chvatal"])
def test_tie_rules_replayed(case):
    A, b, c = lpgen.dense_lp(int(case[-1]), 64, 128) if case.startswith("dense") else _embedded(case)
    r = oracle.solve(A, b, c)
    assert r.status == oracle.OPTIMAL
    replay_strict(A, b, c, r.enter, r.row, r.flags)


def test_decision_margin_of_a_near_threshold_alpha():
    """The reported decision margin (which no decision uses) against a hand-worked LP: the
    entering column's second entry, 1.5e-9, is the value closest to a threshold (eps_p =
    1e-9), so the first pivot's margin is their difference; every other value of the pivot
    is O(1) from its threshold or rival (d = (-3, -2), x_B after the step = (1, 1 - 1.5e-9))."""
    A = np.array([[1.0, 1.0], [1.5e-9, 1.0]])
    b = np.array([1.0, 1.0])
    c = np.array([3.0, 2.0])
    o = oracle.Oracle(A, b, c)
    o.run(1)
    r = o.result()
    assert r.enter[0] == 0 and r.row[0] == 0
    assert r.margin[0] == abs(1.5e-9 - 1e-9)
    # nothing of the second pivot (if any) and no tiny residue counts below it
    assert np.all(r.margin >= 0.0)
