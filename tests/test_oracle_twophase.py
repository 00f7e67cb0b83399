"""Pins of the oracle's two-phase start (Section 3.4, "Finding the initial feasible
solution"): LPs with >=, = rows and right-hand sides of any sign.

Nothing here reuses the oracle's arithmetic: the references are a hand-derived optimum,
brute-force vertex enumeration, scipy's HiGHS, KKT certificates (which prove optimality
of the returned x and y by themselves) and invariances of the LP under row scaling."""
import numpy as np
import pytest

import lpgen
import oracle
from lputil import (assert_kkt_general, brute_force_general, check_drive_outs, general_standard, highs_general,
                    small_general_lps)

LE, GE, EQ = oracle.ROW_LE, oracle.ROW_GE, oracle.ROW_EQ
# a heavier share of >= / = / negated rows than the generator's default, for small LPs
HEAVY = dict(ge_frac=0.2, eq_frac=0.1, neg_frac=0.1)


def test_hand_derived_equality_lp():
    """min 4x1 + x2 s.t. 3x1 + x2 = 3, 4x1 + 3x2 >= 6, x1 + 2x2 <= 4.  The equality gives
    x2 = 3 - 3x1; the >= row becomes x1 <= 0.6, the <= row x1 >= 0.4, and the objective
    x1 + 3, so the optimum is x = (0.4, 1.8) with value 3.4.  Both x1 and x2 are basic,
    so the duals solve y^T A = c on them: y = (1.4, 0, -0.2)."""
    A = np.array([[3.0, 1.0], [4.0, 3.0], [1.0, 2.0]])
    b = np.array([3.0, 6.0, 4.0])
    c = np.array([4.0, 1.0])
    r = oracle.solve(A, b, c, sense="min", row_type=[EQ, GE, LE])
    assert r.status == oracle.OPTIMAL
    np.testing.assert_allclose(r.x, [0.4, 1.8], rtol=0, atol=1e-14)
    assert abs(r.objective - 3.4) < 1e-14
    np.testing.assert_allclose(r.y, [1.4, 0.0, -0.2], rtol=0, atol=1e-14)


@pytest.mark.parametrize("case", ["le_ge_contradiction", "eq_negative_rhs"])
def test_infeasible_lps(case):
    if case == "le_ge_contradiction":  # x1 + x2 <= 1 and x1 + x2 >= 2
        A, b, rt = np.array([[1.0, 1.0], [1.0, 1.0]]), np.array([1.0, 2.0]), [LE, GE]
    else:  # x1 + 2 x2 = -1 has no solution with x >= 0
        A, b, rt = np.array([[1.0, 2.0], [1.0, 0.0]]), np.array([-1.0, 3.0]), [EQ, LE]
    r = oracle.solve(A, b, np.array([1.0, 1.0]), row_type=rt)
    assert r.status == oracle.INFEASIBLE
    assert highs_general(A, b, np.array([1.0, 1.0]), rt)[0] == "INFEASIBLE"


def test_small_degenerate_lps_vs_highs_and_vertices():
    """400 tiny degenerate LPs: the status agrees with HiGHS, the objective with HiGHS and
    (for rows of full rank) with brute-force vertex enumeration, and every optimum carries
    a KKT certificate.  Many of them end phase 1 with an artificial variable basic at
    zero, which the drive-out pivots must remove without leaving the feasible set."""
    drive_outs = infeasible = unbounded = 0
    for A, b, c, rt in small_general_lps(3, 400):
        r = oracle.solve(A, b, c, row_type=rt, max_iter=500)
        ref, obj = highs_general(A, b, c, rt)
        assert r.status_name == ref, (A, b, c, rt)
        drive_outs += int(np.any(r.flags & oracle.FLAG_DRIVEOUT))
        infeasible += ref == "INFEASIBLE"
        unbounded += ref == "UNBOUNDED"
        if ref != "OPTIMAL":
            continue
        assert abs(r.objective - obj) <= 1e-9 * (1 + abs(obj))
        assert_kkt_general(A, b, c, r.x, r.y, rt)
        if np.linalg.matrix_rank(general_standard(A, b, rt)) == A.shape[0]:
            best, _ = brute_force_general(A, b, c, rt)
            assert abs(r.objective - best) <= 1e-9 * (1 + abs(best))
    # the law exercises every branch of the phase switch
    assert drive_outs >= 20 and infeasible >= 20 and unbounded >= 20, (drive_outs, infeasible, unbounded)


@pytest.mark.parametrize("m,n,seed", [(60, 120, 0), (60, 120, 1), (60, 120, 2), (150, 300, 0)])
def test_general_law_vs_highs(m, n, seed):
    A, b, c, rt = lpgen.general_lp(seed, m, n, **HEAVY)
    assert (b < 0).any() and (rt == GE).any() and (rt == EQ).any()
    r = oracle.solve(A, b, c, row_type=rt)
    ref, obj = highs_general(A, b, c, rt)
    assert ref == "OPTIMAL" and r.status == oracle.OPTIMAL
    assert abs(r.objective - obj) <= 1e-9 * abs(obj)
    assert_kkt_general(A, b, c, r.x, r.y, rt)


def test_redundant_rows_keep_an_artificial_basic():
    """Appending a copy of an = row and the sum of two = rows adds constraints that hold
    whenever the others do: same optimum, and the artificial variable of a redundant row
    cannot be driven out, so one stays basic (at zero)."""
    A, b, c, rt = lpgen.general_lp(4, 40, 80, **HEAVY)
    eq = np.flatnonzero(rt == EQ)
    assert eq.size >= 2
    A2 = np.vstack([A, A[eq[0]], A[eq[0]] + A[eq[1]]])
    b2 = np.concatenate([b, [b[eq[0]], b[eq[0]] + b[eq[1]]]])
    rt2 = np.concatenate([rt, [EQ, EQ]]).astype(np.int32)
    o = oracle.Oracle(A2, b2, c, row_type=rt2)
    o.run()
    r = o.result()
    ref, obj = highs_general(A, b, c, rt)
    assert r.status == oracle.OPTIMAL and abs(r.objective - obj) <= 1e-9 * abs(obj)
    assert_kkt_general(A2, b2, c, r.x, r.y, rt2)
    art_basic = [v for v in r.basis if v >= o.ncols]
    assert any(rt2[v - o.ncols] == EQ for v in art_basic)


def test_negated_rows_are_the_same_lp():
    """Row i of A'x <= b written as -A'_i x >= -b_i is the same constraint: the solve
    normalises it back bit for bit, so pivots and x are identical, and the dual of a
    written-negated row is the negated dual."""
    A, b, c = lpgen.dense_lp(5, 30, 60)
    flip = np.arange(30) % 3 == 0
    A2 = np.where(flip[:, None], -A, A)
    b2 = np.where(flip, -b, b)
    rt = np.where(flip, GE, LE).astype(np.int32)
    r1 = oracle.solve(A, b, c)
    r2 = oracle.solve(A2, b2, c, row_type=rt)
    assert r1.status == r2.status == oracle.OPTIMAL
    assert np.array_equal(r1.enter, r2.enter) and np.array_equal(r1.row, r2.row)
    assert np.array_equal(r1.x, r2.x) and np.array_equal(np.where(flip, -r1.y, r1.y), r2.y)
    assert_kkt_general(A2, b2, c, r2.x, r2.y, rt)


def test_all_le_rows_take_one_phase():
    A, b, c = lpgen.dense_lp(6, 40, 80)
    o = oracle.Oracle(A, b, c, row_type=np.zeros(40, np.int32))
    assert o.phase == 0 and o.ncols == 80
    o.run()
    r1, r2 = o.result(), oracle.solve(A, b, c)
    assert np.array_equal(r1.enter, r2.enter) and r1.objective == r2.objective


def test_unbounded_in_phase_two():
    """x1 + x2 >= 1, x1 - x3 <= 2: x3 grows without limit, and c_3 > 0."""
    A = np.array([[1.0, 1.0, 0.0], [1.0, 0.0, -1.0]])
    b = np.array([1.0, 2.0])
    c = np.array([1.0, 0.0, 1.0])
    o = oracle.Oracle(A, b, c, row_type=[GE, LE])
    assert o.run() == oracle.UNBOUNDED and o.phase == 2
    assert highs_general(A, b, c, [GE, LE])[0] == "UNBOUNDED"


def test_resume_across_the_phase_switch():
    A, b, c, rt = lpgen.general_lp(7, 50, 100, **HEAVY)
    full = oracle.solve(A, b, c, row_type=rt)
    o = oracle.Oracle(A, b, c, row_type=rt)
    cap, phases = 0, set()
    while True:
        cap += 7
        st = o.run(cap)
        phases.add(o.phase)
        if st != oracle.ITER_LIMIT:
            break
    r = o.result()
    assert phases == {1, 2}
    assert r.status == full.status and np.array_equal(r.enter, full.enter) and np.array_equal(r.flags, full.flags)


@pytest.mark.parametrize("S,D,seed", [(3, 4, 0), (6, 9, 1), (12, 15, 2)])
def test_transportation_problem(S, D, seed):
    """All rows are =, no slack exists, phase 1 starts from artificial variables only, and
    one row is redundant (supplies and demands have the same total)."""
    from lputil import transportation_lp
    A, b, c, rt = transportation_lp(seed, S, D)
    o = oracle.Oracle(A, b, c, sense="min", row_type=rt)
    assert o.run() == oracle.OPTIMAL
    r = o.result()
    ref, obj = highs_general(A, b, c, rt, sense="min")
    assert ref == "OPTIMAL" and abs(r.objective - obj) <= 1e-9 * abs(obj)
    assert_kkt_general(A, b, c, r.x, r.y, rt, sense="min")
    assert np.all(np.abs(r.x - np.round(r.x)) < 1e-9)  # integral data: vertices are integral
    # the redundant row keeps an artificial variable in the basis
    assert any(v >= o.ncols for v in r.basis)


def test_one_equality_row_closed_form():
    """max sum c_j x_j s.t. sum a_j x_j = beta (a > 0): the optimum is beta * max_j c_j / a_j,
    like the one-row <= case, since the row must be tight anyway when c > 0."""
    rng = np.random.default_rng(9)
    a = rng.uniform(0.5, 2.0, 7)
    c = rng.uniform(1.0, 3.0, 7)
    r = oracle.solve(a[None, :], np.array([4.0]), c, row_type=[EQ])
    assert r.status == oracle.OPTIMAL
    assert abs(r.objective - 4.0 * np.max(c / a)) <= 1e-12 * r.objective


@pytest.mark.parametrize("coef,want", [((-1.0, -3.0), 1), ((-3.0, -3.0), 0)])
def test_drive_out_takes_the_largest_entry(coef, want):
    """max x0 + x1 + 2x2 s.t. a0 x0 + a1 x1 = 0 (row 0), x0 + x1 + x2 <= 4 (row 1), with
    a0, a1 < 0.  Phase 1 starts from the artificial variable of row 0 (variable 3, the
    columns being x0, x1, x2) at level 0: its reduced costs are d_j = -a_j > 0, so phase 1
    is optimal at once with the artificial variable basic at zero.  Row 0 of the tableau is
    (a0, a1, 0, ., 0): the drive-out enters the column of the largest |entry|, x1 for
    (-1, -3) and, on equal magnitudes (-3, -3), the lowest column x0, with step 0.
    Phase 2 then lets x2 replace the slack of row 1 (theta = 4): x = (0, 0, 4),
    objective 8, whichever column was driven in."""
    A = np.array([[coef[0], coef[1], 0.0], [1.0, 1.0, 1.0]])
    r = oracle.solve(A, np.array([0.0, 4.0]), np.array([1.0, 1.0, 2.0]), row_type=[EQ, LE])
    assert r.status == oracle.OPTIMAL
    assert r.flags[0] & oracle.FLAG_DRIVEOUT
    assert r.enter[0] == want and r.row[0] == 0 and r.leave[0] == 3
    assert list(r.enter[1:]) == [2] and list(r.row[1:]) == [1]
    np.testing.assert_allclose(r.x, [0.0, 0.0, 4.0], rtol=0, atol=0)
    assert r.objective == 8.0


def test_drive_outs_replayed_on_small_lps():
    """Every drive-out of the tiny degenerate law, replayed from the unit basis with numpy:
    the entering column has the largest |entry| of its tableau row (lowest column on equal
    magnitudes), among the nonbasic columns that are not artificial variables."""
    judged = 0
    for A, b, c, rt in small_general_lps(3, 400):
        r = oracle.solve(A, b, c, row_type=rt, max_iter=500)
        judged += check_drive_outs(A, b, rt, r.enter, r.row, r.flags)
    assert judged >= 20
