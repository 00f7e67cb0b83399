"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a temporary copy of the oracle's C source (a dropped
term, a wrong sign, a transposed operand, a wrong comparison, a missing tabu-list
update), builds it with the oracle's own flags, and checks that the pins used in
test_oracle_pins reject it.  Everything runs on the CPU."""
import os
import subprocess

import numpy as np
import pytest

import lpgen
import oracle
from test_oracle_pins import _embedded
from lputil import (assert_kkt, assert_kkt_general, brute_force, check_drive_outs, highs_general, replay_check,
                    replay_strict, small_general_lps)

SRC = os.path.join(os.path.dirname(oracle.__file__), "simplex_oracle.c")

MUTANTS = {
    "dropped_cost_term": ("p->d[j] = p->chat[j] - s;", "p->d[j] = -s;"),
    "W_update_sign": ("p->W[j] = fma(dq, p->rho[j], p->W[j]);", "p->W[j] = fma(-dq, p->rho[j], p->W[j]);"),
    "ftran_transposed": ("s = fma(row[k], a[k], s);", "s = fma(p->Binv[(size_t)k * m + i], a[k], s);"),
    "xB_update_sign": ("fma(-p->alpha[i], theta, p->xB[i])", "fma(p->alpha[i], theta, p->xB[i])"),
    "entering_argmax": ("(q_free < 0 || p->d[j] < p->d[q_free])", "(q_free < 0 || p->d[j] > p->d[q_free])"),
    "aspiration_argmax": ("if (q_all < 0 || p->d[j] < p->d[q_all]) q_all = j;",
                          "if (q_all < 0 || p->d[j] > p->d[q_all]) q_all = j;"),
    "no_entering_mask": ("if (p->tenure > 0) p->tabu_until[leave] = p->t + p->tenure;", "(void)leave;"),
    "ratio_argmax": ("if (p->ratio[i] < theta_min) theta_min = p->ratio[i];",
                     "if (theta_min == INFINITY || p->ratio[i] > theta_min) theta_min = p->ratio[i];"),
    "pivot_row_not_divided": ("p->rho[j] = rowr[j] / ar;", "p->rho[j] = rowr[j];"),
    "no_leaving_list_append": ("if (list_add(p, q, p->basis[r])) return -1;", "(void)0;"),
    "slack_price_wrong_index": ("p->d[j] = p->chat[j] - p->W[j - n];", "p->d[j] = p->chat[j] - p->W[0];"),
    "no_alpha_finite_check": ("if (!isfinite(p->alpha[i])) return OR_NUMERICAL;", "(void)0;"),
    "no_step_finite_check": ("if (!isfinite(theta_min)) return OR_NUMERICAL;", "(void)0;"),
    # two-phase start
    "artificial_cost_zero": ("(v >= n2 && art[v - n2]) ? 1.0 : 0.0;", "(v >= n2 && art[v - n2]) ? 0.0 : 0.0;"),
    "no_row_negation": ("sg[i] = b[i] < 0.0 ? -1.0 : 1.0;", "sg[i] = 1.0;"),
    "surplus_sign": ("if (ge[i]) A2[(size_t)(k++) * m + i] = -1.0;", "if (ge[i]) A2[(size_t)(k++) * m + i] = 1.0;"),
    "infeasibility_test_sign": ("if (p->z > p->eps_f) return OR_INFEASIBLE;", "if (p->z < -p->eps_f) return OR_INFEASIBLE;"),
    "no_drive_out": ("if (best >= 0 && drive_out(p, best, r)) return -1;", "(void)best;"),
    "no_barring": ("p->pos[leave] = (p->art && leave >= n && p->art[leave - n]) ? POS_BARRED : -1;",
                   "p->pos[leave] = -1;"),
    "reprice_transposed": ("if (cb != 0.0) s = fma(cb, p->Binv[(size_t)i * m + j], s);",
                           "if (cb != 0.0) s = fma(cb, p->Binv[(size_t)j * m + i], s);"),
    "no_phase2_costs": ("memcpy(p->chat, p->chat2, sizeof(double) * N);", "(void)0;"),
    "dual_ignores_row_sign": ("y[i] = s * p->W[i] * (p->rsign ? p->rsign[i] : 1.0);", "y[i] = s * p->W[i];"),
    # tie rules (Sections 2.2/3.4 and the readings of Step 4 and of the phase switch)
    "no_lclear": ("if (r_free < 0) { p->L_len[q] = 0; flags |= FLAG_LCLEAR; p->n_lclear++; }",
                  "if (r_free < 0) { flags |= FLAG_LCLEAR; p->n_lclear++; }"),
    "entering_tie_highest": [("if (q_all < 0 || p->d[j] < p->d[q_all]) q_all = j;",
                              "if (q_all < 0 || p->d[j] <= p->d[q_all]) q_all = j;"),
                             ("(q_free < 0 || p->d[j] < p->d[q_free])", "(q_free < 0 || p->d[j] <= p->d[q_free])")],
    "driveout_first_not_largest": ("if (fabs(t) > p->eps_p && fabs(t) > fabs(bt)) { best = j; bt = t; }",
                                   "if (fabs(t) > p->eps_p && best < 0) { best = j; bt = t; }"),
}


def _build(tmp_path, name, subs):
    """subs: one (old, new) pair, or a list of them applied together."""
    src = open(SRC).read()
    for old, new in ([subs] if isinstance(subs, tuple) else subs):
        assert src.count(old) == 1, f"mutation anchor for {name} not unique"
        src = src.replace(old, new)
    path = tmp_path / f"{name}.c"
    path.write_text(src)
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(path), "-lm"])
    return str(so)


def _pins_pass(lib_path):
    """A compact run of the pins; returns False as soon as one rejects the build."""
    import json
    from scipy.optimize import linprog
    try:
        rng = np.random.default_rng(11)
        for k in range(12):
            m, n = 3, 4
            vals = np.array([-1.0, 0.0, 1.0, 2.0, 0.5])
            A = rng.choice(vals, size=(m, n)) + 0.1 * rng.random((m, n))
            A[0] = 0.5 + rng.random(n)
            b = rng.integers(0, 4, size=m).astype(float)
            b[0] = 3.0
            c = rng.random(n) * 3 - 0.5
            r = oracle.solve(A, b, c, lib_path=lib_path, max_iter=500)
            best, _ = brute_force(A, b, c)
            if r.status != oracle.OPTIMAL or abs(r.objective - best) > 1e-9 * (1 + abs(best)):
                return False
            assert_kkt(A, b, c, r.x, r.y)
        for seed in range(2):
            A, b, c = lpgen.dense_lp(seed, 30, 60)
            r = oracle.solve(A, b, c, lib_path=lib_path, max_iter=2000)
            ref = linprog(-c, A_ub=A, b_ub=b, method="highs")
            if r.status != oracle.OPTIMAL or abs(r.objective + ref.fun) > 1e-9 * abs(ref.fun):
                return False
            assert_kkt(A, b, c, r.x, r.y)
            replay_check(A, b, c, r.enter, r.row)
        # entering ties (equal reduced costs) go to the lowest index
        r = oracle.solve(np.array([[1.0, 1.0]]), np.array([2.0]), np.array([3.0, 3.0]), lib_path=lib_path)
        if list(r.enter) != [0]:
            return False
        A0, b0, c0 = lpgen.dense_lp(3, 30, 20)
        Ad, cd = np.hstack([A0, A0]), np.concatenate([c0, c0])
        r = oracle.solve(Ad, b0, cd, lib_path=lib_path)
        replay_strict(Ad, b0, cd, r.enter, r.row, r.flags)
        # the leaving-side tabu list on degenerate LPs where it decides pivots
        for m, seed in ((150, 9), (150, 8)):
            A, b, c = lpgen.degenerate_lp(seed, m, 2 * m)
            r = oracle.solve(A, b, c, lib_path=lib_path)
            if r.status != oracle.OPTIMAL:
                return False
            replay_strict(A, b, c, r.enter, r.row, r.flags)
        for name in ("beale", "chvatal"):
            Ae, be, ce = _embedded(name)
            r = oracle.solve(Ae, be, ce, lib_path=lib_path, max_iter=2000)
            if r.status != oracle.OPTIMAL:
                return False
            replay_check(Ae, be, ce, r.enter, r.row)
        with open(os.path.join(os.path.dirname(__file__), "golden", "cycling_lps.json")) as f:
            d = json.load(f)["beale"]
        A, b, c = np.array(d["A"], float), np.array(d["b"], float), np.array(d["c"], float)
        r = oracle.solve(A, b, c, lib_path=lib_path, max_iter=200)
        if r.status != oracle.OPTIMAL or abs(r.objective - d["optimum"]) > 1e-12:
            return False
        # overflow stops the solve (the two cases of test_numerical_status_on_overflow)
        r = oracle.solve(np.array([[1e-8]]), np.array([1e301]), np.array([1.0]), lib_path=lib_path)
        if r.status != oracle.NUMERICAL:
            return False
        r = oracle.solve(np.array([[1e-8, 0.0], [1e301, 1.0]]), np.array([0.0, 1.0]), np.array([1.0, 1.0]),
                         lib_path=lib_path)
        if r.status != oracle.NUMERICAL or r.iterations != 1:
            return False
        # two-phase start: the hand-derived optimum, the status against HiGHS and a KKT
        # certificate on the tiny degenerate law, the general law against HiGHS
        r = oracle.solve(np.array([[3.0, 1.0], [4.0, 3.0], [1.0, 2.0]]), np.array([3.0, 6.0, 4.0]),
                         np.array([4.0, 1.0]), sense="min", row_type=[2, 1, 0], lib_path=lib_path)
        if r.status != oracle.OPTIMAL or abs(r.objective - 3.4) > 1e-14:
            return False
        for A, b, c, rt in small_general_lps(3, 250):
            r = oracle.solve(A, b, c, row_type=rt, max_iter=500, lib_path=lib_path)
            check_drive_outs(A, b, rt, r.enter, r.row, r.flags)
            ref, obj = highs_general(A, b, c, rt)
            if r.status_name != ref:
                return False
            if ref == "OPTIMAL":
                if abs(r.objective - obj) > 1e-9 * (1 + abs(obj)):
                    return False
                assert_kkt_general(A, b, c, r.x, r.y, rt)
        A, b, c, rt = lpgen.general_lp(0, 60, 120, ge_frac=0.2, eq_frac=0.1, neg_frac=0.1)
        r = oracle.solve(A, b, c, row_type=rt, lib_path=lib_path)
        ref, obj = highs_general(A, b, c, rt)
        if r.status != oracle.OPTIMAL or abs(r.objective - obj) > 1e-9 * abs(obj):
            return False
        assert_kkt_general(A, b, c, r.x, r.y, rt)
    except (AssertionError, ValueError):
        return False
    return True


def test_unmutated_source_passes(tmp_path):
    so = tmp_path / "liborig.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), SRC, "-lm"])
    assert _pins_pass(str(so))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_build(tmp_path, name, MUTANTS[name])), f"pins did not catch mutant {name}"
