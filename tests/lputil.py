"""Independent checks for LP results: brute-force vertex enumeration, KKT conditions and a
replay of a pivot log with dense linear algebra.  None of these reuse the oracle's
arithmetic: they work from the basis alone (numpy.linalg)."""
from __future__ import annotations

import itertools

import numpy as np


def full_matrix(A):
    """(A', I_m): the standard form of Section 2.1."""
    m = A.shape[0]
    return np.hstack([np.asarray(A, float), np.eye(m)])


def brute_force(A, b, c, sense="max"):
    """Best objective over all basic feasible solutions of A'x + s = b, x, s >= 0.

    Returns (objective, x) of the best vertex.  Exact for bounded LPs up to the
    conditioning of the bases (tiny integer-ish instances here)."""
    A = np.asarray(A, float)
    m, n = A.shape
    M = full_matrix(A)
    cf = np.concatenate([np.asarray(c, float), np.zeros(m)])
    best, bestx = None, None
    for cols in itertools.combinations(range(n + m), m):
        B = M[:, cols]
        if abs(np.linalg.det(B)) < 1e-10:
            continue
        xb = np.linalg.solve(B, b)
        if np.any(xb < -1e-10):
            continue
        x = np.zeros(n + m)
        x[list(cols)] = xb
        obj = cf @ x
        if best is None or (obj > best if sense == "max" else obj < best):
            best, bestx = obj, x[:n]
    return best, bestx


def kkt_residuals(A, b, c, x, y, sense="max"):
    """Max violations of primal feasibility, dual feasibility, complementary slackness and
    the duality gap for  max/min c^T x  s.t.  A x <= b, x >= 0  with duals y."""
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    c = np.asarray(c, float)
    sgn = 1.0 if sense == "max" else -1.0  # min c^T x == -max (-c)^T x
    cs, ys = sgn * c, sgn * np.asarray(y, float)
    slack = b - A @ x
    red = A.T @ ys - cs
    return dict(
        x_neg=float(max(0.0, -x.min())) if x.size else 0.0,
        primal=float(max(0.0, -slack.min())),
        y_neg=float(max(0.0, -ys.min())),
        dual=float(max(0.0, -red.min())) if red.size else 0.0,
        comp_row=float(np.max(np.abs(ys * slack))),
        comp_col=float(np.max(np.abs(x * red))) if red.size else 0.0,
        gap=float(abs(cs @ x - b @ ys)),
    )


def assert_kkt(A, b, c, x, y, sense="max", tol=1e-8):
    r = kkt_residuals(A, b, c, x, y, sense)
    scale = 1.0 + float(np.max(np.abs(b))) + float(np.max(np.abs(c))) * (1.0 + float(np.sum(np.abs(x))))
    bad = {k: v for k, v in r.items() if v > tol * scale}
    assert not bad, f"KKT violated: {bad} (scale {scale})"


def replay_check(A, b, c, enter, row, sense="max", tenure=5, eps=1e-9, tol=1e-7):
    """Replays a pivot log from the slack basis with numpy and checks each pivot against
    the rule stated in Steps 3-6: the entering variable has a negative reduced cost that
    is minimal among the variables the entering mask allows (or among all improving ones
    when the mask allows none), and the leaving row attains the minimum ratio."""
    A = np.asarray(A, float)
    m, n = A.shape
    M = full_matrix(A)
    chat = np.concatenate([(-1.0 if sense == "max" else 1.0) * np.asarray(c, float), np.zeros(m)])
    basis = list(range(n, n + m))
    tabu_until = np.full(n + m, -1)
    for t, (q, r) in enumerate(zip(enter, row)):
        B = M[:, basis]
        pi = np.linalg.solve(B.T, chat[basis])
        d = chat - M.T @ pi
        nonbasic = np.ones(n + m, bool)
        nonbasic[basis] = False
        improving = nonbasic & (d < -eps)
        assert d[q] < tol, f"pivot {t}: entering {q} has d={d[q]}"
        allowed = improving & (tabu_until < t)
        pool = allowed if allowed.any() else improving
        assert pool[q], f"pivot {t}: entering {q} is masked (tabu until {tabu_until[q]})"
        dmin = d[pool].min()
        assert d[q] <= dmin + tol * (1 + abs(dmin)), f"pivot {t}: d[{q}]={d[q]} > min {dmin}"
        alpha = np.linalg.solve(B, M[:, q])
        xb = np.linalg.solve(B, b)
        R = alpha > eps
        assert R[r], f"pivot {t}: row {r} has alpha {alpha[r]}"
        ratios = np.where(R, np.maximum(xb, 0.0) / np.where(R, alpha, 1.0), np.inf)
        th = ratios.min()
        assert ratios[r] <= th + tol * (1 + abs(th)), f"pivot {t}: ratio {ratios[r]} > min {th}"
        leave = basis[r]
        if tenure > 0:
            tabu_until[leave] = t + tenure
        basis[r] = q
    return basis


def basis_sets(n, m, enter, row):
    """Sequence of basis sets (frozensets) after each pivot, starting with the slack basis."""
    basis = list(range(n, n + m))
    out = [frozenset(basis)]
    for q, r in zip(enter, row):
        basis[r] = q
        out.append(frozenset(basis))
    return out


# ---- LPs with row types (<= 0, >= 1, = 2) and b of any sign ----

def general_standard(A, b, row_type):
    """M with the caller's columns, then a slack column +e_i for each <= row and a surplus
    column -e_i for each >= row (ascending i): the constraints read M X = b, X >= 0."""
    A = np.asarray(A, float)
    m = A.shape[0]
    cols = [A]
    for i in range(m):
        if row_type[i] != 2:
            e = np.zeros((m, 1))
            e[i, 0] = 1.0 if row_type[i] == 0 else -1.0
            cols.append(e)
    return np.hstack(cols)


def brute_force_general(A, b, c, row_type, sense="max"):
    """Best objective over all basic feasible solutions of M X = b, X >= 0 (M as above, of
    full row rank); (None, None) when there is no feasible vertex."""
    A = np.asarray(A, float)
    m, n = A.shape
    M = general_standard(A, b, row_type)
    assert np.linalg.matrix_rank(M) == m, "brute force needs rows of full rank"
    N = M.shape[1]
    cf = np.concatenate([np.asarray(c, float), np.zeros(N - n)])
    best, bestx = None, None
    for cols in itertools.combinations(range(N), m):
        B = M[:, cols]
        if abs(np.linalg.det(B)) < 1e-10:
            continue
        xb = np.linalg.solve(B, b)
        if np.any(xb < -1e-10):
            continue
        x = np.zeros(N)
        x[list(cols)] = xb
        obj = cf @ x
        if best is None or (obj > best if sense == "max" else obj < best):
            best, bestx = obj, x[:n]
    return best, bestx


def highs_general(A, b, c, row_type, sense="max"):
    """(status, objective) from scipy's HiGHS: status 'OPTIMAL', 'INFEASIBLE' or 'UNBOUNDED'."""
    from scipy.optimize import linprog
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    rt = np.asarray(row_type)
    Aub = np.vstack([A[rt == 0], -A[rt == 1]])
    bub = np.concatenate([b[rt == 0], -b[rt == 1]])
    kw = dict(A_ub=Aub, b_ub=bub) if Aub.shape[0] else {}
    if (rt == 2).any():
        kw.update(A_eq=A[rt == 2], b_eq=b[rt == 2])
    sg = -1.0 if sense == "max" else 1.0
    res = linprog(sg * np.asarray(c, float), method="highs", **kw)
    name = {0: "OPTIMAL", 2: "INFEASIBLE", 3: "UNBOUNDED"}.get(res.status, f"status{res.status}")
    return name, (sg * res.fun if res.status == 0 else None)


def kkt_general_residuals(A, b, c, x, y, row_type, sense="max"):
    """Max violations of the optimality conditions of  max/min c^T x  s.t.  row i of A x
    (<=, >=, =) b_i, x >= 0, with duals y: primal rows, x >= 0, dual signs (for max:
    y_i >= 0 on <= rows, <= 0 on >= rows, free on = rows), A^T y >= c, complementary
    slackness and the duality gap."""
    A = np.asarray(A, float)
    b = np.asarray(b, float)
    c = np.asarray(c, float)
    rt = np.asarray(row_type)
    sgn = 1.0 if sense == "max" else -1.0
    cs, ys = sgn * c, sgn * np.asarray(y, float)
    Ax = A @ x
    viol = np.where(rt == 0, Ax - b, np.where(rt == 1, b - Ax, np.abs(Ax - b)))
    ysign = np.where(rt == 0, -ys, np.where(rt == 1, ys, 0.0))
    red = A.T @ ys - cs
    return dict(
        x_neg=float(max(0.0, -x.min())) if x.size else 0.0,
        primal=float(max(0.0, viol.max())),
        y_sign=float(max(0.0, ysign.max())),
        dual=float(max(0.0, -red.min())) if red.size else 0.0,
        comp_row=float(np.max(np.abs(ys * (b - Ax)))),
        comp_col=float(np.max(np.abs(x * red))) if red.size else 0.0,
        gap=float(abs(cs @ x - b @ ys)),
    )


def assert_kkt_general(A, b, c, x, y, row_type, sense="max", tol=1e-8):
    r = kkt_general_residuals(A, b, c, x, y, row_type, sense)
    scale = 1.0 + float(np.max(np.abs(b))) + float(np.max(np.abs(c), initial=0.0)) * (1.0 + float(np.sum(np.abs(x))))
    bad = {k: v for k, v in r.items() if v > tol * scale}
    assert not bad, f"KKT violated: {bad} (scale {scale})"


def small_general_lps(seed, count):
    """Tiny degenerate LPs with integer-ish data and random row types / signs of b: the law
    on which phase 1 often ends with an artificial variable basic at zero."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m, n = int(rng.integers(2, 5)), int(rng.integers(2, 5))
        A = rng.choice([-1.0, 0.0, 1.0, 2.0], size=(m, n))
        rt = rng.choice([0, 1, 2], size=m, p=[0.3, 0.3, 0.4]).astype(np.int32)
        b = rng.choice([0.0, 0.0, 1.0, 2.0, -1.0], size=m)
        c = rng.choice([-1.0, 0.0, 1.0, 2.0], size=n)
        out.append((A, b, c, rt))
    return out


def transportation_lp(seed, S, D):
    """min sum c_sd x_sd over S supplies and D demands: row s sums x_s* = supply_s, row S+d
    sums x_*d = demand_d, all = rows; total supply equals total demand, so one row is
    implied by the others (a redundant = row).  Integer data, numpy seeded.
    Returns (A, b, c, row_type) for the min sense."""
    rng = np.random.default_rng(seed)
    supply = rng.integers(5, 30, size=S).astype(float)
    demand = rng.multinomial(int(supply.sum()) - D, np.full(D, 1.0 / D)).astype(float) + 1.0
    cost = rng.integers(1, 20, size=(S, D)).astype(float)
    A = np.zeros((S + D, S * D))
    for s in range(S):
        for d in range(D):
            A[s, s * D + d] = 1.0
            A[S + d, s * D + d] = 1.0
    return A, np.concatenate([supply, demand]), cost.ravel(), np.full(S + D, 2, dtype=np.int32)


# ---- the tie rules, replayed from the basis alone ----

def _band(values, target, tol):
    """Indices with |values - target| <= tol, and whether some other value sits close
    enough (within 100 tol) that the two cannot be told apart at this precision."""
    dist = np.abs(values - target)
    inside = dist <= tol
    near = (dist > tol) & (dist <= 100 * tol)
    return np.flatnonzero(inside), bool(near.any())


def replay_strict(A, b, c, enter, row, flags, sense="max", tenure=5, leaving_list=True, eps_d=1e-9, eps_p=1e-9,
                  eps_t=1e-9):
    """Replays a pivot log from the slack basis with numpy and checks every decision,
    ties included, against the stated rule:

    - entering (Step 4 with the entering mask): among the nonbasic variables with
      d_j < -eps_d (those the mask allows, else all of them: aspiration), the smallest
      d_j; equal smallest values go to the lowest variable index;
    - leaving (Step 6 with the tabu list of Sections 2.2/3.4): rows with alpha_i > eps_p
      are candidates, theta is their smallest ratio max(x_i, 0)/alpha_i, and a row is
      tied when max(x_i, 0) - alpha_i theta <= eps_t; with one tied row it leaves; with
      several, the lowest one whose basic variable is not in the entering variable's
      list L[q] leaves, or, if L[q] holds all of them, L[q] is emptied and the lowest
      tied row leaves; either way the leaving variable is then appended to L[q];
    - the logged TIE and LCLEAR flags match.

    L is simulated here from the log, independently of any solver.  A decision whose
    inputs lie so close to a threshold that numpy's rounding could change it is not
    judged (the log's own choice is followed there); the number of decisions judged is
    returned with the final basis."""
    A = np.asarray(A, float)
    m, n = A.shape
    M = full_matrix(A)
    chat = np.concatenate([(-1.0 if sense == "max" else 1.0) * np.asarray(c, float), np.zeros(m)])
    basis = list(range(n, n + m))
    tabu_until = np.full(n + m, -1)
    L = {}
    judged = 0
    scale_b = 1.0 + float(np.abs(b).max())
    for t, (q, r, f) in enumerate(zip(enter, row, flags)):
        q, r, f = int(q), int(r), int(f)
        B = M[:, basis]
        pi = np.linalg.solve(B.T, chat[basis])
        d = chat - M.T @ pi
        nonbasic = np.ones(n + m, bool)
        nonbasic[basis] = False
        dtol = 1e-10 * (1.0 + np.abs(chat).max())
        improving = nonbasic & (d < -eps_d)
        allowed = improving & (tabu_until < t)
        pool = np.flatnonzero(allowed if allowed.any() else improving)
        assert q in pool, f"pivot {t}: entering {q} not eligible"
        at_min, close = _band(d[pool], d[pool].min(), dtol)
        if not close:
            assert q == pool[at_min].min(), f"pivot {t}: entering {q}, rule gives {pool[at_min].min()}"
            judged += 1
        alpha = np.linalg.solve(B, M[:, q])
        xb = np.maximum(np.linalg.solve(B, b), 0.0)
        cand = alpha > eps_p
        assert cand[r], f"pivot {t}: row {r} is not a candidate"
        ratios = np.where(cand, xb / np.where(cand, alpha, 1.0), np.inf)
        th = ratios.min()
        level = np.where(cand, xb - alpha * th, np.inf)
        xtol = min(1e-12 * scale_b, 0.5 * eps_t)
        tied = np.flatnonzero(level <= eps_t + xtol)
        sure = np.flatnonzero(level <= eps_t - xtol)
        lst = L.setdefault(q, [])
        if len(tied) == len(sure):
            free = [i for i in tied if not (leaving_list and basis[i] in lst)]
            is_tie = len(tied) >= 2
            clear = is_tie and leaving_list and not free
            want = int(tied.min()) if (not is_tie or not leaving_list or clear) else int(min(free))
            assert r == want, f"pivot {t}: leaving row {r}, rule gives {want} (tied rows {list(tied)})"
            assert bool(f & 2) == is_tie, f"pivot {t}: tie flag {f & 2} but {len(tied)} tied rows"
            assert bool(f & 8) == clear, f"pivot {t}: list-clear flag {f & 8}, rule says {clear}"
            judged += 1
        else:  # follow the log
            is_tie, clear = bool(f & 2), bool(f & 8)
        if is_tie and leaving_list:
            if clear:
                lst.clear()
            lst.append(basis[r])
        if tenure > 0:
            tabu_until[basis[r]] = t + tenure
        basis[r] = q
    return basis, judged


def general_normal_form(A, b, row_type):
    """The form the two-phase start solves: rows with b_i < 0 negated (<= and >= swap),
    a surplus column -e_i for each >= row after the caller's n columns (ascending i),
    then the unit column of every row (a slack for <= rows, an artificial variable for
    >= and = rows).  Returns (M, b2, n2, art) with M of shape m x (n2 + m)."""
    A = np.asarray(A, float)
    m, n = A.shape
    rt = np.asarray(row_type)
    sg = np.where(np.asarray(b) < 0, -1.0, 1.0)
    rt2 = np.where((sg < 0) & (rt == 0), 1, np.where((sg < 0) & (rt == 1), 0, rt))
    ge = np.flatnonzero(rt2 == 1)
    sur = np.zeros((m, len(ge)))
    sur[ge, np.arange(len(ge))] = -1.0
    M = np.hstack([sg[:, None] * A, sur, np.eye(m)])
    return M, sg * np.asarray(b, float), n + len(ge), rt2 != 0


def check_drive_outs(A, b, row_type, enter, row, flags, eps_p=1e-9):
    """Every pivot flagged DRIVEOUT (16), replayed from the unit basis: the entering column
    has the largest |entry| of row r of the tableau, B^-1 M[:, j], over the nonbasic
    columns that are not artificial variables (entries above eps_p only), the lowest such
    column among equal magnitudes.  Returns the number of drive-outs judged."""
    M, b2, n2, art = general_normal_form(A, b, row_type)
    m = M.shape[0]
    basis = list(range(n2, n2 + m))
    judged = 0
    for t, (q, r, f) in enumerate(zip(enter, row, flags)):
        q, r = int(q), int(r)
        if f & 16:
            B = M[:, basis]
            tr = np.linalg.solve(B.T, np.eye(m)[r]) @ M  # row r of B^-1 M
            elig = np.ones(n2 + m, bool)
            elig[basis] = False
            elig[n2:] &= ~art
            mag = np.where(elig, np.abs(tr), 0.0)
            ok = np.flatnonzero(mag > eps_p)
            assert q in ok, f"pivot {t}: drive-out column {q} has entry {tr[q]}"
            top = mag[ok].max()
            at_top, close = _band(mag[ok], top, 1e-12 * (1.0 + top))
            if not close:
                assert q == ok[at_top].min(), f"pivot {t}: drive-out column {q}, rule gives {ok[at_top].min()}"
                judged += 1
        basis[r] = q
    return judged
