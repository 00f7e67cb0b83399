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
