"""Seeded synthetic LP instances, shared by the HIP path's tests/bench and the oracle's.

This module only draws numbers: it holds none of the simplex arithmetic.  Every value
is a pure function of (seed, stream, index) through one counter-based hash, so any
entry can be regenerated on its own and every caller sees identical bits.

Hash (SplitMix64 finaliser of Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014):

    mix(z)    = z += 0x9E3779B97F4A7C15; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
                z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31      (mod 2^64)
    h(s,k,i)  = mix(mix(mix(s) ^ k) ^ i)
    u(s,k,i)  = (h(s,k,i) >> 11) * 2^-53          in [0, 1)
    U(a,b)    = a + (b - a) * u

Instances follow the paper's standard form (Section 2.1): max c^T x s.t. A'x <= b,
x >= 0, b >= 0, with A' an m x n dense matrix returned in column-major (Fortran)
order, so column j is contiguous.  The paper's own random instances (Section 4,
Appendix A) come from an unpublished generator; these laws stand in for them at
comparable shapes.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1
_G = 0x9E3779B97F4A7C15
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB

# stream ids
S_A, S_B, S_C, S_ROWSEL, S_ZEROB, S_SIZE, S_INST, S_EXTRA = 1, 2, 3, 4, 5, 6, 7, 8


def _mix_int(z: int) -> int:
    z = (z + _G) & _M64
    z = ((z ^ (z >> 30)) * _C1) & _M64
    z = ((z ^ (z >> 27)) * _C2) & _M64
    return z ^ (z >> 31)


def _mix_arr(z: np.ndarray) -> np.ndarray:
    z = z + np.uint64(_G)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_C1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_C2)
    return z ^ (z >> np.uint64(31))


def hash_scalar(seed: int, stream: int, idx: int) -> int:
    return _mix_int(_mix_int(_mix_int(seed & _M64) ^ stream) ^ (idx & _M64))


def hash_array(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    key = _mix_int(_mix_int(seed & _M64) ^ stream)
    return _mix_arr(np.asarray(idx, dtype=np.uint64) ^ np.uint64(key))


def uniform(seed: int, stream: int, idx: np.ndarray, lo: float, hi: float) -> np.ndarray:
    h = hash_array(seed, stream, idx)
    u = (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return lo + (hi - lo) * u


def dense_lp(seed: int, m: int, n: int, a=(0.0, 1.0), b=(1.0, 10.0), c=(1.0, 10.0)):
    """Dense law: A'_ij ~ U(a), b_i ~ U(b), c_j ~ U(c); A' column-major, entry (i,j) at index j*m+i."""
    A = np.empty((m, n), dtype=np.float64, order="F")
    cols = max(1, (1 << 22) // max(m, 1))  # ~32 MB of indices per chunk
    for j0 in range(0, n, cols):
        j1 = min(n, j0 + cols)
        idx = np.arange(j0 * m, j1 * m, dtype=np.uint64)
        A[:, j0:j1] = uniform(seed, S_A, idx, *a).reshape(j1 - j0, m).T
    bv = uniform(seed, S_B, np.arange(m, dtype=np.uint64), *b)
    cv = uniform(seed, S_C, np.arange(n, dtype=np.uint64), *c)
    return A, bv, cv


def _smallest_keys(keys: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k smallest keys, ascending by (key, index)."""
    if k >= keys.shape[-1]:
        return np.argsort(keys, kind="stable")
    part = np.argpartition(keys, k - 1)[:k]
    order = np.lexsort((part, keys[part]))
    return part[order]


def degenerate_lp(seed: int, m: int, n: int, col_frac=0.02, zero_b_frac=0.30, budget_row=False):
    """Degenerate sparse-structured law, stored dense.

    Per column: round(col_frac*m) distinct rows with values U(-1,1) plus one further
    distinct row with a value U(0.5,1).  round(zero_b_frac*m) distinct rows get b_i = 0,
    the rest b_i ~ U(1,10).  c_j ~ U(0,1).  With budget_row=True one dense row
    sum_j x_j <= m is appended (m+1 rows): a bounded companion.
    """
    k = max(1, int(round(col_frac * m)))
    if k + 1 > m:
        raise ValueError("degenerate_lp needs m > round(col_frac*m)")
    rows_out = m + 1 if budget_row else m
    A = np.zeros((rows_out, n), dtype=np.float64, order="F")
    for j in range(n):
        idx = np.arange(j * m, (j + 1) * m, dtype=np.uint64)
        keys = hash_array(seed, S_ROWSEL, idx)
        sel = _smallest_keys(keys, k + 1)
        vals = uniform(seed, S_A, idx[sel], -1.0, 1.0)
        vals[k] = uniform(seed, S_EXTRA, idx[sel[k:k + 1]], 0.5, 1.0)[0]
        A[sel, j] = vals
    bv = uniform(seed, S_B, np.arange(m, dtype=np.uint64), 1.0, 10.0)
    nz = int(round(zero_b_frac * m))
    if nz > 0:
        zrows = _smallest_keys(hash_array(seed, S_ZEROB, np.arange(m, dtype=np.uint64)), nz)
        bv[zrows] = 0.0
    cv = uniform(seed, S_C, np.arange(n, dtype=np.uint64), 0.0, 1.0)
    if budget_row:
        A[m, :] = 1.0
        bv = np.concatenate([bv, [float(m)]])
    return A, bv, cv


def diagonal_lp(seed: int, m: int, n: int, off=(0.0, 1e-4)):
    """Nearly diagonal law: A'_jj ~ U(1,2) for j < min(m, n), every other entry U(off)
    (the dense law's bits rescaled), b_i ~ U(1,10), c_j ~ U(1,10), max sense.  Each pivot
    of a Dantzig solve from the slack basis tends to bring in a new structural column in
    place of the slack of its diagonal row, so the basis fills with structural columns
    and the number of slacks that have left grows by about one per pivot."""
    A, bv, cv = dense_lp(seed, m, n, a=off)
    k = min(m, n)
    d = np.arange(k)
    A[d, d] = uniform(seed, S_EXTRA, np.arange(k, dtype=np.uint64), 1.0, 2.0)
    return A, bv, cv


ROW_LE, ROW_GE, ROW_EQ = 0, 1, 2


def general_lp(seed: int, m: int, n: int, ge_frac=0.05, eq_frac=0.02, neg_frac=0.05):
    """General-row law (an LP that needs the two-phase start of Section 3.4), feasible by
    construction and bounded: max c^T x s.t. row i of A'x (<=, >=, =) b_i, x >= 0.

    A'_ij ~ U(0,1) (the dense law's bits), a point x0_j ~ U(0, 2/n) and r = A'x0 (about
    0.5), so that the <= rows keep the dense law's scale.  Row i is >= with probability
    ge_frac (b_i = r_i * U(0.5,1)), = with probability eq_frac (b_i = r_i), else <=
    (b_i = r_i + U(1,10)); so x0 satisfies every row.  Then with probability neg_frac the
    row and b_i are multiplied by -1 and <= / >= swap, which gives b_i < 0.  c_j ~ U(1,10).
    Returns (A, b, c, row_type) with row_type int32 codes ROW_LE, ROW_GE, ROW_EQ.
    Dantzig pivots grow quickly with the share of >= rows (about 800 at m=1000, n=2000 with
    the default mix, 13900 with 20% >= and 10% = rows).
    """
    A, _, cv = dense_lp(seed, m, n)
    x0 = uniform(seed, S_EXTRA, np.arange(n, dtype=np.uint64), 0.0, 2.0 / n)
    r = (A * x0[None, :]).sum(axis=1)
    ui = np.arange(m, dtype=np.uint64)
    kind = uniform(seed, S_ROWSEL, ui, 0.0, 1.0)
    rt = np.where(kind < ge_frac, ROW_GE, np.where(kind < ge_frac + eq_frac, ROW_EQ, ROW_LE)).astype(np.int32)
    bv = np.where(rt == ROW_GE, r * uniform(seed, S_B, ui, 0.5, 1.0),
                  np.where(rt == ROW_EQ, r, r + uniform(seed, S_B, ui, 1.0, 10.0)))
    neg = uniform(seed, S_ZEROB, ui, 0.0, 1.0) < neg_frac
    A[neg, :] *= -1.0
    bv = np.where(neg, -bv, bv)
    rt = np.where(neg & (rt == ROW_LE), ROW_GE, np.where(neg & (rt == ROW_GE), ROW_LE, rt)).astype(np.int32)
    return A, bv, cv, rt


def batch_sizes(seed: int, count: int, m_lo=16, m_hi=256):
    """m_i = m_lo + (h(seed, size, i) mod (m_hi-m_lo+1)); n_i = 2 m_i."""
    span = m_hi - m_lo + 1
    h = hash_array(seed, S_SIZE, np.arange(count, dtype=np.uint64))
    ms = (m_lo + (h % np.uint64(span))).astype(np.int64)
    return ms, 2 * ms


def instance_seed(seed: int, i: int) -> int:
    return hash_scalar(seed, S_INST, i)


def batch_lps(seed: int, count: int, m_lo=16, m_hi=256):
    """Batch law: per-instance dense LPs (config-0 law) with sizes from batch_sizes."""
    ms, ns = batch_sizes(seed, count, m_lo, m_hi)
    out = []
    for i in range(count):
        out.append(dense_lp(instance_seed(seed, i), int(ms[i]), int(ns[i])))
    return out
