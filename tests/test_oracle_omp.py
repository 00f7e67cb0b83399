"""The oracle's -fopenmp build (used for whole solves at the benchmark's sizes and for the
all-cores CPU baseline) gives bit-identical results to the sequential build, and the stored
goldens belong to the current oracle source.  CPU only."""
import os
import sys

import numpy as np
import pytest

import lpgen
import oracle

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_goldens  # noqa: E402


def _same(r1, r2):
    for k in ("enter", "row", "leave", "flags", "basis"):
        assert np.array_equal(getattr(r1, k), getattr(r2, k)), k
    assert r1.status == r2.status and r1.iterations == r2.iterations
    assert r1.objective == r2.objective  # bitwise
    assert np.array_equal(r1.x, r2.x) and np.array_equal(r1.y, r2.y)


@pytest.mark.parametrize("case", ["dense", "degenerate_ties", "two_phase"])
def test_omp_build_is_bit_identical(case):
    lib = oracle.omp_lib(4)
    assert oracle.threads(lib) == 4
    kw = {}
    if case == "dense":
        A, b, c = lpgen.dense_lp(1, 300, 600)
    elif case == "degenerate_ties":
        A, b, c = lpgen.degenerate_lp(9, 150, 300)  # list clears and ties decide pivots here
    else:
        A, b, c, rt = lpgen.general_lp(0, 150, 300, ge_frac=0.2, eq_frac=0.1, neg_frac=0.1)
        kw["row_type"] = rt
    _same(oracle.solve(A, b, c, **kw), oracle.solve(A, b, c, lib_path=lib, **kw))


@pytest.mark.parametrize("name", list(make_goldens.GOLDENS))
def test_goldens_belong_to_this_oracle(name):
    g = make_goldens.load(name)
    assert g["oracle_sha16"] == make_goldens.oracle_sha16(), f"{name}: regenerate with make_goldens.py"
    law, seed, m, n, cap, _ = make_goldens.GOLDENS[name]
    assert (g["law"], g["seed"], g["n"], g["pivot_cap"]) == (law, seed, n, cap)
    assert len(g["enter"]) == len(g["row"]) == len(g["flags"]) == g["iterations"]


def test_golden_prefix_reproduces():
    """The first pivots of the benchmark configuration's golden, recomputed by the
    sequential oracle."""
    g = make_goldens.load("dense_m4000_n8000_s0")
    A, b, c = lpgen.dense_lp(0, 4000, 8000)
    o = oracle.Oracle(A, b, c)
    o.run(8)
    r = o.result()
    assert list(r.enter) == g["enter"][:8] and list(r.row) == g["row"][:8] and list(r.flags) == g["flags"][:8]
