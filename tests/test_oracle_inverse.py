"""Pins of the oracle's basis inverse (the reference of the GPU reinversion).

The paper never refactorises, so these pins come from the mathematics: closed-form
inverses, a library inverse, the oracle's own product-form B^-1 after a solve, and the
reordering identity inv(B P) = P^T inv(B).  Planted mistakes in the routine must fail
them (mutants at the end)."""
import os
import subprocess

import numpy as np
import pytest

import lpgen
import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "simplex_oracle.c")


def _basis_matrix(A, basis):
    m, n = A.shape
    M = np.hstack([A, np.eye(m)])
    return M[:, basis]


def _pins(lib_path=None):
    inv = lambda A, bas: oracle.basis_inverse(A, bas, lib_path=lib_path)
    rng = np.random.default_rng(5)
    m, n = 7, 5
    A = rng.random((m, n))
    # slack basis: identity
    Bi = inv(A, np.arange(n, n + m))
    assert Bi is not None and np.array_equal(Bi, np.eye(m))
    # shuffled slacks: a permutation matrix, inverse = transpose
    perm = rng.permutation(m)
    Bi = inv(A, n + perm)
    assert Bi is not None
    expect = np.zeros((m, m))
    expect[np.arange(m), perm] = 1.0
    assert np.array_equal(Bi, expect)
    # unit lower bidiagonal (1 on the diagonal, -1 below): inverse = lower-triangular ones
    k = 6
    L = np.eye(k) - np.eye(k, k=-1)
    Bi = inv(L, np.arange(k))
    assert Bi is not None and np.array_equal(Bi, np.tril(np.ones((k, k))))
    # mixed basis of a dense LP against a library inverse and the product-form B^-1
    A, b, c = lpgen.dense_lp(3, 40, 80)
    r = oracle.solve(A, b, c, lib_path=lib_path)
    assert r.status == oracle.OPTIMAL
    Bi = inv(A, r.basis)
    B = _basis_matrix(A, r.basis)
    assert Bi is not None
    np.testing.assert_allclose(Bi, np.linalg.inv(B), rtol=0, atol=1e-11 * np.abs(Bi).max())
    assert np.abs(Bi @ B - np.eye(40)).max() < 1e-12
    o = oracle.Oracle(A, b, c, lib_path=lib_path)
    o.run()
    Binv_eta = o.state()[0]
    np.testing.assert_allclose(Bi, Binv_eta, rtol=0, atol=1e-10 * np.abs(Bi).max())
    # reordering the basis list permutes the rows of the inverse
    q = rng.permutation(40)
    Bq = inv(A, r.basis[q])
    np.testing.assert_allclose(Bq, Bi[q], rtol=0, atol=1e-12 * np.abs(Bi).max())
    # singular: a repeated column
    bad = r.basis.copy()
    bad[1] = bad[0]
    assert inv(A, bad) is None


def test_basis_inverse_pins():
    _pins()


def test_basis_inverse_rejects_wrong_length():
    A = np.ones((3, 2))
    with pytest.raises(ValueError):
        oracle.basis_inverse(A, np.arange(2))


MUTANTS = {
    "no_partial_pivoting": ("if (fabs(T[(size_t)i * w + c]) > fabs(T[(size_t)piv * w + c])) piv = i;", "(void)0;"),
    "elimination_sign": ("T[(size_t)i * w + j] -= f * T[(size_t)c * w + j];",
                         "T[(size_t)i * w + j] += f * T[(size_t)c * w + j];"),
    "pivot_row_not_scaled": ("for (int32_t j = 0; j < w; ++j) T[(size_t)c * w + j] /= pv;", "(void)pv;"),
    "slack_column_shifted": ("(i == v - n ? 1.0 : 0.0)", "(i == v - n - 1 ? 1.0 : 0.0)"),
    "augmented_identity_transposed": ("T[(size_t)p * w + m + p] = 1.0;", "T[(size_t)p * w + m + (m - 1 - p)] = 1.0;"),
}


def _pins_pass(lib_path):
    try:
        _pins(lib_path)
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_inverse_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(path), "-lm"])
    assert not _pins_pass(str(so)), f"pins did not catch mutant {name}"
