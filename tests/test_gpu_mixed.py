"""The mixed-precision form through the C ABI: FP32 screening of the reduced costs, the
shortlist re-priced in FP64, and the periodic FP64 reinversion.

Without reinversion the re-priced reduced costs are FP64 dot products like the FP64
path's, so the mixed path must take the oracle's pivots exactly (the same bar as the plain
path) as long as every Dantzig choice is among the FP32 shortlist; the tests below check
that it is, on the dense and degenerate laws.  With reinversion B^-1 is recomputed every 64 pivots, which
changes its rounding, so every result states its objective error and its primal and dual
residuals against the FP64 oracle (at 8000 x 16000 against the oracle's stored whole
solve) and must stay within 1e-9 relative."""
import os
import sys

import numpy as np
import pytest

import lpgen
import oracle
from lputil import assert_kkt, kkt_residuals
from test_gpu_parity import assert_parity

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))

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


def _solve(lpg, A, b, c, **opts):
    with lpg.LP(A, b, c, **opts) as p:
        st = p.solve()
        return st, p.solution(), p.pivots(), p.stats()


def _report(tag, A, b, c, sol, ref_obj):
    r = kkt_residuals(A, b, c, sol["x"], sol["y"])
    err = abs(sol["objective"] - ref_obj) / max(1.0, abs(ref_obj))
    _say(f"  {tag}: objective {sol['objective']:.15g} rel err {err:.2e}; primal {r['primal']:.1e} "
         f"dual {r['dual']:.1e} x<0 {r['x_neg']:.1e} y<0 {r['y_neg']:.1e} gap {r['gap']:.1e}")
    return err, r


def _square_lp(seed, m):
    """max c^T x, A x <= b with A = I + E, E >= 0 small (row sums ~ 0.25): A^-1 b > 0 and
    A^-T c > 0, so the optimal basis holds every structural column (k = m)."""
    rng = np.random.default_rng(seed)
    A = np.eye(m) + (0.5 / m) * rng.random((m, m))
    b = 1.0 + rng.random(m)
    c = 1.0 + rng.random(m)
    return np.asfortranarray(A), b, c


@pytest.mark.parametrize("seed", range(5))
def test_mixed_without_reinversion_follows_oracle_64x128(lpg, seed):
    A, b, c = lpgen.dense_lp(seed, 64, 128)
    ref, (st, sol, _, stats) = assert_parity(lpg, A, b, c, precision="mixed", reinv_period=0)
    assert st == oracle.OPTIMAL and stats["reinversions"] == 0
    assert stats["price32_launches"] == sol["iterations"] + 1
    assert stats["full_prices"] >= 1  # the optimality proof is always a full FP64 pass


@pytest.mark.parametrize("m,n", [(300, 600), (1000, 2000), (97, 301), (250, 120)])
def test_mixed_without_reinversion_follows_oracle(lpg, m, n):
    A, b, c = lpgen.dense_lp(7, m, n)
    ref, (st, sol, piv, stats) = assert_parity(lpg, A, b, c, precision="mixed", reinv_period=0)
    st64, sol64, piv64, _ = _solve(lpg, A, b, c)
    # same pivots as the FP64 GPU path; the re-priced d_q (summed in another order) feeds
    # W and z, so the objective agrees to rounding
    np.testing.assert_array_equal(piv["enter"], piv64["enter"])
    assert abs(sol["objective"] - sol64["objective"]) <= 1e-12 * abs(sol64["objective"])
    _say(f"  full FP64 pricing passes: {stats['full_prices']} of {stats['price32_launches']}")


@pytest.mark.parametrize("seed", range(3))
def test_mixed_degenerate_follows_oracle(lpg, seed):
    """Ties, the entering mask and aspiration (decided by the FP64 fallback pass)."""
    A, b, c = lpgen.degenerate_lp(seed, 120 + 40 * seed, 240 + 80 * seed, budget_row=True)
    ref, (st, sol, _, stats) = assert_parity(lpg, A, b, c, precision="mixed", reinv_period=0)
    assert stats["degenerate"] > 0


def test_mixed_degenerate_500_follows_oracle(lpg):
    A, b, c = lpgen.degenerate_lp(0, 500, 1000, budget_row=True)
    ref, (st, sol, _, stats) = assert_parity(lpg, A, b, c, precision="mixed", reinv_period=0)
    _say(f"  {sol['iterations']} pivots, aspirations {stats['aspirations']}, full passes {stats['full_prices']}")


@pytest.mark.parametrize("m,n", [(300, 600), (1000, 2000), (2000, 4000)])
def test_mixed_with_reinversion_against_oracle(lpg, m, n):
    A, b, c = lpgen.dense_lp(1, m, n)
    _say(f"case: mixed + reinversion every 64, dense m={m} n={n}")
    ref = oracle.solve(A, b, c)
    st, sol, piv, stats = _solve(lpg, A, b, c, precision="mixed")
    assert st == ref.status == oracle.OPTIMAL
    err, res = _report("mixed", A, b, c, sol, ref.objective)
    assert err <= OBJ_RTOL
    assert_kkt(A, b, c, sol["x"], sol["y"])
    assert stats["reinversions"] == sol["iterations"] // 64 and stats["reinv_failed"] == 0
    k = min(len(ref.enter), len(piv["enter"]))
    diff = np.nonzero(ref.enter[:k] != piv["enter"][:k])[0]
    _say(f"  {sol['iterations']} pivots (oracle {len(ref.enter)}), {stats['reinversions']} reinversions "
         f"{stats['reinv_ms']:.2f} ms, pivots equal to the oracle's up to "
         f"{diff[0] if diff.size else k}")


def test_reinvert_matches_oracle_inverse(lpg):
    """lp_reinvert mid-solve: B^-1, x_B, W and z against the oracle's basis inverse and
    state at the same pivot; the solve then resumes to the oracle's optimum."""
    for A, b, c, T in ((*lpgen.dense_lp(2, 300, 600), 40),
                       (*lpgen.degenerate_lp(1, 200, 400, budget_row=True), 120)):
        m = A.shape[0]
        ref = oracle.solve(A, b, c)
        T = min(T, len(ref.enter) - 3)  # stop before the optimum
        _say(f"case: reinvert at pivot {T} of {len(ref.enter)}, m={m}")
        o = oracle.Oracle(A, b, c)
        o.run(T)
        Binv_o, xB_o, W_o, z_o = o.state()
        with lpg.LP(A, b, c) as p:
            assert p.solve(T) == oracle.ITER_LIMIT
            basis = p.solution()["basis"]
            np.testing.assert_array_equal(basis, o.result().basis)
            p.reinvert()
            Binv, xB, W, z = p.tableau()
            exact = oracle.basis_inverse(A, basis)
            scale = np.abs(exact).max()
            assert np.abs(Binv - exact).max() <= 1e-10 * scale
            assert np.abs(Binv - Binv_o).max() <= 1e-9 * scale
            assert np.abs(xB - xB_o).max() <= 1e-9 * (1 + np.abs(xB_o).max())
            assert np.abs(W - W_o).max() <= 1e-9 * (1 + np.abs(W_o).max())
            assert abs(z - z_o) <= 1e-9 * (1 + abs(z_o))
            assert p.stats()["reinversions"] == 1
            st = p.solve()
            sol = p.solution()
        assert st == ref.status
        assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * max(1.0, abs(ref.objective))


def test_reinvert_slack_basis_is_identity(lpg):
    A, b, c = lpgen.dense_lp(0, 50, 70)
    with lpg.LP(A, b, c) as p:
        p.reinvert()
        Binv, xB, W, z = p.tableau()
    assert np.array_equal(Binv, np.eye(50)) and np.array_equal(xB, b) and not W.any() and z == 0.0


@pytest.mark.parametrize("m", [1, 37, 128, 129, 200, 1100, 2100, 4200])
def test_reinvert_all_structural_basis(lpg, m):
    """k = m structural basic columns: the single-workgroup inverse (k <= 128) and every
    panel shape of the blocked LU (R up to 4200)."""
    A, b, c = _square_lp(m, m)
    _say(f"case: square LP m=n={m}, reinvert at the optimum")
    with lpg.LP(A, b, c) as p:
        assert p.solve() == oracle.OPTIMAL
        sol = p.solution()
        assert (sol["basis"] < m).all()
        Binv0, xB0, W0, z0 = p.tableau()
        p.reinvert()
        Binv, xB, W, z = p.tableau()
        assert p.stats()["reinv_failed"] == 0
    B = A[:, sol["basis"]]
    rows = np.random.default_rng(0).choice(m, min(m, 64), replace=False)
    assert np.abs(Binv[rows] @ B - np.eye(m)[rows]).max() < 1e-11
    assert np.abs(Binv - Binv0).max() <= 1e-10 * np.abs(Binv).max()
    assert np.abs(xB - xB0).max() <= 1e-10 * np.abs(xB).max()
    assert np.abs(W - W0).max() <= 1e-10 * np.abs(W).max()
    assert abs(z - z0) <= 1e-10 * abs(z)


@pytest.mark.parametrize("m", [300, 2100])
def test_mixed_square_lp(lpg, m):
    """Reinversions of every size on the way to k = m."""
    A, b, c = _square_lp(m + 1, m)
    st64, sol64, _, _ = _solve(lpg, A, b, c)
    st, sol, _, stats = _solve(lpg, A, b, c, precision="mixed")
    assert st == st64 == oracle.OPTIMAL
    err, _ = _report(f"square m={m}", A, b, c, sol, sol64["objective"])
    assert err <= OBJ_RTOL
    assert stats["reinversions"] == sol["iterations"] // 64 and stats["reinv_failed"] == 0
    assert_kkt(A, b, c, sol["x"], sol["y"])


def test_mixed_profile_modes_agree(lpg):
    A, b, c = lpgen.dense_lp(4, 500, 1000)
    base = _solve(lpg, A, b, c, precision="mixed")
    for prof in (1, 2):
        st, sol, piv, stats = _solve(lpg, A, b, c, precision="mixed", profile=prof)
        assert st == base[0] and sol["objective"] == base[1]["objective"]
        np.testing.assert_array_equal(piv["enter"], base[2]["enter"])
        assert stats["price32_ms"] > 0 and stats["shortlist_ms"] > 0 and stats["update_ms"] > 0
        assert stats["price32_bytes"] > 0
        _say(f"  profile={prof}: price32 {stats['price32_ms']:.2f} ms shortlist {stats['shortlist_ms']:.2f} ms "
             f"update {stats['update_ms']:.2f} ms")


def test_mixed_reset_is_deterministic(lpg):
    A, b, c = lpgen.dense_lp(5, 700, 1400)
    with lpg.LP(A, b, c, precision="mixed") as p:
        p.solve()
        s1, p1 = p.solution(), p.pivots()
        r1 = p.stats()["reinversions"]
        p.reset()
        p.solve()
        s2, p2 = p.solution(), p.pivots()
        assert p.stats()["reinversions"] == r1 > 0
    assert s1["objective"] == s2["objective"]
    np.testing.assert_array_equal(p1["enter"], p2["enter"])
    np.testing.assert_array_equal(s1["x"], s2["x"])


@pytest.mark.parametrize("opts", [dict(shortlist_k=1), dict(shortlist_k=5), dict(iters_per_sync=3),
                                  dict(iters_per_sync=64, reinv_period=100), dict(sense="min")])
def test_mixed_options(lpg, opts):
    A, b, c = lpgen.dense_lp(6, 300, 600)
    sense = opts.get("sense", "max")
    if sense == "min":
        c = -c
    ref = oracle.solve(A, b, c, sense=sense)
    st, sol, _, stats = _solve(lpg, A, b, c, precision="mixed", **opts)
    assert st == ref.status
    assert abs(sol["objective"] - ref.objective) <= OBJ_RTOL * max(1.0, abs(ref.objective))
    assert_kkt(A, b, c, sol["x"], sol["y"], sense=sense)
    if opts.get("iters_per_sync") == 64:
        # read-backs every 64 pivots: a reinversion runs at the first read-back at least
        # 100 pivots after the previous one, i.e. at 128, 256, ...
        assert stats["reinversions"] == sol["iterations"] // 128


def test_mixed_rejects_entries_beyond_fp32_range(lpg):
    """The mixed form screens with an FP32 copy of A': an entry beyond FLT_MAX is an
    argument error there (host and device inputs), and accepted by the FP64 path."""
    import torch
    A, b, c = lpgen.dense_lp(1, 4, 5)
    A[2, 3] = 1e39
    with pytest.raises(lpg.LPError) as e:
        lpg.LP(A, b, c, precision="mixed")
    assert e.value.code == -1
    dA = torch.from_numpy(np.asfortranarray(A).T.copy()).cuda().t()
    with pytest.raises(lpg.LPError) as e:
        lpg.LP.from_torch(dA, torch.from_numpy(b).cuda(), torch.from_numpy(c).cuda(), precision="mixed")
    assert e.value.code == -1
    with lpg.LP(A, b, c) as p:
        assert p.solve() in (lpg.LP_OPTIMAL, lpg.LP_UNBOUNDED)


def test_mixed_unbounded_and_trivial(lpg):
    A, b, c = lpgen.dense_lp(2, 20, 30)
    A[:, 5] = -np.abs(A[:, 5])
    c[5] = 100.0
    ref = oracle.solve(A, b, c)
    with lpg.LP(A, b, c, precision="mixed") as p:
        st = p.solve()
        stats = p.stats()
    assert st == ref.status == oracle.UNBOUNDED and stats["ray"] == ref.ray
    A, b, c = lpgen.dense_lp(3, 20, 30)
    with lpg.LP(A, b, -c, precision="mixed") as p:
        assert p.solve() == oracle.OPTIMAL
        stats = p.stats()
        assert stats["iterations"] == 0 and stats["full_prices"] == 1


def test_mixed_8000x16000_against_oracle(lpg):
    """The mixed-precision configuration: objective error and residuals against the FP64
    oracle's optimum (its whole solve is stored by tests/golden/make_goldens.py), and the
    FP64 GPU path's time on the same GPU for comparison."""
    import make_goldens
    g = make_goldens.load("dense_m8000_n16000_s0")
    _say("case: dense m=8000 n=16000 seed 0, mixed vs the FP64 oracle")
    A, b, c = lpgen.dense_lp(0, 8000, 16000)
    st64, sol64, piv64, s64 = _solve(lpg, A, b, c)
    st, sol, piv, stats = _solve(lpg, A, b, c, precision="mixed")
    assert st == st64 == oracle.OPTIMAL and g["status"] == "OPTIMAL"
    err, _ = _report("mixed 8000x16000 vs oracle", A, b, c, sol, g["objective"])
    assert err <= OBJ_RTOL
    assert_kkt(A, b, c, sol["x"], sol["y"])
    # without a fallback or a reinversion changing the order of events, the mixed form
    # takes the oracle's pivots; the first ones are compared
    k = 12
    np.testing.assert_array_equal(piv["enter"][:k], np.asarray(g["enter"][:k]))
    np.testing.assert_array_equal(piv["row"][:k], np.asarray(g["row"][:k]))
    _say(f"  pivots {sol['iterations']} (oracle {g['iterations']}); solve {stats['solve_ms']:.1f} ms "
         f"(FP64 path {s64['solve_ms']:.1f} ms); reinversions {stats['reinversions']} in {stats['reinv_ms']:.1f} ms; "
         f"full FP64 passes {stats['full_prices']}")
