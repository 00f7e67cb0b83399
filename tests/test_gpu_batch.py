"""Batched form: one persistent launch solves many LPs; each must equal lp_solve on that LP
alone (status, pivot count, pivot log, objective bit for bit), which itself follows the
oracle.  Covered in both execution modes (one wavefront per LP, one workgroup per LP) and
under the autotuner, on mixed sizes, degenerate and cycling LPs, and the 4096-LP batch."""
import json
import os
import sys

import numpy as np
import pytest

import lpgen
import oracle
from lputil import assert_kkt

pytestmark = pytest.mark.gpu


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


def _serial(lpg, A, b, c, **opts):
    with lpg.LP(A, b, c, **opts) as p:
        st = p.solve()
        sol = p.solution()
        piv = p.pivots()
    return st, sol, piv


def _check_against_serial(lpg, lps, res, bt, idx, **opts):
    for i in idx:
        A, b, c = lps[i]
        st, sol, piv = _serial(lpg, A, b, c, **opts)
        g = bt.get(i)
        assert res["status"][i] == st, (i, res["status"][i], st)
        assert res["iterations"][i] == sol["iterations"], (i, res["iterations"][i], sol["iterations"])
        assert res["objective"][i] == sol["objective"], (i, res["objective"][i], sol["objective"])
        np.testing.assert_array_equal(g["enter"], piv["enter"])
        np.testing.assert_array_equal(g["row"], piv["row"])
        np.testing.assert_array_equal(g["flags"], piv["flags"])
        np.testing.assert_array_equal(g["basis"], sol["basis"])
        np.testing.assert_array_equal(g["x"], sol["x"])


def _mixed_batch(seed, count, m_lo, m_hi):
    ms, ns = lpgen.batch_sizes(seed, count, m_lo, m_hi)
    return [lpgen.dense_lp(lpgen.instance_seed(seed, i), int(ms[i]), int(ns[i])) for i in range(count)]


@pytest.mark.parametrize("small_m", [0, 64, -1])
def test_batch_equals_serial(lpg, small_m):
    _say(f"case: 40 dense LPs m in [16,120], batch_small_m={small_m}")
    lps = _mixed_batch(3, 40, 16, 120)
    with lpg.Batch(lps, batch_small_m=small_m) as bt:
        bt.solve()
        res = bt.results()
        stats = bt.stats()
        _check_against_serial(lpg, lps, res, bt, range(len(lps)))
    if small_m == 0:
        assert stats["narrow_lps"] == 0
    if small_m == 64:
        assert stats["narrow_lps"] == sum(1 for A, _, _ in lps if A.shape[0] <= 64)
    assert (res["status"] == oracle.OPTIMAL).all()


@pytest.mark.parametrize("binv", [64, 256])
def test_batch_binv_in_lds_equals_serial(lpg, binv):
    """LPs that keep B^-1 in LDS (a second persistent launch) still equal lp_solve bit for
    bit, on dense, degenerate (ties, tabu list) and overflowing LPs."""
    from test_gpu_parity import NUMERICAL_LPS
    lps = _mixed_batch(3, 40, 16, 120)
    lps += [lpgen.degenerate_lp(s, 60 + 10 * s, 120 + 20 * s, budget_row=True) for s in range(3)]
    lps += NUMERICAL_LPS
    _say(f"case: {len(lps)} LPs, B^-1 in LDS for m <= {binv}")
    with lpg.Batch(lps, batch_small_m=0, batch_binv_lds_m=binv) as bt:
        bt.solve()
        res = bt.results()
        stats = bt.stats()
        _check_against_serial(lpg, lps, res, bt, range(len(lps)))
    assert stats["binv_lds_m"] == binv
    assert stats["binv_lds_lps"] == sum(1 for A, _, _ in lps if A.shape[0] <= binv)
    assert stats["binv_lds_lps"] > 0


def test_batch_degenerate_and_special_lps(lpg):
    """Ties, the tabu list, unbounded, trivially optimal and overflowing (NUMERICAL) LPs
    inside one batch."""
    from test_oracle_pins import _embedded
    lps = [lpgen.degenerate_lp(s, 60 + 10 * s, 120 + 20 * s, budget_row=True) for s in range(6)]
    lps += [lpgen.degenerate_lp(s, 40, 80) for s in range(4)]
    lps += [_embedded("beale"), _embedded("chvatal")]
    with open(os.path.join(os.path.dirname(__file__), "golden", "cycling_lps.json")) as f:
        cyc = json.load(f)
    for name in ("beale", "chvatal"):
        d = cyc[name]
        lps.append((np.array(d["A"], float), np.array(d["b"], float), np.array(d["c"], float)))
    A, b, c = lpgen.dense_lp(2, 20, 30)
    A[:, 5] = -np.abs(A[:, 5])
    c[5] = 100.0
    lps.append((A, b, c))
    A, b, c = lpgen.dense_lp(3, 20, 30)
    lps.append((A, b, -c))
    from test_gpu_parity import NUMERICAL_LPS
    lps += NUMERICAL_LPS
    for small_m in (0, 64):
        _say(f"case: special LPs, batch_small_m={small_m}")
        with lpg.Batch(lps, batch_small_m=small_m) as bt:
            bt.solve()
            res = bt.results()
            for i, (A, b, c) in enumerate(lps):
                ref = oracle.solve(A, b, c)
                g = bt.get(i)
                assert res["status"][i] == ref.status, (i, res["status"][i], ref.status)
                np.testing.assert_array_equal(g["enter"], ref.enter)
                np.testing.assert_array_equal(g["row"], ref.row)
                np.testing.assert_array_equal(g["flags"], ref.flags)
                assert abs(res["objective"][i] - ref.objective) <= 1e-9 * max(1.0, abs(ref.objective))
            _check_against_serial(lpg, lps, res, bt, range(len(lps)))


def test_batch_sparse_column_mode(lpg):
    """LPs long enough (ld >= 1024) for the update and FTRAN to switch to the columns of
    B^-1 that can differ from unit vectors: the batched solver takes the same switch, so it
    still equals lp_solve bit for bit."""
    lps = [lpgen.dense_lp(11 + k, m, 2 * m) for k, m in enumerate((1024, 1100, 1257))]
    lps.append(lpgen.degenerate_lp(4, 1030, 2060, budget_row=True))
    _say("case: batch of 4 LPs m in {1024, 1100, 1257, 1030 degenerate}")
    for small_m in (0, -1):
        _say(f"  batch_small_m={small_m}: batched solve")
        with lpg.Batch(lps, batch_small_m=small_m) as bt:
            bt.solve()
            res = bt.results()
            _say("  serial solves")
            _check_against_serial(lpg, lps, res, bt, range(len(lps)))
        assert (res["status"][:3] == oracle.OPTIMAL).all()
    # the serial run did use sparse mode: less than the dense read of B^-1 per launch
    A, b, c = lps[1]
    with lpg.LP(A, b, c, profile=1) as p:
        p.solve()
        st = p.stats()
    m = A.shape[0]
    assert st["update_launches"] > 0
    assert st["update_bytes"] < 8.0 * m * m * st["update_launches"]


def test_batch_iteration_limit(lpg):
    lps = _mixed_batch(5, 12, 30, 80)
    with lpg.Batch(lps, max_iter=7) as bt:
        bt.solve()
        res = bt.results()
        _check_against_serial(lpg, lps, res, bt, range(len(lps)), max_iter=7)
    limited = res["status"] == oracle.ITER_LIMIT
    assert limited.any() and (res["iterations"][limited] == 7).all()
    assert (res["iterations"][~limited] <= 7).all() and (res["status"][~limited] == oracle.OPTIMAL).all()


def test_batch_4096_mixed_sizes(lpg):
    """The batched configuration: 4096 LPs, m ~ U{16..256}, n = 2m, per-instance seeds."""
    _say("case: 4096 LPs m in [16,256]")
    lps = lpgen.batch_lps(0, 4096)
    with lpg.Batch(lps) as bt:
        bt.solve()
        res = bt.results()
        stats = bt.stats()
        _say(f"  solve {stats['solve_ms']:.2f} ms, narrow {stats['narrow_lps']} wide {stats['wide_lps']}, "
             f"B^-1 in LDS {stats['binv_lds_lps']} (m <= {stats['binv_lds_m']}), "
             f"tune {stats['tune_ms']:.0f} ms, mask {stats['narrow_bucket_mask']:#x}")
        assert (res["status"] == oracle.OPTIMAL).all()
        rng = np.random.default_rng(0)
        sample = sorted(set(rng.choice(4096, 24, replace=False).tolist()) | {0, 4095})
        _check_against_serial(lpg, lps, res, bt, sample)
        for i in sample[:8]:
            A, b, c = lps[i]
            ref = oracle.solve(A, b, c)
            g = bt.get(i)
            np.testing.assert_array_equal(g["enter"], ref.enter)
            np.testing.assert_array_equal(g["row"], ref.row)
        for i in range(4096):
            A, b, c = lps[i]
            g = bt.get(i)
            # duals from the basis: KKT certificate of every LP's optimum
            m = A.shape[0]
            M = np.hstack([A, np.eye(m)])
            y = np.linalg.solve(M[:, g["basis"]].T, np.concatenate([c, np.zeros(m)])[g["basis"]])
            assert_kkt(A, b, c, g["x"], y)


def test_tune_table_round_trip(lpg, tmp_path):
    """The autotuner's modes saved to a JSON table are taken by a new batch without timing,
    and the results do not depend on where the modes came from."""
    lps = _mixed_batch(5, 300, 16, 200)
    path = str(tmp_path / "tune.json")
    with lpg.Batch(lps) as bt:
        bt.solve()
        bt.tune_save(path)
        s1 = bt.stats()
        r1 = bt.results()
    text = open(path).read()
    recs = json.loads(text)
    assert any("bucket" in r for r in recs) and any("binv_lds_m" in r for r in recs)
    with lpg.Batch(lps) as bt:
        bt.tune_load(path)
        bt.solve()
        s2 = bt.stats()
        r2 = bt.results()
    _say(f"  tune {s1['tune_ms']:.1f} ms from scratch, {s2['tune_ms']:.1f} ms with the table "
         f"({s2['tuned_from_table']} buckets)")
    assert s2["tuned_from_table"] > 0
    assert s2["narrow_bucket_mask"] == s1["narrow_bucket_mask"] and s2["binv_lds_m"] == s1["binv_lds_m"]
    for k in ("status", "iterations", "objective"):
        np.testing.assert_array_equal(r1[k], r2[k])


def test_batch_generated_on_device(lpg):
    """lp_batch_create_dense: the 4096-LP batch law generated in device memory equals, bit
    for bit in its results, the same law built by the tests' generator and uploaded."""
    _say("case: 4096 LPs generated on the device vs the same LPs from host arrays")
    lps = lpgen.batch_lps(0, 4096)
    with lpg.Batch.dense(4096, 0) as g:
        assert [A.shape for A, _, _ in lps] == list(zip(g.m.tolist(), g.n.tolist()))
        g.solve()
        rg = g.results()
        sample = [0, 1, 2047, 4095]
        xg = [g.get(i)["x"] for i in sample]
    with lpg.Batch(lps) as h:
        h.solve()
        rh = h.results()
        xh = [h.get(i)["x"] for i in sample]
    for k in ("status", "objective", "iterations"):
        np.testing.assert_array_equal(rg[k], rh[k])
    for a, b in zip(xg, xh):
        np.testing.assert_array_equal(a, b)
    assert (rg["status"] == oracle.OPTIMAL).all()
