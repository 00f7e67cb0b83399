"""The entry point that allocates nothing (lp_solve_device_noalloc), through the C ABI,
against the entry points it stands for (lp_create_device + lp_solve + lp_get_solution):
two calls in a row on one GPU, the second with a smaller LP, so that the second runs on the
array the first one left behind (the last pair with rows of 1024 and more: B^-1 as compact
columns in the array too)."""
import sys

import numpy as np
import pytest

import lpgen

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


def _device(torch, A, b, c):
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    return dA, torch.from_numpy(b).cuda(), torch.from_numpy(c).cuda()


@pytest.mark.parametrize("sizes", [((400, 800, 0), (130, 257, 1)), ((1000, 2000, 2), (61, 90, 3)),
                                   ((1100, 600, 4), (1030, 300, 5))])
def test_noalloc_matches_the_handle_path(lpg, sizes):
    import torch
    torch.cuda.set_device(0)
    for m, n, seed in sizes:
        _say(f"case: lp_solve_device_noalloc dense m={m} n={n} seed {seed}")
        A, b, c = lpgen.dense_lp(seed, m, n)
        dA, db, dc = _device(torch, A, b, c)
        x = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        y = torch.full((m,), np.nan, dtype=torch.float64, device="cuda")
        obj = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        st, it = lpg.solve_device_noalloc(dA, db, dc, x, y, obj)
        torch.cuda.synchronize()
        with lpg.LP.from_torch(dA, db, dc) as p:
            st_ref = p.solve()
            sol = p.solution()
        assert st == st_ref == lpg.LP_OPTIMAL
        assert it == sol["iterations"]
        np.testing.assert_array_equal(x.cpu().numpy(), sol["x"])
        np.testing.assert_array_equal(y.cpu().numpy(), sol["y"])
        assert obj.item() == sol["objective"]


def test_noalloc_rejects_what_does_not_fit(lpg):
    import torch
    torch.cuda.set_device(0)
    A, b, c = lpgen.dense_lp(0, 3000, 6000)  # about 216 MB of buffers
    dA, db, dc = _device(torch, A, b, c)
    with pytest.raises(lpg.LPError) as e:
        lpg.solve_device_noalloc(dA, db, dc)
    assert "bytes" in str(e.value)
    A2, b2, c2 = _device(torch, A[:50, :80], b[:50].copy(), c[:80].copy())
    with pytest.raises(lpg.LPError):
        lpg.solve_device_noalloc(A2, b2, c2, precision=lpg.LP_MIXED)
    b2[3] = -1.0
    with pytest.raises(lpg.LPError) as e:
        lpg.solve_device_noalloc(A2, b2, c2)
    assert e.value.code == -2
