"""The benchmark's command-line contract, checked without a GPU: more than one GPU is
refused with a message and a nonzero exit before anything touches a device, and the
defaults describe the single-GPU headline workload."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for n in (2, 8):
        res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                             capture_output=True, text=True, timeout=120)
        assert res.returncode == 2, res
        assert "one GPU" in res.stderr and res.stdout == ""


def test_defaults_are_the_headline_workload():
    """Defaults (read from bench.py's argument declarations, not by running it): one GPU,
    the m = 4000, n = 8000 dense LP, 64 pivots per graph replay; the roofline peak is the
    MI355X's 8 TB/s."""
    sys.path.insert(0, ROOT)
    import bench
    src = open(os.path.join(ROOT, "bench.py")).read()
    for decl in ('"--gpus", type=int, default=1', '"--m", type=int, default=4000', '"--n", type=int, default=8000',
                 '"--iters-per-sync", type=int, default=64'):
        assert decl in src, decl
    assert bench.HBM_PEAK_GBS == 8000.0
    assert set(bench.KERNEL_NAMES) >= {"price", "update", "finish"}
