"""Benchmark of the dense revised simplex iteration on one MI355X.

A step is one simplex iteration (pricing, FTRAN, ratio test, B^-1 update) of the dense
LP  max c^T x  s.t.  A'x <= b, x >= 0  with m = 4000 rows and n = 8000 columns
(A'_ij ~ U(0,1), b_i ~ U(1,10), c_j ~ U(1,10), seed 0), all data resident in HBM.
W warm-up pivots run first, then exactly K pivots of the iteration graph are timed
(`value`).  A second pass of K pivots launches the same kernels directly, each with
start and stop HIP events bound to its dispatch, for the per-kernel durations behind
the roofline of the dominant kernel.  The printed line also carries the time to
optimality (median of 5 solves after a warm-up), the mixed-precision form against the
FP64 path and against the FP64 path with the same reinversion period on its own
configuration, the batched form (solve, and with the host-to-device upload), and the CPU
oracle's rate on a bounded sample of the same solve.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

_ROOT = os.path.dirname(os.path.abspath(__file__))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

METRIC = "simplex iter/s + solve time (m=4000,n=8000); batched LPs/s; % HBM peak"
HBM_PEAK_GBS = 8000.0
# Profile keys and the kernels they time.  In the FP64 form "price" counts every pricing
# pass: k_price for the first iteration of each launch sequence and k_price_fin (the
# previous iteration's ratio-test finish fused with the pricing pass) for the others, which
# "price_fin" also shows alone; "finish" is the k_finish that closes each sequence.
KERNEL_NAMES = {"price": "k_price", "price_fin": "k_price_fin", "update": "k_update", "finish": "k_finish",
                "price32": "k_price32", "shortlist": "k_shortlist"}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_steps(lp, k):
    """Exactly k pivots from the current state (lp_iterate: no iteration runs past them); an
    LP that finishes early restarts from the slack basis (inside the timed region)."""
    remaining = k
    while remaining > 0:
        cur = lp.stats()["iterations"]
        st = lp.iterate(remaining)
        done = lp.stats()["iterations"] - cur
        remaining -= done
        if remaining > 0 and st != 0:  # finished before the target: start over
            lp.reset()


def measured_traffic(kernel):
    """HBM bytes per launch (read + write, copy-calibrated) recorded under profiles/ for the
    current kernel source, or None if no summary matches it."""
    import glob
    import hashlib
    src = os.path.join(_ROOT, "paper_1803_04378_amd", "csrc", "lp_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(_ROOT, "profiles", "*.md"))):
        text = open(path).read()
        for block in text.split("```json")[1:]:
            try:
                rec = json.loads(block.split("```")[0])
            except ValueError:
                continue
            if rec.get("kernel_sha16") == sha and kernel in rec.get("traffic_bytes", {}):
                return rec["traffic_bytes"][kernel]
    return None


def kernel_table(s0, s1):
    """Per-kernel average duration (HIP events of the profiling mode) and, for the
    streaming kernels, algorithmic bytes per launch and the rate they imply.  In the mixed
    form the FP32 screening and shortlist kernels run once per iteration (their launch
    count is the update kernel's); its rare FP64 passes run inside the screening kernel's
    launch and are not timed separately."""
    out = {}
    for name in KERNEL_NAMES:
        ms = s1[f"{name}_ms"] - s0[f"{name}_ms"]
        key = "update" if name in ("price32", "shortlist") else name
        launches = s1[f"{key}_launches"] - s0[f"{key}_launches"]
        if launches <= 0 or ms <= 0:
            continue
        avg_s = ms / launches * 1e-3
        row = dict(launches=launches, avg_us=round(avg_s * 1e6, 3))
        if name in ("price", "price_fin", "update", "price32"):
            # (k_price and k_price_fin stream the same columns: bytes per pricing pass)
            bkey = "price" if name == "price_fin" else name
            blaunch = s1[f"{bkey}_launches"] - s0[f"{bkey}_launches"] if name == "price_fin" else launches
            byts = (s1[f"{bkey}_bytes"] - s0[f"{bkey}_bytes"]) / blaunch
            row.update(bytes_per_launch=byts, gbs=round(byts / avg_s / 1e9, 1))
        out[name] = row
    return out


def timed_leg(lpg, torch, dev, opts, warmup, steps, profile):
    with lpg.LP.from_torch(*dev, profile=profile, **opts) as lp:
        run_steps(lp, warmup)
        torch.cuda.synchronize()
        s0 = lp.stats()
        t0 = time.perf_counter()
        run_steps(lp, steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s1 = lp.stats()
    return t1 - t0, kernel_table(s0, s1)


def timed_solves(lp, torch, reps):
    """One warm-up solve, then `reps` solves from the slack basis; returns the times and
    the status of the last one."""
    lp.solve()
    times = []
    for _ in range(reps):
        lp.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = lp.solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times, st


def solve_leg(lpg, torch, dev, opts, reps=5):
    """Time to optimality: median of `reps` solves after a warm-up solve."""
    with lpg.LP.from_torch(*dev, **opts) as lp:
        times, st = timed_solves(lp, torch, reps)
        sol = lp.solution()
    ts = statistics.median(times)
    return dict(status=lpg.STATUS_NAMES[st], seconds=round(ts, 5), runs=[round(t, 5) for t in times],
                iterations=sol["iterations"], objective=sol["objective"], iter_per_s=round(sol["iterations"] / ts, 1))


def mixed_leg(lpg, torch, m, n, seed, steps, stream, profile_only=False, reps=5):
    """Mixed-precision form on its own configuration (dense law, m x n): time to optimality
    against the FP64 path on the same GPU, objective error and KKT residuals against the
    FP64 path's optimum, the objective errors of both against the FP64 oracle's optimum
    where its whole solve is stored, and a profiled stretch of iterations for the
    per-kernel split."""
    import numpy as np

    import lpgen
    A, b, c = lpgen.dense_lp(seed, m, n)
    with torch.cuda.stream(stream):
        dA = torch.from_numpy(A.T).to("cuda").t()
        db = torch.from_numpy(b).cuda()
        dc = torch.from_numpy(c).cuda()
    torch.cuda.synchronize()
    dev = (dA, db, dc)
    opts = dict(iters_per_sync=16, stream=stream.cuda_stream)
    out = {"workload": f"dense LP m={m}, n={n}, seed {seed}; FP32 shortlist top-16 re-priced in FP64, "
                       f"FP64 reinversion every 64 pivots; times are medians of {reps} solves after a warm-up"}
    sols = {}
    # the plain FP64 path, the same with reinversion every 64 pivots (separates the two
    # effects), and the mixed form
    variants = {"fp64": dict(precision="fp64"), "fp64_reinv64": dict(precision="fp64", reinv_period=64),
                "mixed": dict(precision="mixed")}
    for prec, vopt in (() if profile_only else variants.items()):
        with lpg.LP.from_torch(*dev, **vopt, **opts) as lp:
            times, st = timed_solves(lp, torch, reps)
            ts = statistics.median(times)
            sol = lp.solution()
            stt = lp.stats()
            if prec == "mixed":
                # one reinversion of the optimal basis (the largest basis block of the solve)
                t0 = time.perf_counter()
                for _ in range(3):
                    lp.reinvert()
                torch.cuda.synchronize()
                reinv_opt = dict(k=int((sol["basis"] < n).sum()), ms=round((time.perf_counter() - t0) / 3 * 1e3, 3))
        sols[prec] = sol
        row = dict(status=lpg.STATUS_NAMES[st], seconds=round(ts, 5), runs=[round(t, 5) for t in times],
                   iterations=sol["iterations"], iter_per_s=round(sol["iterations"] / ts, 1),
                   objective=sol["objective"])
        if prec != "fp64":
            # reinversion counters of the last solve (stats restart at each reset)
            row.update(reinversions=stt["reinversions"], reinv_ms=round(stt["reinv_ms"], 3))
        if prec == "mixed":
            row.update(full_fp64_prices=stt["full_prices"], reinversion_at_optimum=reinv_opt)
        out[prec] = row
    if sols:
        out["speedup_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 4)
        out["speedup_vs_fp64_reinv64"] = round(out["fp64_reinv64"]["seconds"] / out["mixed"]["seconds"], 4)
        ref = sols["fp64"]["objective"]
        x, y = sols["mixed"]["x"], sols["mixed"]["y"]
        slack = b - A @ x
        red = A.T @ y - c
        out["error_vs_fp64"] = dict(objective_rel=abs(sols["mixed"]["objective"] - ref) / max(1.0, abs(ref)),
                                    primal=float(max(0.0, -slack.min(), -x.min())),
                                    dual=float(max(0.0, -red.min(), -y.min())),
                                    gap=float(abs(c @ x - b @ y)))
        # against the FP64 oracle's optimum, stored with its whole solve by
        # tests/golden/make_goldens.py (the default workload only)
        gold = os.path.join(_ROOT, "tests", "golden", f"dense_m{m}_n{n}_s{seed}.json")
        if os.path.exists(gold):
            with open(gold) as f:
                g = json.load(f)
            go = g["objective"]
            out["error_vs_oracle"] = dict(
                oracle_objective=go, oracle_pivots=len(g["enter"]),
                mixed_objective_rel=abs(sols["mixed"]["objective"] - go) / max(1.0, abs(go)),
                fp64_objective_rel=abs(sols["fp64"]["objective"] - go) / max(1.0, abs(go)),
                fp64_pivots_equal=sols["fp64"]["iterations"] == len(g["enter"]))
    with lpg.LP.from_torch(*dev, precision="mixed", profile=2, **opts) as lp:
        run_steps(lp, 40)
        torch.cuda.synchronize()
        s0 = lp.stats()
        run_steps(lp, steps)
        torch.cuda.synchronize()
        s1 = lp.stats()
    out["kernels"] = kernel_table(s0, s1)
    del dA, db, dc
    return out


def general_leg(lpg, torch, m, n, seed, stream, reps=3):
    """Two-phase start (rows <=, >=, =, b of any sign), general-row law at m x n: time to
    optimality (median of `reps` solves after a warm-up, phase switch included), the split
    between the phases, and the optimality residuals of the GPU's result for the given rows."""
    import numpy as np

    import lpgen
    A, b, c, rt = lpgen.general_lp(seed, m, n)
    t0 = time.perf_counter()
    lp = lpg.LP(A, b, c, row_type=rt, stream=stream.cuda_stream)
    create = time.perf_counter() - t0
    with lp:
        times, st = timed_solves(lp, torch, reps)
        sol = lp.solution()
        stats = lp.stats()
    ts = statistics.median(times)
    x, y = sol["x"], sol["y"]
    Ax = A @ x
    viol = np.where(rt == 0, Ax - b, np.where(rt == 1, b - Ax, np.abs(Ax - b)))
    # max sense: A^T y >= c, y >= 0 on <= rows, y <= 0 on >= rows
    red = A.T @ y - c
    ysign = np.where(rt == 0, -y, np.where(rt == 1, y, 0.0))
    return dict(workload=f"general-row LP m={m}, n={n}, seed {seed}: A'~U(0,1), rows >= (5%), = (2%), "
                         f"<= (rest), 5% negated (b < 0), b on the dense law's scale, c~U(1,10); "
                         f"{int((rt == 1).sum())} >= rows, "
                         f"{int((rt == 2).sum())} = rows, {int((b < 0).sum())} with b < 0",
                status=lpg.STATUS_NAMES[st], seconds=round(ts, 5), runs=[round(t, 5) for t in times],
                iterations=sol["iterations"], iter_per_s=round(sol["iterations"] / ts, 1),
                phase1_pivots=stats["phase1_iterations"], drive_outs=stats["drive_outs"],
                switch_ms=round(stats["phase_switch_ms"], 3), objective=sol["objective"],
                primal_violation=float(max(0.0, viol.max())),
                dual_violation=float(max(0.0, -red.min(), ysign.max())),
                gap=float(abs(c @ x - b @ y)), create_s=round(create, 4))


def batch_leg(lpg, count, serial_sample):
    """Batched form: `count` LPs, m ~ U{16..256}, n = 2m, dense law with per-instance seeds,
    solved in one persistent launch, against serial lp_solve calls on a sample of them; and
    the same batch generated in device memory (creation without the host -> device upload)."""
    import numpy as np

    import lpgen
    lps = lpgen.batch_lps(0, count)
    t0 = time.perf_counter()
    bt0 = lpg.Batch(lps)  # host -> device upload of every LP (and the pooled work memory)
    create = time.perf_counter() - t0
    import tempfile
    table = os.path.join(tempfile.mkdtemp(prefix="lpgpu_tune_"), "batch_tune.json")
    with bt0 as bt:
        t0 = time.perf_counter()
        bt.solve()  # the first solve also runs the autotuner
        first = time.perf_counter() - t0
        bt.tune_save(table)
        t0 = time.perf_counter()
        bt.solve()
        wall = time.perf_counter() - t0
        st = bt.stats()
        res = bt.results()
    # a second batch of the same law that takes the saved table: its first solve times nothing
    with lpg.Batch(lps) as bt2:
        bt2.tune_load(table)
        t0 = time.perf_counter()
        bt2.solve()
        first_cached = time.perf_counter() - t0
        st2 = bt2.stats()
    # the same batch generated in device memory (no host arrays, no upload): creation time,
    # and its results against the uploaded batch's, bit for bit
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with lpg.Batch.dense(count, 0) as bg:
        gen_create = time.perf_counter() - t0
        bg.tune_load(table)
        bg.solve()
        stg = bg.stats()
        rg = bg.results()
    gen_same = all(np.array_equal(rg[k], res[k]) for k in ("status", "objective", "iterations"))
    iters = int(res["iterations"].sum())
    idx = list(range(0, count, max(1, count // serial_sample)))[:serial_sample]
    handles = [lpg.LP(*lps[i]) for i in idx]
    for h in handles[:4]:
        h.solve()
        h.reset()
    t0 = time.perf_counter()
    for h in handles:
        h.solve()
    serial = (time.perf_counter() - t0) / len(handles)
    for h in handles:
        h.close()
    lps_per_s = count / (st["solve_ms"] * 1e-3)
    model = batch_bytes(lps, res["iterations"])
    return dict(lps=count, lps_per_s=round(lps_per_s, 1), solve_ms=round(st["solve_ms"], 3),
                model_bytes=model, model_gbs=round(model / (st["solve_ms"] * 1e-3) / 1e9, 1),
                first_solve_ms_with_tuning=round(first * 1e3, 3),
                lps_per_s_first_solve=round(count / first, 1),
                first_solve_ms_from_tune_table=round(first_cached * 1e3, 3),
                tune_ms_from_table=round(st2["tune_ms"], 1), buckets_from_table=st2["tuned_from_table"],
                lps_per_s_first_solve_from_table=round(count / first_cached, 1),
                create_ms=round(create * 1e3, 3),
                lps_per_s_with_upload=round(count / (create + st["solve_ms"] * 1e-3), 1),
                create_ms_generated_on_device=round(gen_create * 1e3, 3),
                lps_per_s_with_generation=round(count / (gen_create + stg["solve_ms"] * 1e-3), 1),
                generated_equals_uploaded=bool(gen_same),
                wall_ms=round(wall * 1e3, 3), pivots=iters, all_optimal=bool((res["status"] == 1).all()),
                narrow_lps=st["narrow_lps"], wide_lps=st["wide_lps"], tune_ms=round(st["tune_ms"], 1),
                serial_ms_per_lp=round(serial * 1e3, 4), serial_sample=len(handles),
                serial_lps_per_s=round(1.0 / serial, 1), speedup_vs_serial=round(lps_per_s * serial, 1))


def batch_bytes(lps, iters):
    """Algorithmic bytes of the batched solve: per pivot of an m x n LP, pricing reads A'
    (8 m n, nonbasic columns bounded by n) and the update reads and writes B^-1 with FTRAN
    on the way (16 m ld); the B^-1 term is an upper bound (the sparse-column mode of LPs with
    ld >= 1024 touches fewer columns, none here)."""
    total = 0.0
    for (A, _, _), k in zip(lps, iters):
        m, n = A.shape
        ld = (m + 7) // 8 * 8
        total += float(k) * (8.0 * m * n + 16.0 * m * ld)
    return total


def reinversion_leg(lpg, torch, m, stream, reps=3):
    """One reinversion of an all-structural basis (k = m): the nearly diagonal law m x m is
    solved to its optimum, whose basis holds every structural column, then lp_reinvert is
    timed.  FLOPs: LU 2/3 k^3, the two triangular solves of X = M^-1 2 k^3 (m = k: no
    -B21 B11^-1 product); rate against the FP64 matrix peak of 78.6 TFLOP/s."""
    import lpgen
    A, b, c = lpgen.diagonal_lp(1, m, m)
    with lpg.LP(A, b, c, stream=stream.cuda_stream) as lp:
        st = lp.solve()
        k = int((lp.solution()["basis"] < m).sum())
        lp.reinvert()  # warm
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            lp.reinvert()
            times.append(time.perf_counter() - t0)
        failed = lp.stats()["reinv_failed"]
    ts = statistics.median(times)
    flops = (2.0 / 3.0) * k ** 3 + 2.0 * k ** 3
    return dict(workload=f"nearly diagonal LP m=n={m} at its optimum (status {lpg.STATUS_NAMES[st]}), "
                         f"basis block k={k}", k=k, ms=round(ts * 1e3, 3), runs_ms=[round(t * 1e3, 3) for t in times],
                gflop=round(flops / 1e9, 2), tflops=round(flops / ts / 1e12, 3),
                frac_fp64_mfma_peak=round(flops / ts / 78.6e12, 4), failed=failed)


def degenerate_leg(lpg, torch, stream, warmup=200, steps=2000):
    """The degenerate law at full size (5000 x 10000, and 5001 x 10000 with the budget row):
    iterations/s over `steps` pivots after `warmup`."""
    import lpgen
    out = {}
    for name, budget in (("degenerate_m5000_n10000", False), ("degenerate_budget_m5001_n10000", True)):
        A, b, c = lpgen.degenerate_lp(0, 5000, 10000, budget_row=budget)
        with lpg.LP(A, b, c, stream=stream.cuda_stream) as lp:
            run_steps(lp, warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_steps(lp, steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            stt = lp.stats()
        out[name] = dict(pivots=steps, after=warmup, seconds=round(dt, 4), iter_per_s=round(steps / dt, 1),
                         degenerate=stt["degenerate"], ties=stt["ties"])
    return out


def cpu_baseline(A, b, c, pivots, budget_s=20.0):
    """The oracle on the host's cores: its -fopenmp build (bit-identical results) on every
    core OpenMP is given, over the whole solve or as many 25-pivot chunks as fit in
    budget_s, and the sequential build on the first `pivots` pivots."""
    import oracle
    lib = oracle.omp_lib(0)
    cores = oracle.threads(lib)
    o = oracle.Oracle(A, b, c, lib_path=lib)
    t0 = time.perf_counter()
    st = oracle.ITER_LIMIT
    while st == oracle.ITER_LIMIT and time.perf_counter() - t0 < budget_s:
        st = o.run(o.iterations + 25)
    dt = time.perf_counter() - t0
    done = o.iterations
    whole = st != oracle.ITER_LIMIT
    o1 = oracle.Oracle(A, b, c)
    t1 = time.perf_counter()
    o1.run(pivots)
    dt1 = time.perf_counter() - t1
    shape = f"m={A.shape[0]},n={A.shape[1]}"
    return dict(value=round(done / dt, 3), unit="iter/s", cores=cores, kind="oracle",
                sample=(f"the whole {shape} solve ({done} pivots, {oracle.STATUS_NAMES[st]}) in {dt:.1f} s"
                        if whole else f"first {done} pivots of the {shape} solve in {dt:.1f} s") +
                       f" on {cores} threads (OpenMP build, bit-identical to the sequential oracle)",
                single_core=dict(value=round(o1.iterations / dt1, 3), unit="iter/s", cores=1,
                                 sample=f"first {o1.iterations} pivots of the {shape} solve, sequential build, "
                                        f"{dt1:.1f} s"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--m", type=int, default=4000)
    ap.add_argument("--n", type=int, default=8000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--iters-per-sync", type=int, default=64)
    ap.add_argument("--cpu-pivots", type=int, default=100, help="oracle sample size (0 = skip)")
    ap.add_argument("--batch", type=int, default=4096, help="LPs in the batched leg (0 = skip)")
    ap.add_argument("--mixed-m", type=int, default=8000, help="rows of the mixed-precision leg (0 = skip)")
    ap.add_argument("--mixed-n", type=int, default=16000)
    ap.add_argument("--general-m", type=int, default=4000, help="rows of the two-phase leg (0 = skip)")
    ap.add_argument("--general-n", type=int, default=8000)
    ap.add_argument("--mixed-profile-only", action="store_true",
                    help="only the profiled stretch of the mixed-precision form (for profiler runs)")
    ap.add_argument("--reinv-m", type=int, default=3000, help="order of the reinversion leg's basis block (0 = skip)")
    ap.add_argument("--degenerate", type=int, default=1, help="degenerate-law leg at 5000 x 10000 (0 = skip)")
    ap.add_argument("--serial-sample", type=int, default=256,
                    help="LPs of the batch also solved one by one with lp_solve")
    ap.add_argument("--quick", action="store_true",
                    help="timed leg only (no cross-check, time-to-optimality or CPU legs); for profiler runs")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="finally copy a buffer of this many MiB three times: a kernel of known traffic "
                         "for scaling hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding of this "
              "path is a design note, not a built component.", file=sys.stderr)
        sys.exit(2)

    import torch

    import lpgen
    import paper_1803_04378_amd as lpg

    if args.mixed_profile_only:
        torch.cuda.set_device(0)
        stream = torch.cuda.Stream()
        _log(f"bench: mixed-precision profiled stretch m={args.mixed_m} n={args.mixed_n}")
        out = mixed_leg(lpg, torch, args.mixed_m, args.mixed_n, args.seed, args.steps, stream, profile_only=True)
        print(json.dumps({"mixed": out}), flush=True)
        return

    m, n = args.m, args.n
    _log(f"bench: generating dense LP m={m} n={n} seed={args.seed}")
    A, b, c = lpgen.dense_lp(args.seed, m, n)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dA = torch.from_numpy(A.T).to("cuda").t()  # (m, n), column-major
        db = torch.from_numpy(b).cuda()
        dc = torch.from_numpy(c).cuda()
    torch.cuda.synchronize()
    dev = (dA, db, dc)
    opts = dict(iters_per_sync=args.iters_per_sync, stream=stream.cuda_stream)

    _log(f"bench: timed leg warmup={args.warmup} steps={args.steps}")
    elapsed, _ = timed_leg(lpg, torch, dev, opts, args.warmup, args.steps, profile=0)
    value = args.steps / elapsed
    # Per-kernel durations: the same iteration launched directly, each kernel with start
    # and stop events bound to its own dispatch (no launch gaps inside the timings).
    _log("bench: per-kernel timing leg (dispatch-bound HIP events)")
    el2, kern = timed_leg(lpg, torch, dev, opts, args.warmup, args.steps, profile=2)
    streaming = {k: v for k, v in kern.items() if "gbs" in v}
    if "price_fin" in streaming:
        # all but the first pricing pass of each launch sequence run in k_price_fin: that
        # kernel, timed alone, carries the roofline ("price" mixes the two kernels)
        streaming.pop("price", None)
    dominant = max(streaming, key=lambda k: streaming[k]["avg_us"]) if streaming else None
    roofline = None
    if dominant:
        kd = kern[dominant]
        roofline = {"bound": "hbm", "achieved": kd["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(kd["gbs"] / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(KERNEL_NAMES[dominant]),
                    "kernel": KERNEL_NAMES[dominant], "bytes_per_launch": kd["bytes_per_launch"],
                    "avg_us": kd["avg_us"]}
    # model bytes of one iteration: one pricing pass and one update pass
    iter_bytes = (kern["price"]["bytes_per_launch"] + kern["update"]["bytes_per_launch"]
                  if "price" in kern and "update" in kern and "bytes_per_launch" in kern["update"] else None)

    extra = {"direct_launch_iter_per_s": round(args.steps / el2, 2)}
    if not args.quick:
        _log("bench: graph leg with event nodes around every kernel")
        el1, k1 = timed_leg(lpg, torch, dev, opts, args.warmup, args.steps, profile=1)
        extra["kernels_graph_events_us"] = {k: v["avg_us"] for k, v in k1.items()}
        extra["graph_events_iter_per_s"] = round(args.steps / el1, 2)
        _log("bench: time to optimality")
        extra["solve"] = solve_leg(lpg, torch, dev, opts)

    if not args.quick and args.mixed_m > 0:
        _log(f"bench: mixed-precision leg m={args.mixed_m} n={args.mixed_n}")
        extra["mixed"] = mixed_leg(lpg, torch, args.mixed_m, args.mixed_n, args.seed, 200, stream)

    if not args.quick and args.general_m > 0:
        _log(f"bench: two-phase leg m={args.general_m} n={args.general_n}")
        extra["two_phase"] = general_leg(lpg, torch, args.general_m, args.general_n, args.seed, stream)

    if not args.quick and args.reinv_m > 0:
        _log(f"bench: reinversion leg, k = m = {args.reinv_m}")
        extra["reinversion"] = reinversion_leg(lpg, torch, args.reinv_m, stream)

    if not args.quick and args.degenerate:
        _log("bench: degenerate law 5000 x 10000")
        extra["degenerate"] = degenerate_leg(lpg, torch, stream)

    if not args.quick and args.batch > 0:
        _log(f"bench: batched leg, {args.batch} LPs")
        extra["batch"] = batch_leg(lpg, args.batch, args.serial_sample)

    cpu = None
    if args.cpu_pivots > 0 and not args.quick:
        _log(f"bench: CPU oracle on {args.cpu_pivots} pivots")
        cpu = cpu_baseline(A, b, c, args.cpu_pivots)

    if args.calibrate_copy > 0:
        _log(f"bench: copy calibration, {args.calibrate_copy} MiB x 3")
        x = torch.empty(args.calibrate_copy << 17, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dense LP max c^T x, A'x<=b, m={m}, n={n}, A'~U(0,1), b~U(1,10), c~U(1,10), "
                               f"seed {args.seed}; plain FP64 path, Dantzig + tabu (tenure 5)",
                   "m": m, "n": n, "iters_per_sync": args.iters_per_sync},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kern,
        "iteration": {"model_bytes": iter_bytes,
                      "gbs": round(iter_bytes * value / 1e9, 1) if iter_bytes else None,
                      "frac_hbm": round(iter_bytes * value / 1e9 / HBM_PEAK_GBS, 4) if iter_bytes else None},
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
