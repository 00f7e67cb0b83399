"""Writes the whole-solve (or long-prefix) pivot logs of the CPU oracle that the GPU
parity tests compare against, at the sizes the benchmark runs.

Calls only the oracle (its -fopenmp build, whose results are bit-identical to the
sequential build: tests/test_oracle_omp.py) and the seeded generators of lpgen; nothing
here reads a GPU result.  Each file records the oracle source's hash, the law, the seed
and the sizes, the status, the pivot count, the objective (user's sense), the final basis,
the pivot log (entering variable, leaving row, leaving variable, flags) and each pivot's
decision margin (how close its closest decision came to its threshold or rival value).

    python tests/golden/make_goldens.py [--threads T] [NAME ...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import lpgen  # noqa: E402
import oracle  # noqa: E402

# name: (law, seed, m, n, pivot cap or None for the default 10 (m + n), what the case covers)
GOLDENS = {
    "dense_m4000_n8000_s0": ("dense", 0, 4000, 8000, None,
                             "the benchmark's configuration: the whole solve"),
    "dense_m8000_n16000_s0": ("dense", 0, 8000, 16000, None,
                              "the mixed-precision configuration, solved in FP64: the whole solve"),
    "dense_m6000_n300_s0": ("dense", 0, 6000, 300, None,
                            "a row stride above 4800, where the update runs its larger workgroups"),
    "diagonal_m9700_n1300_s0": ("diagonal", 0, 9700, 1300, None,
                                "near the row limit, with more than 1024 slacks leaving the basis"),
    "dense_m12000_n150_s0": ("dense", 0, 12000, 150, None,
                             "rows longer than the update kernel's whole-vector staging (chunked dense pass)"),
    "diagonal_m12000_n1600_s0": ("diagonal", 0, 12000, 1600, None,
                                 "long rows in sparse-column mode (staging at the entries of D) until D "
                                 "passes ld/8, then chunked dense"),
    "degenerate_m5000_n10000_s0": ("degenerate", 0, 5000, 10000, 3000,
                                   "the degenerate law at full size: a 3000-pivot prefix"),
    "degenerate_budget_m5001_n10000_s0": ("degenerate_budget", 0, 5000, 10000, 3000,
                                          "the bounded companion (budget row) at full size: a 3000-pivot prefix"),
}


def make(law, seed, m, n):
    if law == "dense":
        return lpgen.dense_lp(seed, m, n)
    if law == "diagonal":
        return lpgen.diagonal_lp(seed, m, n)
    if law == "degenerate":
        return lpgen.degenerate_lp(seed, m, n)
    if law == "degenerate_budget":
        return lpgen.degenerate_lp(seed, m, n, budget_row=True)
    raise ValueError(law)


def oracle_sha16():
    with open(os.path.join(ROOT, "oracle", "simplex_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def path_of(name):
    return os.path.join(HERE, f"{name}.json")


def generate(name, threads=0):
    law, seed, m, n, cap, what = GOLDENS[name]
    A, b, c = make(law, seed, m, n)
    lib = oracle.omp_lib(threads)
    t0 = time.perf_counter()
    o = oracle.Oracle(A, b, c, lib_path=lib)
    o.run(cap)
    r = o.result()
    dt = time.perf_counter() - t0
    rec = {
        "_what": f"oracle pivot log, {what}",
        "_command": f"python tests/golden/make_goldens.py {name}",
        "oracle_sha16": oracle_sha16(),
        "law": law, "seed": seed, "m": int(A.shape[0]), "n": n, "pivot_cap": cap,
        "status": r.status_name, "iterations": int(r.iterations), "objective": float(r.objective),
        "counts": {k: int(v) for k, v in r.counts.items()}, "ray": int(r.ray),
        "basis": [int(v) for v in r.basis],
        "enter": [int(v) for v in r.enter], "row": [int(v) for v in r.row],
        "leave": [int(v) for v in r.leave], "flags": [int(v) for v in r.flags],
        "margin": [float(f"{v:.4g}") if v != float("inf") else None for v in r.margin],
        "oracle_seconds": round(dt, 1), "oracle_threads": oracle.threads(lib),
    }
    with open(path_of(name), "w") as f:
        json.dump(rec, f, separators=(",", ":"))
        f.write("\n")
    return rec


def load(name):
    with open(path_of(name)) as f:
        return json.load(f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(GOLDENS))
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    for name in args.names:
        rec = generate(name, args.threads)
        print(f"{name}: {rec['status']} after {rec['iterations']} pivots, objective {rec['objective']!r}, "
              f"{rec['oracle_seconds']} s on {rec['oracle_threads']} threads", flush=True)


if __name__ == "__main__":
    main()
