"""Autotuner of the row mapping of the gathering kernels.

    python -m paper_2112_07862_amd.tune [--workloads swiss_roll_100k sphere_1m]
                                        [--candidates default wide ...] [--build-only]

Each candidate is a set of build-time parameters (lanes per row for
one-chunk rows, entries per round for wider rows, rounds in flight for
each).  The tuner builds one library per candidate under _build/tune/,
then, on a GPU, runs bench.py on each workload against each library (in a
subprocess, selected by MEMBED_LIBRARY) and prints nodes/s and the average
Chebyshev step time, best first.  The library's defaults are the winner of
this sweep on the manifold workloads; a different graph family can be tuned
the same way and built with the winning parameters
(`paper_2112_07862_amd.build.build(defines=...)`).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys

from . import build as B

# name -> (lanes per row for one-chunk rows, entries per round, rounds for
# one-chunk rows, rounds for wider rows)
CANDIDATES = {
    "default": (4, 2, 6, 8),
    "one_chunk_8r": (4, 2, 8, 8),
    "wide": (8, 4, 4, 4),
    "narrow": (2, 1, 12, 16),
    "mid": (8, 2, 4, 8),
}


def defines(c):
    l1, epl, u1, u = c
    return (f"ME_ROW_LANES_1={l1}", f"ME_ROW_EPL={epl}", f"ME_ROW_UNR_1={u1}", f"ME_ROW_UNR={u}")


def lib_path(name: str) -> str:
    return os.path.join(B.OBJ, "tune", f"libmembed_{name}.so")


def build_all(names, jobs=8):
    os.makedirs(os.path.join(B.OBJ, "tune"), exist_ok=True)
    for name in names:
        B.build(jobs=jobs, defines=defines(CANDIDATES[name]), out=lib_path(name))
        print(f"[tune] built {name}: {' '.join(defines(CANDIDATES[name]))}", flush=True)


def measure(name: str, workload: str, steps: int, warmup: int) -> dict:
    env = dict(os.environ, MEMBED_LIBRARY=lib_path(name))
    cmd = [sys.executable, os.path.join(B.ROOT, "bench.py"), "--workload", workload,
           "--steps", str(steps), "--warmup", str(warmup), "--no-cpu-baseline"]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{name} {workload}: bench failed\n{r.stderr[-2000:]}")
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"nodes_per_s": d["value"], "step_us": d["roofline"]["avg_us"],
            "iterations": d["iterations"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["swiss_roll_100k", "sphere_1m"])
    ap.add_argument("--candidates", nargs="+", default=list(CANDIDATES))
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--build-only", action="store_true")
    a = ap.parse_args()
    build_all(a.candidates)
    if a.build_only:
        return 0
    rows = []
    for name in a.candidates:
        res = {w: measure(name, w, a.steps, a.warmup) for w in a.workloads}
        rows.append((name, res))
        print(f"[tune] {name}: " + "  ".join(
            f"{w} {r['nodes_per_s']:.0f} nodes/s, step {r['step_us']:.2f} us"
            for w, r in res.items()), flush=True)
    # rank by the geometric mean of nodes/s over the workloads
    def score(item):
        prod = 1.0
        for r in item[1].values():
            prod *= r["nodes_per_s"]
        return prod ** (1.0 / len(item[1]))
    rows.sort(key=score, reverse=True)
    print("[tune] ranking (geometric mean of nodes/s):")
    for name, res in rows:
        print(f"  {name:<14} {score((name, res)):>12.0f}  {' '.join(defines(CANDIDATES[name]))}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
