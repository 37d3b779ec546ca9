#!/usr/bin/env python3
"""Writes sphere_1m_reference.json: the CPU FP64 oracle's values for the
1,000,000-point sphere graph (uniform on the unit 2-sphere plus isotropic
noise of standard deviation 1e-3, symmetrised 12-NN, Gaussian weights,
seed 0), the largest configuration of the method, where the oracle cannot
run inside a test.

Calls only `oracle` (and `synthgraphs` for the input).  eps = lambda_2(Q)
(Section 4.2) and the K + 1 smallest generalized eigenvalues of (A, B)
(Section 4.3) come from ARPACK Lanczos for the smallest algebraic
eigenvalues (products only; a sparse LU of these operators does not fit).
That route agrees with the shift-invert route to 2e-12 relative on a
50,000-point sphere (tests/test_oracle_pins.py pins both on smaller graphs).

    python tests/golden/make_sphere_1m_reference.py   (about an hour, ~20 GB)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthgraphs as sg  # noqa: E402

N, KNN, K, SEED = 1_000_000, 12, 16, 0
SAMPLE_SEED, SAMPLE = 5, 200


def pattern_sha256(rowptr, col) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(rowptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(col, dtype=np.int32).tobytes())
    return h.hexdigest()


def main():
    t0 = time.time()
    g = sg.manifold_graph("sphere", N, KNN, SEED)
    print(f"graph {time.time() - t0:.0f} s nnz={g.nnz}", flush=True)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val, eps_method="smallest")
    print(f"operators {time.time() - t0:.0f} s eps={ops['eps']!r}", flush=True)
    lam, _ = oracle.sparse_generalized_eigs(ops["A"], ops["b"], K, method="smallest")
    print(f"eigenvalues {time.time() - t0:.0f} s", flush=True)
    rows = np.sort(np.random.default_rng(SAMPLE_SEED).choice(N, SAMPLE, replace=False))
    qd = ops["Q"].diagonal()
    out = {
        "graph": {"manifold": "sphere", "n": N, "knn": KNN, "seed": SEED, "nnz": int(g.nnz),
                  "w_sha256": pattern_sha256(g.rowptr, g.col)},
        "K": K,
        "eps": float(ops["eps"]),
        "mu": float(ops["mu"]),
        "components": int(ops["components"]),
        "max_qdiag": float(qd.max()),
        "nnz_t": int(len(ops["t_col"])),
        "t_sha256": pattern_sha256(ops["t_rowptr"], ops["t_col"]),
        "t_count_sha256": hashlib.sha256(
            np.ascontiguousarray(ops["t_count"], dtype=np.int32).tobytes()).hexdigest(),
        "mean_log_r": float(np.mean(np.log(ops["r"]))),
        "lam": [float(x) for x in lam],
        "sample_rows": rows.tolist(),
        "d": [float(x) for x in ops["d"][rows]],
        "qdiag": [float(x) for x in qd[rows]],
        "r": [float(x) for x in ops["r"][rows]],
        "b": [float(x) for x in ops["b"][rows]],
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "sphere_1m_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"done {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
