#!/usr/bin/env python3
"""Throughput of the manifold-graph embedding hot path on one MI355X.

One step = the whole path for one graph, from the device CSR of W to the
B-orthonormal N x K FP64 embedding: validation, two-hop pattern T, Q,
eps = lambda_2(Q) (its own LOBPCG), mu, b, and the LOBPCG solve of (A, B) to
relative residual <= tol, certified in FP64.  The input CSR is resident in
HBM before the timed region starts.

Default workload: N = 1,000,000 points uniform on the unit 2-sphere plus
isotropic noise of standard deviation 1e-3, symmetrised 12-NN graph with
Gaussian weights, sigma = median 12-NN distance, K = 16, tol = 1e-6, seed 0,
mixed precision.

Prints one JSON line (rank 0): metric, value (nodes/s of the 1M sphere),
latency, roofline of the timed kernel (HIP events on its stream, algorithmic
bytes), and, as extra keys, the batched mix (512 graphs, one batched call,
beside the plain FP64 single-graph path), the serving stream at several
offered Poisson rates (p50/p99 latency below saturation and the saturation
throughput), and the CPU oracle's throughput on a bounded sample of the same
workload family.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "graph nodes embedded/sec at rel. residual ≤1e-6; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
SERVE_BASE_RATE = 200.0  # Poisson arrivals per second of the serving recipe
KERNELS = {"spmm": 1, "gram": 2, "combine": 3, "cheb": 4}
KERNEL_NAMES = {"spmm": "k_spmm (difference-form SpMM of A on the LOBPCG block)",
                "gram": "k_gram (Rayleigh-Ritz Gram S^T B S, S^T A S on MFMA)",
                "combine": "k_combine (block update X, P, AX, AP)",
                "cheb": "k_cheb_step (Chebyshev preconditioner step: fused SpMM + recurrence)"}


# committed rocprofv3 counter summaries of the Chebyshev step, by (workload,
# precision, iterate storage), each taken at the default degree and eps target
TRAFFIC_FILES = {
    ("swiss_roll_100k", "mixed", "fp32"): "cheb_step_swiss_roll_100k_hbm_bytes.txt",
    ("sphere_1m", "mixed", "fp16"): "cheb_step_fp16_sphere_1m.txt",
    ("sphere_1m", "mixed", "fp32"): "cheb_step_sphere_1m_hbm_bytes.txt",
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2112_07862_amd", "csrc", f)
                  for f in ("slot_ops.hip", "rowops.h", "engine.h", "common.h", "build.hip")]


def code_text(text: str) -> str:
    """Source text without // comments, trailing blanks and empty lines:
    edits to comments leave the kernels, and their counters, unchanged."""
    import re
    out = []
    for line in text.splitlines():
        line = re.sub(r"//.*$", "", line).rstrip()
        if line:
            out.append(line)
    return "\n".join(out)


def kernel_source_hash(texts=None) -> str:
    """sha256 of the code (comments stripped) of the kernel sources, or of
    `texts` given in the same order."""
    import hashlib
    h = hashlib.sha256()
    if texts is None:
        texts = []
        for f in KERNEL_SOURCES:
            with open(f, encoding="utf-8") as fh:
                texts.append(fh.read())
    for t in texts:
        h.update(code_text(t).encode())
    return h.hexdigest()


def measured_traffic(args):
    """HBM bytes per launch of the Chebyshev step from the committed
    rocprofv3 counter summary of this workload and configuration, or None
    when there is none or the kernel sources changed since the counters were
    taken."""
    name = TRAFFIC_FILES.get((args.workload, args.precision, args.cheb_iterates))
    if name is None or args.cheb_degree != 128 or args.eps_tol is not None:
        return None
    try:
        kv = {}
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sources_sha256") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(kind: str, n: int, knn: int, K: int, seed: int) -> dict:
    """The oracle as it stands (operators + shift-invert Lanczos) on a
    smaller graph of the same family."""
    import oracle
    import synthgraphs as sg
    g = sg.manifold_graph(kind, n, knn, seed)
    t0 = time.perf_counter()
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    oracle.generalized_eigs(ops["A"], ops["b"], K, dense_max=0)
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    return {"value": n / dt, "unit": "nodes/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{kind} N={n} {knn}-NN K={K} seed={seed}: CPU FP64 oracle (operators, "
                      f"eps by ARPACK shift-invert, K+1 pairs by ARPACK shift-invert); "
                      f"{dt:.2f} s wall, os.cpu_count()={os.cpu_count()}",
            "seconds": dt}


def _gen(spec):
    import synthgraphs as sg
    kind, n, k, K, seed = spec
    return sg.manifold_graph(kind, n, k, seed)


def _gen_serve(spec):
    import synthgraphs as sg
    t, kind, n, k, K, seed = spec
    return sg.manifold_graph(kind, n, k, seed)


def _gen_main(spec):
    import synthgraphs as sg
    kind, n, knn = spec
    return sg.manifold_graph(kind, n, knn, 0)


def generate(main_spec, batch_count: int, serve_count: int, workers: int = 16):
    """Every input graph of the run (the main workload, the batched mix with
    seeds 1000 + g, the serving stream with seed 7), generated on host worker
    processes before the GPU is touched."""
    import synthgraphs as sg
    from concurrent.futures import ProcessPoolExecutor
    bspecs = sg.batch_specs(count=batch_count) if batch_count else []
    sspecs = sg.serve_arrivals(serve_count, rate=SERVE_BASE_RATE) if serve_count else []
    with ProcessPoolExecutor(max_workers=min(workers, os.cpu_count() or 1)) as ex:
        fmain = ex.submit(_gen_main, main_spec) if main_spec else None
        bgraphs = list(ex.map(_gen, bspecs, chunksize=4))
        sgraphs = list(ex.map(_gen_serve, sspecs, chunksize=2))
        gmain = fmain.result() if fmain else None
    return gmain, (bspecs, bgraphs), (sspecs, sgraphs)


def batch_leg(me, specs, graphs, precision: str, cheb_degree: int, steps: int,
              warmup: int, launch: str = "auto") -> dict:
    """Batched mix: every graph embedded by one batched call per step
    (mixed precision); beside it the plain FP64 single-graph path (one me.embed
    per graph, FP64) on every 8th graph of the same mix."""
    import torch
    Ks = [s[3] for s in specs]
    dev = [me.to_device(g) for g in graphs]
    torch.cuda.synchronize()
    total_n = sum(g.n for g in graphs)
    opts = dict(precision=precision, seed=0, cheb_degree=cheb_degree, launch=launch)
    tol = 1e-6
    for w in range(warmup):
        t = time.perf_counter()
        me.embed_batch(dev, Ks, tol=tol, **opts)
        print(f"[bench] batch warmup {w}: {time.perf_counter() - t:.2f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    lat, bad = [], 0
    t0 = time.perf_counter()
    for s_ in range(steps):
        ts = time.perf_counter()
        res = me.embed_batch(dev, Ks, tol=tol, **opts)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        bad += sum(1 for _, _, i in res if i["status"] not in (0, 2) or i["max_residual"] > tol)
        its = [i["iterations"] for _, _, i in res]
        print(f"[bench] batch step {s_}: {lat[-1]:.2f} s, not converged {bad}, iterations "
              f"median {int(np.median(its))} max {max(its)}", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    value = total_n * steps / elapsed if bad == 0 else 0.0
    sample = list(range(0, len(graphs), 8))
    ts = time.perf_counter()
    sn, sbad = 0, 0
    for q in sample:
        X, lam, info = me.embed(dev[q], Ks[q], tol=tol, precision="fp64", seed=0,
                                cheb_degree=cheb_degree)
        sn += graphs[q].n
        sbad += info["status"] not in (0, 2) or info["max_residual"] > tol
    torch.cuda.synchronize()
    single = sn / (time.perf_counter() - ts) if sbad == 0 else 0.0
    print(f"[bench] batch {value:.0f} nodes/s, FP64 one graph at a time {single:.0f} nodes/s",
          file=sys.stderr, flush=True)
    return {
        "workload": f"batch_{len(graphs)}", "graphs": len(graphs), "total_nodes": total_n,
        "n_range": [500, 20000], "manifolds": ["square", "swiss_roll", "torus"], "knn": 8,
        "K": [4, 8, 16], "tol": tol, "precision": precision, "steps": steps,
        "nodes_per_s": value, "s_per_batch": elapsed / max(steps, 1), "failed": bad,
        "single_graph_fp64": {"nodes_per_s": single, "graphs": len(sample),
                              "note": "me.embed one graph at a time, FP64, every 8th graph "
                                      "of the same mix"},
        "speedup_vs_single_fp64": value / single if single > 0 else None,
    }


def serve_run(me, specs, dev, ns, rate: float, precision: str, cheb_degree: int) -> dict:
    """Drives the continuous-batching server with the stream's requests at
    Poisson rate `rate` (the stream's arrival gaps rescaled) against the wall
    clock; latency = completion - arrival."""
    times = [s[0] * SERVE_BASE_RATE / rate for s in specs]
    count = len(specs)
    tol = 1e-6
    srv = me.Server(precision=precision, seed=0, cheb_degree=cheb_degree)
    for q in range(2):  # warm-up: two requests through the server
        srv.submit(dev[q], 8, tol)
    while srv.step() > 0:
        pass
    srv.poll()
    arrive, lat, nodes, bad = {}, [], 0, 0
    nxt, done, steps = 0, 0, 0
    t0 = time.perf_counter()
    t_last = t0
    while done < count:
        now = time.perf_counter() - t0
        while nxt < count and times[nxt] <= now:
            t = srv.submit(dev[nxt], specs[nxt][4], tol)
            arrive[t] = (times[nxt], ns[nxt])
            nxt += 1
        if done == nxt and nxt < count:  # idle until the next arrival
            time.sleep(max(0.0, times[nxt] - (time.perf_counter() - t0)))
            continue
        srv.step()
        steps += 1
        fin = srv.poll()
        tf = time.perf_counter()
        for t, X, lam, info in fin:
            ta, n = arrive.pop(t)
            lat.append(tf - t0 - ta)
            nodes += n
            done += 1
            if info["status"] not in (0, 2) or info["max_residual"] > tol:
                bad += 1
            t_last = tf
    srv.close()
    span = t_last - t0
    offered = sum(ns) / max(times[-1], 1e-9)
    out = {"rate_per_s": rate, "offered_nodes_per_s": offered,
           "nodes_per_s": nodes / span if bad == 0 else 0.0,
           "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "span_s": span, "rounds": steps, "failed": bad}
    print(f"[bench] serve rate {rate:g}/s: offered {offered:.3g} nodes/s, served "
          f"{out['nodes_per_s']:.3g} nodes/s, p50 {out['p50_ms']:.0f} ms, p99 "
          f"{out['p99_ms']:.0f} ms", file=sys.stderr, flush=True)
    return out


FP64_VECTOR_PEAK_TFLOPS = 78.6


def _events_ms(fn, reps: int = 1):
    """Milliseconds of fn() on the current stream, HIP events around it."""
    import torch
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        r = fn()
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) / reps, r


def knn_leg(me, points_by_name: dict) -> dict:
    """GPU kNN graph construction (exact brute force) of the workloads' point
    sets; checked against the input generator's graph of the same points.
    The distance kernel is bound by FP64 vector arithmetic: per pair, dim
    subtractions, dim products and dim - 1 additions."""
    import torch
    out = {}
    for name, (x, k, g) in points_by_name.items():
        pts = torch.as_tensor(x, device="cuda")
        me.knn_graph(pts, k)  # warm-up
        ms, (csr, sigma) = _events_ms(lambda: me.knn_graph(pts, k))
        n, dim = x.shape
        same = bool(np.array_equal(csr.rowptr.cpu().numpy(), g.rowptr)
                    and np.array_equal(csr.col.cpu().numpy(), g.col))
        flops = float(n) * float(n - 1) * (3 * dim - 1)
        tf = flops / (ms * 1e-3) / 1e12
        out[name] = {"n": int(n), "dim": int(dim), "k": int(k), "ms": ms,
                     "points_per_s": n / (ms * 1e-3), "nnz": int(csr.nnz),
                     "same_graph_as_generator": same,
                     "roofline": {"bound": "alu", "achieved": tf,
                                  "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
                                  "note": "whole call (distances, selection, union); the "
                                          "distance arithmetic has no fused multiply-adds, "
                                          "so half the FMA peak is its ceiling"}}
        print(f"[bench] knn {name}: {ms:.1f} ms, {tf:.1f} TFLOP/s, same graph {same}",
              file=sys.stderr, flush=True)
        del pts, csr
    return out


def vbc_leg(me, graphs_by_name: dict) -> dict:
    """Betweenness centrality and its variance (the manifold-graph check):
    n breadth-first searches with path counts and the accumulation, about
    4 nnz edge visits per source."""
    out = {}
    for name, g in graphs_by_name.items():
        d = me.to_device(g)
        me.betweenness(d)
        ms, (cb, v) = _events_ms(lambda: me.betweenness(d))
        ev = 4.0 * g.n * g.nnz
        out[name] = {"n": int(g.n), "nnz": int(g.nnz), "ms": ms, "vbc": v,
                     "edge_visits_per_s": ev / (ms * 1e-3)}
        print(f"[bench] betweenness {name}: {ms:.1f} ms, VBC {v:.4g}", file=sys.stderr,
              flush=True)
    return out


def cluster_leg(me, per_square: int = 30000) -> dict:
    """Section 5.1's evaluation on a labelled synthetic manifold: three unit
    squares side by side, one 10-NN graph, embedded with K = 3 on the GPU;
    k-means and GMM into 3 clusters; RI, Precision, Purity and NMI of each
    and their average (Table 3's convention)."""
    import torch
    import synthgraphs as sg
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.random((per_square, 2)) + np.array([1.0 * q, 0.0])
                        for q in range(3)])
    y = torch.as_tensor(np.repeat(np.arange(3), per_square), device="cuda")
    g = sg.knn_graph(x, 10)
    X, lam, info = me.embed(g, 3, tol=1e-6, seed=0, precision="mixed")
    u = [0.2, 0.5, 0.8]
    me.kmeans(X, 3, u)
    ms_k, (lab, cen, it_k) = _events_ms(lambda: me.kmeans(X, 3, u))
    ms_g, (labg, w, mu, cov, ll, it_g) = _events_ms(lambda: me.gmm(X, 3, lab))
    sk = me.cluster_scores(y, lab, 3, 3)
    sgm = me.cluster_scores(y, labg, 3, 3)
    avg = {k: (sk[k] + sgm[k]) / 2 for k in sk}
    print(f"[bench] clustering: kmeans {ms_k:.1f} ms, gmm {ms_g:.1f} ms, average {avg}",
          file=sys.stderr, flush=True)
    return {"n": int(3 * per_square), "K": 3, "C": 3, "embed_status": info["status_name"],
            "kmeans": {"ms": ms_k, "iterations": it_k, **sk},
            "gmm": {"ms": ms_g, "iterations": it_g, **sgm}, "average": avg}


def serve_leg(me, specs, graphs, rates, precision: str, cheb_degree: int) -> dict:
    """Serving: the same request stream (N log-uniform in [1000, 200000] on
    square / Swiss roll / sphere, 10-NN, K = 8, tol 1e-6) offered at several
    Poisson rates.  The recipe's 200/s overloads one GPU; the lower rates give
    the latency below saturation.  The saturation point is the throughput
    sustained under overload."""
    import torch
    dev = [me.to_device(g) for g in graphs]
    torch.cuda.synchronize()
    ns = [g.n for g in graphs]
    runs = [serve_run(me, specs, dev, ns, r, precision, cheb_degree) for r in rates]
    top = max(runs, key=lambda r: r["rate_per_s"])
    mean_n = float(np.mean(ns))
    sat = top["nodes_per_s"]
    below = [r for r in runs if r["offered_nodes_per_s"] < 0.9 * sat]
    return {
        "workload": f"serve_{len(graphs)}", "requests": len(graphs),
        "n_range": [1000, 200000], "manifolds": ["square", "swiss_roll", "sphere"], "knn": 10,
        "K": 8, "tol": 1e-6, "precision": precision, "mean_n": mean_n, "runs": runs,
        "saturation": {"nodes_per_s": sat, "requests_per_s": sat / mean_n,
                       "note": f"throughput sustained at the highest offered rate "
                               f"({top['rate_per_s']:g}/s, "
                               f"{top['offered_nodes_per_s']:.3g} nodes/s offered)"},
        "below_saturation": [{"rate_per_s": r["rate_per_s"],
                              "load": r["offered_nodes_per_s"] / sat if sat > 0 else None,
                              "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"]} for r in below],
    }


def envelope(args, value, ms_per_step, steps, warmup, dtype, config) -> dict:
    return {"metric": METRIC, "value": value, "unit": "nodes/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def bench_batch(args) -> int:
    """A line for the batched mix alone (--workload batch)."""
    print(f"[bench] generating batch of {args.batch_count}", file=sys.stderr, flush=True)
    _, (specs, graphs), _ = generate(None, args.batch_count, 0)
    import paper_2112_07862_amd as me
    b = batch_leg(me, specs, graphs, args.precision, args.cheb_degree, args.steps, args.warmup,
                  args.launch)
    out = envelope(args, b["nodes_per_s"], b["s_per_batch"] * 1e3, args.steps, args.warmup,
                   "f64" if args.precision == "fp64" else "f32+f64",
                   {k: b[k] for k in ("workload", "graphs", "total_nodes", "n_range", "knn",
                                      "K", "tol", "precision")})
    out["batch"] = b
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args) -> int:
    """A line for the serving stream alone (--workload serve)."""
    print(f"[bench] generating {args.serve_count} requests", file=sys.stderr, flush=True)
    _, _, (specs, graphs) = generate(None, 0, args.serve_count)
    import paper_2112_07862_amd as me
    sv = serve_leg(me, specs, graphs, args.serve_rates, args.precision, args.cheb_degree)
    top = max(sv["runs"], key=lambda r: r["rate_per_s"])
    out = envelope(args, sv["saturation"]["nodes_per_s"], top["span_s"] * 1e3 / top["rounds"],
                   top["rounds"], 2, "f64" if args.precision == "fp64" else "f32+f64",
                   {k: sv[k] for k in ("workload", "requests", "n_range", "knn", "K", "tol",
                                       "precision")})
    out["latency_ms"] = {"p50": top["p50_ms"], "p99": top["p99_ms"]}
    out["serving"] = sv
    print(json.dumps(out), flush=True)
    return 0


CPU_SAMPLE_N = {"sphere_1m": 50_000, "swiss_roll_100k": 100_000, "square_2k": 2000}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere_1m",
                    help="sphere_1m (default), swiss_roll_100k, square_2k, batch or serve")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--time-kernel", default="cheb", choices=list(KERNELS))
    ap.add_argument("--cheb-degree", type=int, default=128)
    ap.add_argument("--cheb-iterates", default="fp32", choices=["fp32", "fp16"],
                    help="storage of the Chebyshev iterates (mixed precision)")
    ap.add_argument("--eps-tol", type=float, default=None)
    ap.add_argument("--launch", default="auto", choices=["auto", "stream", "graph"],
                    help="enqueue LOBPCG rounds kernel by kernel or as a replayed HIP graph")
    ap.add_argument("--cpu-sample-n", type=int, default=None,
                    help="nodes of the CPU oracle's sample graph (default per workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-mix and serving legs of the default line")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--serve-count", type=int, default=120)
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[10.0, 25.0, 40.0, 200.0],
                    help="Poisson arrival rates (requests/s) the serving stream is offered at")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device-to-device copies of MIB MiB (the known-size "
                         "reference for the HBM byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path "
              "(--gpus 1); multi-GPU sharding is described in DESIGN.md and not built.",
              file=sys.stderr)
        return 2

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}), flush=True)
        return 0
    import synthgraphs as sg

    kind, n, knn, K, tol = sg.CONFIGS[args.workload]
    extras = not args.no_extras
    print(f"[bench] generating {args.workload}: {kind} N={n} {knn}-NN K={K} tol={tol}"
          + (f"; batch of {args.batch_count}; {args.serve_count} serving requests"
             if extras else ""), file=sys.stderr, flush=True)
    g, (bspecs, bgraphs), (sspecs, sgraphs) = generate(
        (kind, n, knn), args.batch_count if extras else 0, args.serve_count if extras else 0)
    import torch
    import paper_2112_07862_amd as me
    dcsr = me.to_device(g)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    opts = dict(precision=args.precision, seed=0, cheb_degree=args.cheb_degree,
                cheb_iterates=args.cheb_iterates, launch=args.launch)
    if args.eps_tol is not None:
        opts["eps_tol"] = args.eps_tol

    def step():
        X, lam, info = me.embed(dcsr, K, tol=tol, **opts)
        return info

    for w in range(args.warmup):
        info = step()
        print(f"[bench] warmup {w}: iters={info['iterations']} eps_iters={info['eps_iterations']} "
              f"rho={info['max_residual']:.2e}", file=sys.stderr, flush=True)

    me.kernel_timing(KERNELS[args.time_kernel])
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        info = step()
        stream.synchronize()
        lat.append(time.perf_counter() - ts)
        infos.append(info)
        print(f"[bench] step {s}: {lat[-1] * 1e3:.1f} ms iters={info['iterations']} "
              f"eps_iters={info['eps_iterations']} rho={info['max_residual']:.2e} "
              f"status={info['status_name']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = me.kernel_timing_read()
    me.kernel_timing(0)

    ok = all(i["status"] in (0, 2) and i["max_residual"] <= tol for i in infos)
    value = n * args.steps / elapsed if ok else 0.0
    avg_ms = kt["total_ms"] / max(kt["launches"], 1)
    achieved = (kt["bytes"] / max(kt["launches"], 1)) / (avg_ms * 1e-3) / 1e9 if kt["launches"] else 0.0
    out = envelope(args, value, elapsed * 1e3 / args.steps, args.steps, args.warmup,
                   "f64" if args.precision == "fp64" else "f32+f64",
                   {"workload": args.workload, "manifold": kind, "n": n, "knn": knn, "K": K,
                    "tol": tol, "precision": args.precision, "preconditioner": "chebyshev",
                    "cheb_degree": args.cheb_degree, "cheb_iterates": args.cheb_iterates,
                    "launch": args.launch, "seed": 0})
    out.update({
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "note": "one graph's solve, repeated; serving latencies are under "
                               "'serving'"},
        "iterations": int(np.median([i["iterations"] for i in infos])),
        "eps_iterations": int(np.median([i["eps_iterations"] for i in infos])),
        "max_residual": max(i["max_residual"] for i in infos),
        "all_converged": ok,
        "phases_ms": {"build_incl_eps": float(np.median([i["ms_build"] for i in infos])),
                      "solve": float(np.median([i["ms_solve"] for i in infos]))},
        "roofline": {
            "kernel": KERNEL_NAMES[args.time_kernel],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args) if args.time_kernel == "cheb" else None,
            "launches": kt["launches"],
            "avg_us": avg_ms * 1e3,
            "bytes_per_launch": kt["bytes"] / max(kt["launches"], 1),
        },
    })
    # context for the roofline, outside the timed region: a plain device copy
    # moving the same bytes as one launch (and a large one), and the other
    # row-streaming kernels of the solve measured the same way
    bpl = kt["bytes"] / max(kt["launches"], 1)
    same = copy_rate(int(bpl), stream)
    large = copy_rate(2 << 30, stream)
    out["roofline"]["copy_same_bytes_GBps"] = same
    out["roofline"]["copy_2GiB_GBps"] = large
    out["roofline"]["frac_of_copy_same_bytes"] = achieved / same if same > 0 else None
    others = {}
    for kname in ("spmm", "gram"):
        me.kernel_timing(KERNELS[kname])
        step()
        stream.synchronize()
        k2 = me.kernel_timing_read()
        me.kernel_timing(0)
        if k2["launches"]:
            ms = k2["total_ms"] / k2["launches"]
            gbs = k2["bytes"] / k2["launches"] / (ms * 1e-3) / 1e9
            others[kname] = {"kernel": KERNEL_NAMES[kname], "achieved": gbs, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS, "avg_us": ms * 1e3,
                             "launches": k2["launches"],
                             "bytes_per_launch": k2["bytes"] / k2["launches"]}
    out["other_kernels"] = others
    del dcsr
    if extras:
        print("[bench] batched mix ...", file=sys.stderr, flush=True)
        out["batch"] = batch_leg(me, bspecs, bgraphs, "mixed", args.cheb_degree,
                                 args.batch_steps, 1)
        print("[bench] serving ...", file=sys.stderr, flush=True)
        out["serving"] = serve_leg(me, sspecs, sgraphs, args.serve_rates, "mixed",
                                   args.cheb_degree)
        # the rows around the path: graph construction, the manifold check,
        # the clustering of the embedding
        import synthgraphs as sg
        pts = {}
        for wl in ("swiss_roll_100k", "sphere_1m"):
            kd, nn, kk, _, _ = sg.CONFIGS[wl]
            xp = sg.sample_points(kd, nn, np.random.default_rng(0))
            pts[wl] = (xp, kk, g if wl == args.workload else sg.knn_graph(xp, kk))
        out["knn"] = knn_leg(me, pts)
        del pts
        out["vbc"] = vbc_leg(me, {"square_2k": sg.manifold_graph("square", 2000, 8, 0),
                                  "swiss_roll_20k": sg.manifold_graph("swiss_roll", 20_000, 10, 0)})
        out["clustering"] = cluster_leg(me)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cn = args.cpu_sample_n or CPU_SAMPLE_N.get(args.workload, 50_000)
        out["cpu_baseline"] = cpu_baseline(kind, min(cn, n), knn, K, 0)
    print(json.dumps(out), flush=True)
    return 0


def copy_rate(traffic_bytes: int, stream, reps: int = 50) -> float:
    """GB/s of torch's device-to-device copy moving `traffic_bytes` (half
    read, half written), timed with events on `stream`."""
    import torch
    n = max(traffic_bytes // 8, 1)  # floats per buffer: n * 4 read + n * 4 written
    a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        for _ in range(5):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.copy_(a)
        e1.record(stream)
    e1.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 8.0 * n / sec / 1e9


if __name__ == "__main__":
    sys.exit(main())
