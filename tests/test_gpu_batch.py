"""Batched embedding (many graphs in one solve) through the C ABI.

Bars: every graph of a batch matches the CPU FP64 oracle to the same bars as
a single solve (eigenvalues relative 1e-6, sine of the largest B-principal
angle 1e-5 with the tolerance set from the smallest relative gap, X^T B X = I
to 1e-10); a graph's result in a batch is bitwise identical to the same graph
solved as a batch of one; a failing graph does not disturb the others."""
import os

import numpy as np
import pytest
import torch

import oracle
import synthgraphs as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def me():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2112_07862_amd as pkg
    pkg.load()
    return pkg


def _mix():
    """Uneven sizes, all three block widths, eps = 0 graphs, a dense one, a
    disconnected one."""
    return [
        ("square_1500", sg.manifold_graph("square", 1500, 8, 11), 4),
        ("swiss_2000", sg.manifold_graph("swiss_roll", 2000, 8, 12), 8),
        ("torus_1200", sg.manifold_graph("torus", 1200, 8, 13), 16),
        ("sphere_900", sg.manifold_graph("sphere", 900, 10, 14), 8),
        ("square_600", sg.manifold_graph("square", 600, 8, 15), 16),
        ("grid_bipartite", sg.grid(20, 25), 4),
        ("ring_203", sg.ring(203, 3), 5),
        ("tri_mesh", sg.tri_mesh(3), 3),
        # two components: the order's search moves on to the second one
        ("two_squares", sg.disjoint_union([sg.manifold_graph("square", 400, 8, 16),
                                           sg.manifold_graph("square", 300, 8, 17)]), 4),
    ]


_oracle = {}


def _oracle_of(name, g, K):
    if name not in _oracle:
        ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
        lam, V = oracle.generalized_eigs(ops["A"], ops["b"], K)
        _oracle[name] = (ops, lam, V)
    return _oracle[name]


def _tol(mix):
    gaps = []
    for name, g, K in mix:
        _, lam, _ = _oracle_of(name, g, K)
        if K < g.n:
            gaps.append((lam[K] - lam[K - 1]) / abs(lam[K - 1]) if lam[K - 1] != 0 else 1.0)
    return min(1e-6, 1e-5 * min(gaps) / 4)


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_oracle(me, precision):
    mix = _mix()
    tol = _tol(mix)
    print(f"[gpu] batch of {len(mix)} {precision} tol={tol:.2e}", flush=True)
    res = me.embed_batch([g for _, g, _ in mix], [K for _, _, K in mix], tol=tol, seed=5,
                         precision=precision)
    for (name, g, K), (X, lam, info) in zip(mix, res):
        ops, lam_o, V_o = _oracle_of(name, g, K)
        assert info["status"] in (0, 2), (name, info)
        lam = _np(lam)
        # |lambda| below 1e-8 a_max counts as zero (the library's residual convention)
        scale = np.maximum(np.abs(lam_o[:K]), 1e-8 * ops["A"].diagonal().max())
        assert np.max(np.abs(lam - lam_o[:K]) / scale) <= 1e-6, (name, lam, lam_o[:K])
        X = _np(X)
        s = oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"])
        assert s <= 1e-5, (name, s)
        G = X.T @ (ops["b"][:, None] * X)
        assert np.abs(G - np.eye(K)).max() <= 1e-10, name


def test_batch_alone_bitwise(me):
    """A graph's arithmetic does not depend on its batch companions."""
    mix = _mix()
    graphs = [g for _, g, _ in mix]
    Ks = [K for _, _, K in mix]
    together = me.embed_batch(graphs, Ks, tol=1e-8, seed=2, precision="mixed")
    for q, (name, g, K) in enumerate(mix):
        alone = me.embed_batch([g], [K], tol=1e-8, seed=2, precision="mixed")[0]
        Xa, la, ia = alone
        Xt, lt, it = together[q]
        assert ia["status"] == it["status"], name
        assert ia["iterations"] == it["iterations"], (name, ia["iterations"], it["iterations"])
        assert ia["eps_iterations"] == it["eps_iterations"], name
        assert torch.equal(Xa, Xt), name
        assert torch.equal(la, lt), name
        assert ia["eps"] == it["eps"] and ia["mu"] == it["mu"], name


def test_batch_single_graph_matches_embed(me):
    """A batch of one and the single-graph entry point agree to the solve tolerance."""
    g = sg.manifold_graph("square", 2000, 8, 0)
    X1, l1, i1 = me.embed(g, 4, tol=1e-8, seed=0)
    X2, l2, i2 = me.embed_batch([g], [4], tol=1e-8, seed=0)[0]
    assert i1["status"] == 0 and i2["status"] == 0
    np.testing.assert_allclose(_np(l1), _np(l2), rtol=1e-9)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    assert oracle.sin_principal_angle_b(_np(X1), _np(X2), ops["b"]) <= 1e-6


def test_batch_of_one_takes_fp16_iterates(me):
    """A batch of one graph is an engine of one graph, so FP16 iterates apply
    there (the run differs from the FP32 one) and its pairs agree with the
    single-graph entry point's FP16 solve to the solve tolerance."""
    g = sg.manifold_graph("square", 2000, 8, 0)
    X1, l1, i1 = me.embed(g, 8, tol=1e-8, seed=0, precision="mixed", cheb_iterates="fp16")
    X2, l2, i2 = me.embed_batch([g], [8], tol=1e-8, seed=0, precision="mixed",
                                cheb_iterates="fp16")[0]
    X3, l3, i3 = me.embed_batch([g], [8], tol=1e-8, seed=0, precision="mixed")[0]
    assert i1["status"] == 0 and i2["status"] == 0 and i3["status"] == 0
    assert not np.array_equal(_np(X2), _np(X3))
    np.testing.assert_allclose(_np(l1), _np(l2), rtol=1e-9)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    assert oracle.sin_principal_angle_b(_np(X1), _np(X2), ops["b"]) <= 1e-6


def test_batch_failing_graph_isolated(me):
    """A malformed graph reports its own error; the others are unaffected."""
    good = sg.manifold_graph("square", 800, 8, 21)
    bad = sg.manifold_graph("square", 700, 8, 22)
    # a self loop on node 0 (keep the CSR sorted and symmetric)
    rp, col, val = bad.rowptr.copy(), bad.col.copy(), bad.val.copy()
    ins = int(np.searchsorted(col[rp[0]:rp[1]], 0))
    col = np.insert(col, rp[0] + ins, 0)
    val = np.insert(val, rp[0] + ins, 1.0)
    rp = rp.copy()
    rp[1:] += 1
    bad = sg.CSR(bad.n, rp, col, val)
    res = me.embed_batch([good, bad, good], [4, 4, 8], tol=1e-8, seed=1)
    assert res[1][2]["status_name"] == "ME_ERR_SELF_LOOP"
    assert res[1][0] is None
    alone4 = me.embed_batch([good], [4], tol=1e-8, seed=1)[0]
    alone8 = me.embed_batch([good], [8], tol=1e-8, seed=1)[0]
    assert torch.equal(res[0][0], alone4[0]) and torch.equal(res[2][0], alone8[0])


def test_batch_mix_recipe_small(me):
    """The batched-mix recipe (uniform manifold from square / Swiss roll /
    torus, 8-NN, K in {4, 8, 16}, log-uniform N) at small N: every graph
    converges and matches the oracle."""
    specs = sg.batch_specs(count=12, seed=1000, nmin=300, nmax=1500)
    graphs = [sg.manifold_graph(kind, n, k, s) for kind, n, k, K, s in specs]
    Ks = [K for _, _, _, K, _ in specs]
    mix = [(f"mix{q}", g, K) for q, (g, K) in enumerate(zip(graphs, Ks))]
    tol = _tol(mix)
    res = me.embed_batch(graphs, Ks, tol=tol, seed=0, precision="mixed")
    for (name, g, K), (X, lam, info) in zip(mix, res):
        ops, lam_o, V_o = _oracle_of(name, g, K)
        assert info["status"] == 0, (name, info)
        assert np.max(np.abs(_np(lam) - lam_o[:K]) / np.abs(lam_o[:K])) <= 1e-6, name
        assert oracle.sin_principal_angle_b(_np(X), V_o[:, :K], ops["b"]) <= 1e-5, name


def test_fp16_iterates_never_depend_on_the_batch(me):
    """FP16 iterates are chosen by the call (one input graph), not by how many
    graphs reach the solver: a large graph beside a tiny one (solved densely)
    or beside a malformed one gets bitwise the FP32-iterate result it gets
    beside a second large graph."""
    big = sg.manifold_graph("square", 2000, 8, 0)
    big2 = sg.manifold_graph("torus", 1800, 8, 1)
    tiny = sg.tri_mesh(3)
    bad = sg.manifold_graph("square", 500, 8, 2)
    val = bad.val.copy()
    val[5] = -1.0
    bad = sg.CSR(bad.n, bad.rowptr, bad.col, val)
    kw = dict(tol=1e-8, seed=0, precision="mixed", cheb_iterates="fp16")
    ref = me.embed_batch([big, big2], [8, 8], **kw)[0]
    fp32 = me.embed_batch([big, big2], [8, 8], tol=1e-8, seed=0, precision="mixed")[0]
    assert torch.equal(ref[0], fp32[0])
    for other, K in ((tiny, 3), (bad, 4)):
        got = me.embed_batch([big, other], [8, K], **kw)[0]
        assert got[2]["status"] == 0 and got[2]["iterations"] == ref[2]["iterations"]
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    solo = me.embed_batch([big], [8], **kw)[0]
    assert not torch.equal(solo[0], ref[0])


def _gen(spec):
    kind, n, k, K, seed = spec
    return sg.manifold_graph(kind, n, k, seed)


def _oracle_of_spec(spec):
    kind, n, k, K, seed = spec
    g = sg.manifold_graph(kind, n, k, seed)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    lam, V = oracle.generalized_eigs(ops["A"], ops["b"], K, dense_max=1500)
    return ops["eps"], ops["b"], lam, V[:, :K]


def _one_blas_thread():
    # the pool's processes share the host's cores: one BLAS thread each
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


@pytest.mark.timeout(900)
def test_batch_full_recipe_512(me):
    """The full batched recipe: 512 graphs (seeds 1000 + g), N log-uniform in
    [500, 20000], square / Swiss roll / torus, 8-NN, K in {4, 8, 16}, mixed
    precision, tol 1e-6, one batched call.  Every graph converges; every 16th
    graph is compared with the oracle (eps relative 1e-9, eigenvalues relative
    1e-6, B-principal angle 1e-5 where tol / relgap allows it) and is bitwise
    equal to the same graph solved as a batch of one."""
    from concurrent.futures import ProcessPoolExecutor
    specs = sg.batch_specs(count=512)
    workers = min(16, os.cpu_count() or 1)
    print("[gpu] batch recipe: generating 512 graphs and 32 oracle solves", flush=True)
    with ProcessPoolExecutor(max_workers=workers, initializer=_one_blas_thread) as ex:
        graphs = list(ex.map(_gen, specs, chunksize=8))
        sample = list(range(0, 512, 16))
        ref = dict(zip(sample, ex.map(_oracle_of_spec, [specs[q] for q in sample])))
    Ks = [s[3] for s in specs]
    tol = 1e-6
    print(f"[gpu] batch recipe 512 graphs, total N {sum(g.n for g in graphs)}", flush=True)
    res = me.embed_batch(graphs, Ks, tol=tol, seed=0, precision="mixed")
    for q, (X, lam, info) in enumerate(res):
        assert info["status"] == 0 and info["max_residual"] <= tol, (q, specs[q], info)
    for q in sample:
        X, lam, info = res[q]
        eps_o, b, lam_o, V_o = ref[q]
        K = Ks[q]
        assert abs(info["eps"] - eps_o) <= 1e-9 * eps_o, (q, info["eps"], eps_o)
        lam = _np(lam)
        assert np.max(np.abs(lam - lam_o[:K]) / lam_o[:K]) <= 1e-6, (q, specs[q])
        relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
        if tol / relgap <= 2.5e-6:
            assert oracle.sin_principal_angle_b(_np(X), V_o, b) <= 1e-5, (q, specs[q])
        Xa, la, ia = me.embed_batch([graphs[q]], [K], tol=tol, seed=0, precision="mixed")[0]
        assert ia["iterations"] == info["iterations"], q
        assert torch.equal(Xa, X) and torch.equal(la, res[q][1]), q
