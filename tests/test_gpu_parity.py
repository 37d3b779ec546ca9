"""Parity of the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs.

Bars: two-hop pattern, counts and sizes bit-exact; per-node scalars to FP64
rounding; eps and mu relative 1e-9; generalized eigenvalues relative 1e-6;
sine of the largest B-principal angle of the K-subspace 1e-5 (with the solve
tolerance set from the oracle's relative gap, so that the bound
sin theta <= rho / relgap is below 1e-5); X^T B X = I to 1e-10."""
import numpy as np
import pytest
import scipy.sparse as sp
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


def _graphs():
    return {
        "square_2k": lambda: sg.manifold_graph("square", 2000, 8, 0),
        "swiss_3k": lambda: sg.manifold_graph("swiss_roll", 3000, 10, 1),
        "sphere_3k": lambda: sg.manifold_graph("sphere", 3000, 12, 2),
        "torus_2500": lambda: sg.manifold_graph("torus", 2500, 8, 3),
        "random_300": lambda: sg.random_graph(300, 0.05, 4),
        # levels of 1411 and 2166 nodes: the order's node-parallel form
        "random_4000": lambda: sg.random_graph(4000, 0.0015, 7),
        "ring_40": lambda: sg.ring(40, 2),
        "ring_203": lambda: sg.ring(203, 3),
        "tri_mesh": lambda: sg.tri_mesh(3),
        "line_5": lambda: sg.line(5),
        "grid_bipartite": lambda: sg.grid(30, 40),
        "star_1500": lambda: sg.star(1500),
        "two_squares": lambda: sg.disjoint_union([sg.manifold_graph("square", 400, 8, 5),
                                                  sg.manifold_graph("square", 300, 8, 6)]),
    }


GRAPHS = _graphs()
_cache = {}


def oracle_ops(name):
    if name not in _cache:
        g = GRAPHS[name]()
        _cache[name] = (g, oracle.build_ops(g.n, g.rowptr, g.col, g.val))
    return _cache[name]


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", list(GRAPHS))
def test_operators_match_oracle(me, name):
    g, ops = oracle_ops(name)
    print(f"[gpu] operators {name} n={g.n}", flush=True)
    h = me.build_graph_ops(g)
    ex = h.export()
    # two-hop pattern: bit-exact
    assert h.nnz_t == len(ops["t_col"])
    assert np.array_equal(_np(ex["t_rowptr"]), ops["t_rowptr"])
    assert np.array_equal(_np(ex["t_col"]), ops["t_col"])
    assert np.array_equal(_np(ex["t_count"]), ops["t_count"])
    # per-node scalars
    np.testing.assert_allclose(_np(ex["d"]), ops["d"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(_np(ex["qdiag"]), ops["Q"].diagonal(), rtol=1e-13, atol=0)
    # eps, mu
    if ops["eps"] == 0.0:
        assert h.eps == 0.0 and h.mu == 0.0 and h.two_hop_disconnected == (ops["components"] > 1)
    else:
        assert abs(h.eps - ops["eps"]) <= 1e-9 * ops["eps"], (h.eps, ops["eps"])
        assert abs(h.mu - ops["mu"]) <= 1e-9 * ops["mu"]
    np.testing.assert_allclose(_np(ex["r"]), ops["r"], rtol=2e-9, atol=0)
    np.testing.assert_allclose(_np(ex["b"]), ops["b"], rtol=2e-9, atol=0)
    h.close()


@pytest.mark.parametrize("name", ["square_2k", "sphere_3k", "random_300", "ring_40", "tri_mesh",
                                  "star_1500"])
@pytest.mark.parametrize("k", [1, 3, 8, 16])
def test_apply_matches_oracle(me, name, k):
    g, ops = oracle_ops(name)
    print(f"[gpu] apply {name} k={k}", flush=True)
    h = me.build_graph_ops(g)
    X = sg.initial_block(g.n, k, 99)
    Xd = torch.tensor(X, device="cuda")
    # the handle's own eps and mu (equal to the oracle's within 1e-9)
    L, Q = ops["L"], ops["Q"]
    A = L - h.mu * Q + h.eps * sp.identity(g.n)
    for which, M in (("A", A), ("Q", Q)):
        Y = _np(h.apply(which, Xd))
        ref = M @ X
        scale = np.abs(M).max() * np.abs(X).max() * 64
        assert np.max(np.abs(Y - ref)) <= 1e-14 * scale, which
    YB = _np(h.apply("B", Xd))
    np.testing.assert_allclose(YB, ops["b"][:, None] * X, rtol=2e-9)
    h.close()


EMBED_CASES = [
    # name, K
    ("square_2k", 1),
    ("square_2k", 4),
    ("sphere_3k", 16),
    ("torus_2500", 8),
    ("swiss_3k", 8),
    ("random_300", 5),
    ("ring_203", 3),
    ("tri_mesh", 3),
]


@pytest.mark.parametrize("name,K", EMBED_CASES)
def test_embed_matches_oracle(me, name, K):
    g, ops = oracle_ops(name)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-6, 1e-5 * relgap / 4)
    print(f"[gpu] embed {name} n={g.n} K={K} tol={tol:.2e} relgap={relgap:.3g}", flush=True)
    X, lam, info = me.embed(g, K, tol=tol, seed=1)
    X, lam = _np(X), _np(lam)
    assert info["status"] == 0, info
    np.testing.assert_array_less(np.abs(lam - lam_o[:K]) / np.abs(lam_o[:K]), 1e-6)
    s = oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"])
    assert s <= 1e-5, s
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    rho = oracle.relative_residuals(ops["A"], ops["b"], X, lam)
    assert np.all(rho <= tol * 1.01 + 1e-12), rho
    # sign convention: largest-magnitude entry of each column positive
    idx = np.argmax(np.abs(X), axis=0)
    assert np.all(X[idx, np.arange(K)] > 0)


def test_embed_eps_zero_graph(me):
    """A bipartite grid: two-hop graph disconnected, eps = mu = 0, A = L;
    lambda_1 = 0 with a constant vector; the K-subspace matches the oracle's
    at the tolerance its relative gap requires."""
    g, ops = oracle_ops("grid_bipartite")
    K = 4
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-8, 1e-5 * relgap / 4)
    X, lam, info = me.embed(g, K, tol=tol, seed=2)
    assert info["status_name"] == "ME_WARN_EPS_ZERO"
    lam, X = _np(lam), _np(X)
    assert abs(lam[0]) < 1e-10
    np.testing.assert_allclose(lam[1:], lam_o[1:K], rtol=1e-6)
    assert oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"]) <= 1e-5
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    # the first column is the B-normalised constant vector
    c = np.ones(g.n) / np.sqrt(ops["b"].sum())
    assert np.max(np.abs(X[:, 0] - c)) <= 1e-6



@pytest.mark.parametrize("n,K", [(2, 1), (2, 2), (3, 2), (3, 3)])
def test_smallest_graphs(me, n, K):
    """Paths of two and three nodes: no node of either has a two-hop pair
    that keeps the two-hop graph connected (n = 2: T empty; n = 3: only the
    ends pair up), so eps = mu = 0 and A = L (Section 4.2); the K smallest
    generalized pairs of (L, B), up to K = n, against the oracle's dense
    solve."""
    g = sg.line(n, 1.5)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    h = me.build_graph_ops(g)
    assert h.eps == 0.0 and h.mu == 0.0
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    X, lam, info = me.embed(g, K, tol=1e-10, seed=0)
    assert info["status_name"] == "ME_WARN_EPS_ZERO", info
    X, lam = _np(X), _np(lam)
    np.testing.assert_allclose(lam, lam_o[:K], rtol=1e-10, atol=1e-12)
    assert oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"]) <= 1e-8
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-12


def test_degenerate_inputs_rejected(me):
    """An empty graph is an invalid argument; graphs without edges (one node,
    three nodes) have isolated nodes, which the scale b of Section 4.3 cannot
    take (r_i = 0): rejected as such, also when the caller brings the
    workspace the query sized."""
    empty = sg.CSR(0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    with pytest.raises(me.MembedError) as e:
        me.build_graph_ops(empty)
    assert e.value.name == "ME_ERR_INVALID_ARG"
    for n in (1, 3):
        edgeless = sg.CSR(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
        with pytest.raises(me.MembedError) as e:
            me.build_graph_ops(edgeless)
        assert e.value.name == "ME_ERR_ISOLATED_NODE"
        ws = torch.empty(me.build_workspace_bytes(edgeless), dtype=torch.uint8, device="cuda")
        with pytest.raises(me.MembedError) as e:
            me.build_graph_ops(edgeless, workspace=ws)
        assert e.value.name == "ME_ERR_ISOLATED_NODE"

@pytest.mark.parametrize("w", [6e4, 1e5])
def test_heavy_edge_at_the_fp16_limit(me, w):
    """One edge of a dense random graph weighted 6e4 (below FP16's largest
    finite value, 65504: packed FP16 weights) or 1e5 (past it: the
    mixed-precision preconditioner reads FP32 weights; FP16 would hold
    infinity and every preconditioned column would be dropped).  The heavy
    edge leaves lambda_max / lambda_1 near 5e7, so the bar is the oracle's
    own residual of the returned pairs at tol 1e-5 and B-orthonormality."""
    g0 = sg.random_graph(300, 0.05, 4)
    val = g0.val.copy()
    c = int(g0.col[g0.rowptr[0]])  # the edge (0, c) and its mirror
    val[g0.rowptr[0]] = w
    k = g0.rowptr[c] + np.searchsorted(g0.col[g0.rowptr[c]:g0.rowptr[c + 1]], 0)
    assert g0.col[k] == 0
    val[k] = w
    g = sg.CSR(g0.n, g0.rowptr, g0.col, val)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    tol = 1e-5
    X, lam, info = me.embed(g, 4, tol=tol, seed=1, precision="mixed")
    print(f"[gpu] heavy edge {w:g}: status {info['status_name']} "
          f"iterations {info['iterations']}", flush=True)
    assert info["status"] == 0, info
    X, lam = _np(X), _np(lam)
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    assert np.all(oracle.relative_residuals(ops["A"], ops["b"], X, lam) <= tol * 1.01 + 1e-12)
    lam_o, _ = oracle.generalized_eigs(ops["A"], ops["b"], 4)
    np.testing.assert_allclose(lam, lam_o[:4], rtol=1e-4)


def test_weights_beyond_fp32_refused_in_mixed(me):
    """A weight above FP32's largest value cannot be held by the mixed
    preconditioner's FP32 copy: the embedding is refused with a clear status
    instead of running on infinities; the build itself (FP64) accepts the
    graph."""
    g0 = sg.manifold_graph("square", 2000, 8, 0)
    g = sg.CSR(g0.n, g0.rowptr, g0.col, g0.val * 1e39)
    h = me.build_graph_ops(g)
    assert h.eps > 0.0
    with pytest.raises(me.MembedError) as e:
        me.embed(g, 4, precision="mixed")
    assert e.value.name == "ME_ERR_BAD_WEIGHT"
    # in a batch only that graph fails; its neighbour is solved
    res = me.embed_batch([g, g0], [4, 4], precision="mixed")
    assert res[0][0] is None and res[0][2]["status_name"] == "ME_ERR_BAD_WEIGHT"
    assert res[1][2]["status"] == 0


def test_plain_fp64_square_2000_tol_1e8(me):
    """The plain-method configuration: N = 2000 uniform in the unit square,
    symmetrised 8-NN, K = 4, FP64 throughout, tol 1e-8, seed 0."""
    kind, n, knn, K, tol = sg.CONFIGS["square_2k"]
    assert (kind, n, knn, K, tol) == ("square", 2000, 8, 4, 1e-8)
    g, ops = oracle_ops("square_2k")
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    X, lam, info = me.embed(g, K, tol=tol, seed=0, precision="fp64")
    assert info["status"] == 0 and info["max_residual"] <= tol, info
    X, lam = _np(X), _np(lam)
    assert np.max(np.abs(lam - lam_o[:K]) / lam_o[:K]) <= 1e-6
    rho = oracle.relative_residuals(ops["A"], ops["b"], X, lam)
    assert np.all(rho <= tol * 1.01), rho
    assert tol / relgap <= 1e-5
    assert oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"]) <= 1e-5
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10


def test_embed_with_explicit_start_block_and_determinism(me):
    g, ops = oracle_ops("square_2k")
    X0 = torch.tensor(sg.initial_block(g.n, 4, 5), device="cuda")
    X1, l1, _ = me.embed(g, 4, tol=1e-8, X0=X0)
    X2, l2, _ = me.embed(g, 4, tol=1e-8, X0=X0)
    assert torch.equal(X1, X2) and torch.equal(l1, l2)


@pytest.mark.parametrize("bad,status", [
    ("negative_weight", "ME_ERR_BAD_WEIGHT"),
    ("asymmetric", "ME_ERR_NOT_SYMMETRIC"),
    ("self_loop", "ME_ERR_SELF_LOOP"),
    ("col_range", "ME_ERR_INVALID_ARG"),
    ("unsorted", "ME_ERR_INVALID_ARG"),
    ("isolated", "ME_ERR_ISOLATED_NODE"),
    ("rowptr", "ME_ERR_INVALID_ARG"),
])
def test_invalid_graphs_rejected(me, bad, status):
    g = sg.random_graph(30, 0.2, 7, wlo=1.0, whi=2.0)
    rp, col, val = g.rowptr.copy(), g.col.copy(), g.val.copy()
    n = g.n
    if bad == "negative_weight":
        val[0] = -1.0
    elif bad == "asymmetric":
        val[2] = 0.5
    elif bad == "self_loop":
        col[0] = 0
    elif bad == "col_range":
        col[1] = n + 5
    elif bad == "unsorted":
        col[rp[3]], col[rp[3] + 1] = col[rp[3] + 1], col[rp[3]]
    elif bad == "isolated":
        g = sg.from_edges(4, np.array([0, 1]), np.array([1, 2]), np.array([1.0, 1.0]))
        rp, col, val, n = g.rowptr, g.col, g.val, g.n
    elif bad == "rowptr":
        rp[5] = rp[4] - 1
    bad_g = sg.CSR(n, rp, col.astype(np.int32), val)
    with pytest.raises(me.MembedError) as e:
        me.build_graph_ops(bad_g)
    assert e.value.name == status


def test_k_range_errors(me):
    g = sg.manifold_graph("square", 100, 8, 1)
    with pytest.raises(me.MembedError) as e:
        me.embed(g, 17)
    assert e.value.name == "ME_ERR_K_RANGE"
    with pytest.raises(me.MembedError) as e:
        me.embed(g, 0)
    assert e.value.name == "ME_ERR_K_RANGE"
    g = sg.tri_mesh(3)  # dense path: K <= n
    with pytest.raises(me.MembedError) as e:
        me.embed(g, 11)
    assert e.value.name == "ME_ERR_K_RANGE"
    # smallest LOBPCG graph with the largest block: 3 * 16 <= 49
    g = sg.ring(49, 2)
    X, lam, info = me.embed(g, 16, tol=1e-8)
    assert info["status"] == 0 and info["block"] == 16


@pytest.mark.parametrize("name,K", [("square_2k", 4), ("sphere_3k", 16), ("torus_2500", 8)])
@pytest.mark.parametrize("precond,deg,cop", [("none", None, None), ("jacobi", None, None),
                                             ("chebyshev", 8, None), ("chebyshev", 48, None),
                                             ("chebyshev", 256, None), ("chebyshev", 48, "full"),
                                             ("chebyshev", 128, "full")])
def test_embed_preconditioners(me, name, K, precond, deg, cop):
    """Every preconditioner (Jacobi, Chebyshev on L + eps I or on A) reaches
    the same pairs: the converged result does not depend on it."""
    g, ops = oracle_ops(name)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-6, 1e-5 * relgap / 4)
    X, lam, info = me.embed(g, K, tol=tol, seed=3, precond=precond, cheb_degree=deg, cheb_op=cop)
    assert info["status"] == 0, info
    lam = _np(lam)
    np.testing.assert_array_less(np.abs(lam - lam_o[:K]) / np.abs(lam_o[:K]), 1e-6)
    assert oracle.sin_principal_angle_b(_np(X), V_o[:, :K], ops["b"]) <= 1e-5


@pytest.mark.parametrize("name,K", EMBED_CASES)
def test_embed_mixed_precision_matches_oracle(me, name, K):
    """FP32 preconditioner, FP64 everything else: same bar as FP64."""
    g, ops = oracle_ops(name)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-6, 1e-5 * relgap / 4)
    X, lam, info = me.embed(g, K, tol=tol, seed=1, precision="mixed")
    assert info["status"] == 0, info
    X, lam = _np(X), _np(lam)
    np.testing.assert_array_less(np.abs(lam - lam_o[:K]) / np.abs(lam_o[:K]), 1e-6)
    assert oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"]) <= 1e-5
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    assert np.all(oracle.relative_residuals(ops["A"], ops["b"], X, lam) <= tol * 1.01 + 1e-12)


@pytest.mark.parametrize("name,K", [("sphere_3k", 16), ("torus_2500", 8), ("swiss_3k", 8),
                                    ("random_300", 5)])
def test_embed_fp16_iterates_matches_oracle(me, name, K):
    """FP16 storage of the Chebyshev iterates (block widths 8 and 16): the
    same bar as the FP32 form.  The run differs from the FP32 one, so the FP16
    kernels did the preconditioning; the default is FP32, bit for bit."""
    g, ops = oracle_ops(name)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-6, 1e-5 * relgap / 4)
    X, lam, info = me.embed(g, K, tol=tol, seed=1, precision="mixed", cheb_iterates="fp16")
    assert info["status"] == 0, info
    X, lam = _np(X), _np(lam)
    np.testing.assert_array_less(np.abs(lam - lam_o[:K]) / np.abs(lam_o[:K]), 1e-6)
    assert oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"]) <= 1e-5
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    assert np.all(oracle.relative_residuals(ops["A"], ops["b"], X, lam) <= tol * 1.01 + 1e-12)
    X32, _, i32 = me.embed(g, K, tol=tol, seed=1, precision="mixed", cheb_iterates="fp32")
    Xa, _, ia = me.embed(g, K, tol=tol, seed=1, precision="mixed")
    print(f"[gpu] {name} K={K} iterations fp16 {info['iterations']} fp32 {i32['iterations']}",
          flush=True)
    assert not np.array_equal(_np(X32), X)
    assert torch.equal(Xa, torch.as_tensor(_np(X32)).to(Xa.device)) and ia["iterations"] == i32["iterations"]


def test_fp16_iterates_fall_back_where_they_do_not_apply(me):
    """FP16 iterates serve one-slot embedding solves with one-hop entries,
    block width 8 or 16, buffer addressing and mixed precision; everywhere
    else the request runs the FP32 (or FP64) path, bit for bit."""
    g, _ = oracle_ops("swiss_3k")
    cases = [dict(K=8, precision="mixed", addressing="global"),
             dict(K=8, precision="mixed", cheb_op="full"),
             dict(K=4, precision="mixed"),
             dict(K=8, precision="fp64")]
    for c in cases:
        c = dict(c)
        K = c.pop("K")
        h = me.build_graph_ops(g, **{k: v for k, v in c.items() if k != "cheb_op"})
        X1, l1, i1 = me.embed(h, K, tol=1e-8, seed=3, cheb_iterates="fp32", **c)
        X2, l2, i2 = me.embed(h, K, tol=1e-8, seed=3, cheb_iterates="fp16", **c)
        assert i1["status"] == 0 and i1["iterations"] == i2["iterations"], (c, i1, i2)
        assert torch.equal(X1, X2) and torch.equal(l1, l2), c
        h.close()
    # a batch runs several slots per launch: FP32 iterates
    gs = [GRAPHS["square_2k"](), GRAPHS["torus_2500"]()]
    r1 = me.embed_batch(gs, [8, 8], tol=1e-8, precision="mixed", cheb_iterates="fp32")
    r2 = me.embed_batch(gs, [8, 8], tol=1e-8, precision="mixed", cheb_iterates="fp16")
    for (Xa, la, ia), (Xb, lb, ib) in zip(r1, r2):
        assert ia["status"] == 0 and ia["iterations"] == ib["iterations"]
        assert torch.equal(Xa, Xb) and torch.equal(la, lb)


def cm_order_reference(g):
    """Cuthill-McKee order (pure Python, sequential): start at the lowest
    node on the last breadth-first level of a search from node 0; scan each
    level in order and each node's neighbours in increasing id, appending
    unvisited ones; further components from their lowest unvisited node."""
    n = g.n
    if n <= 48:
        return np.arange(n)
    nbr = [g.col[g.rowptr[i]:g.rowptr[i + 1]].tolist() for i in range(n)]
    level = [-1] * n
    level[0], front = 0, [0]
    while front:
        nxt = []
        for u in front:
            for v in nbr[u]:
                if level[v] < 0:
                    level[v] = level[u] + 1
                    nxt.append(v)
        front = nxt
    last = max(level)
    start = min(i for i in range(n) if level[i] == last)
    seen = [False] * n
    order = []

    def component(s):
        seen[s] = True
        order.append(s)
        front = [s]
        while front:
            nxt = []
            for u in front:
                for v in nbr[u]:
                    if not seen[v]:
                        seen[v] = True
                        nxt.append(v)
            order.extend(nxt)
            front = nxt

    component(start)
    for i in range(n):
        if not seen[i]:
            component(i)
    return np.array(order)


@pytest.mark.parametrize("name", ["square_2k", "sphere_3k", "two_squares", "grid_bipartite",
                                  "star_1500", "tri_mesh", "random_300", "random_4000"])
def test_solver_order_bit_exact(me, name):
    g, _ = oracle_ops(name)
    h = me.build_graph_ops(g)
    perm = _np(h.order())
    assert np.array_equal(np.sort(perm), np.arange(g.n))
    assert np.array_equal(perm, cm_order_reference(g))
    h.close()


def _large_order_graph(name):
    if name == "swiss_100k":
        return sg.manifold_graph("swiss_roll", 100_000, 10, 0)
    if name == "square_40k_plus_two":
        # three components: the per-level search orders the first, the
        # one-workgroup search continues with the others
        return sg.disjoint_union([sg.manifold_graph("square", 40_000, 8, 5),
                                  sg.manifold_graph("sphere", 3_000, 10, 6), sg.ring(50, 2)])
    if name == "expander_60k":
        # levels grow geometrically: a level of tens of thousands of nodes
        # spans many scan chunks
        return sg.sparse_random_graph(60_000, 6.0, 7)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["swiss_100k", "square_40k_plus_two", "expander_60k"])
def test_solver_order_bit_exact_large(me, name):
    """Graphs of 32768 nodes or more take the per-level multi-workgroup
    searches; the order is still that of the sequential algorithm."""
    g = _large_order_graph(name)
    print(f"[gpu] order {name} n={g.n}", flush=True)
    h = me.build_graph_ops(g)
    perm = _np(h.order())
    assert np.array_equal(np.sort(perm), np.arange(g.n))
    assert np.array_equal(perm, cm_order_reference(g))
    h.close()


@pytest.mark.parametrize("name,K", [("square_2k", 4), ("swiss_3k", 8), ("sphere_3k", 16),
                                    ("ring_203", 8), ("grid_bipartite", 4)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_global_addressing_identical(me, name, K, precision):
    """The 64-bit-address form of the product kernels (taken for arrays of
    2 GiB and more) visits the entries in the same order as the 32-bit buffer
    form: the same eps and the same pairs, bit for bit."""
    g, _ = oracle_ops(name)
    h1 = me.build_graph_ops(g, precision=precision)
    h2 = me.build_graph_ops(g, precision=precision, addressing="global")
    assert h1.eps == h2.eps
    X1, l1, i1 = me.embed(h1, K, tol=1e-8, seed=2, precision=precision)
    X2, l2, i2 = me.embed(h2, K, tol=1e-8, seed=2, precision=precision, addressing="global")
    assert i1["status"] in (0, 2) and i1["iterations"] == i2["iterations"], (i1, i2)
    assert torch.equal(X1, X2) and torch.equal(l1, l2)
    h1.close()
    h2.close()


def test_mixed_without_packed_entries(me):
    """An expander has no locality order that keeps every column within 2^15
    of its row, so the FP32 preconditioner reads the full entry arrays
    instead of the packed ones.  Sampled rows of A X - B X Lambda (the
    oracle's row-wise operator) meet the certified bound, X is B-orthonormal,
    and the eigenvalues agree with the FP64 solve."""
    n = 70000
    rng = np.random.default_rng(9)
    i = np.concatenate([np.arange(n), np.repeat(np.arange(n), 2)])
    j = np.concatenate([(np.arange(n) + 1) % n, rng.integers(0, n, 2 * n)])
    g = sg.from_edges(n, i, j, np.ones(i.size))
    h = me.build_graph_ops(g, precision="mixed")
    iperm = np.empty(n, dtype=np.int64)
    iperm[_np(h.order()).astype(np.int64)] = np.arange(n)
    rows_all = np.repeat(np.arange(n), np.diff(g.rowptr))
    assert np.abs(iperm[rows_all] - iperm[g.col]).max() > 32767
    tol = 1e-6
    X, lam, info = me.embed(h, 4, tol=tol, seed=0, precision="mixed")
    assert info["status"] == 0, info
    X, lam = _np(X), _np(lam)
    b = _np(h.export()["b"])
    G = X.T @ (b[:, None] * X)
    assert np.abs(G - np.eye(4)).max() <= 1e-10
    rows = np.sort(np.random.default_rng(3).choice(n, 200, replace=False)).tolist()
    AX = oracle.operator_a_rows(g.n, g.rowptr, g.col, g.val, rows, h.mu, h.eps, X)
    R = AX - b[rows, None] * X[rows] * lam[None, :]
    bound = tol * np.abs(lam) * np.linalg.norm(b[:, None] * X, axis=0)
    assert np.all(np.abs(R) <= bound[None, :] * 1.001), np.abs(R).max(axis=0) / bound
    X2, lam2, info2 = me.embed(h, 4, tol=1e-8, seed=0, precision="fp64")
    assert info2["status"] == 0, info2
    np.testing.assert_allclose(lam, _np(lam2), rtol=1e-6)
    # the 64-bit-address form of the unpacked FP32 step: the same pairs, bit for bit
    h3 = me.build_graph_ops(g, precision="mixed", addressing="global")
    assert h3.eps == h.eps
    X3, lam3, info3 = me.embed(h3, 4, tol=tol, seed=0, precision="mixed", addressing="global")
    assert info3["iterations"] == info["iterations"]
    assert np.array_equal(_np(X3), X) and np.array_equal(_np(lam3), lam)
    h3.close()
    h.close()


@pytest.mark.parametrize("name,K,precision", [("square_2k", 4, "fp64"), ("swiss_3k", 8, "mixed"),
                                              ("sphere_3k", 16, "mixed"), ("tri_mesh", 3, "mixed")])
def test_graph_launch_identical(me, name, K, precision):
    """Rounds replayed as a captured HIP graph run the same kernels with the
    same arguments: the same pairs bit for bit, in a single solve and in a
    batch (whose active sets change as graphs finish, so the graph is
    captured again)."""
    g, _ = oracle_ops(name)
    X1, l1, i1 = me.embed(g, K, tol=1e-8, seed=3, precision=precision, launch="stream")
    X2, l2, i2 = me.embed(g, K, tol=1e-8, seed=3, precision=precision, launch="graph")
    assert i1["status"] == i2["status"] and i1["iterations"] == i2["iterations"]
    assert torch.equal(X1, X2) and torch.equal(l1, l2)
    other = sg.manifold_graph("torus", 1500, 8, 21)
    a = me.embed_batch([g, other], [K, 8], tol=1e-8, seed=3, precision=precision,
                       launch="stream")
    b = me.embed_batch([g, other], [K, 8], tol=1e-8, seed=3, precision=precision, launch="graph")
    for (xa, la, ia), (xb, lb, ib) in zip(a, b):
        assert ia["iterations"] == ib["iterations"]
        assert torch.equal(xa, xb) and torch.equal(la, lb)


@pytest.mark.parametrize("name,K,precision", [("swiss_3k", 8, "mixed"), ("sphere_3k", 16, "fp64"),
                                              ("torus_2500", 8, "mixed")])
def test_cholqr2_matches_oracle(me, name, K, precision):
    """Two B-orthonormalisations of the preconditioned block per iteration
    (CholQR2): the same bar as one; the run differs from the one-pass run,
    so the second pass ran."""
    g, ops = oracle_ops(name)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-6, 1e-5 * relgap / 4)
    X, lam, info = me.embed(g, K, tol=tol, seed=1, precision=precision, cholqr_passes=2)
    assert info["status"] == 0, info
    X, lam = _np(X), _np(lam)
    np.testing.assert_array_less(np.abs(lam - lam_o[:K]) / np.abs(lam_o[:K]), 1e-6)
    assert oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"]) <= 1e-5
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    assert np.all(oracle.relative_residuals(ops["A"], ops["b"], X, lam) <= tol * 1.01 + 1e-12)
    X1, _, i1 = me.embed(g, K, tol=tol, seed=1, precision=precision)
    print(f"[gpu] {name} K={K} {precision}: iterations CholQR2 {info['iterations']} "
          f"CholQR {i1['iterations']}", flush=True)
    assert not np.array_equal(_np(X1), X)


@pytest.mark.parametrize("name,K", [("square_2k", 4), ("swiss_3k", 8), ("sphere_3k", 16),
                                    ("torus_2500", 8)])
def test_fp32_product_certified_or_rejected(me, name, K):
    """The FP32 product A W inside the iteration (W rounded to FP32; X, the
    Grams and the certificate FP64), an option kept for this measurement.  A
    result the FP64 certificate accepts meets the FP64 product's bars; one it
    rejects ends at max_iter with ME_WARN_NOT_CONVERGED and a certified
    residual above the target.  Measured: the 2000-node square converges
    (15 iterations against 14), the 3000-node Swiss roll does not (its
    implicitly updated A X drifts away from A X; certified residual of order
    1 after 2000 iterations, against 26 iterations with the FP64 product)."""
    g, ops = oracle_ops(name)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-6, 1e-5 * relgap / 4)
    X, lam, info = me.embed(g, K, tol=tol, seed=1, precision="mixed", product="fp32",
                            max_iter=300)
    X64, _, i64 = me.embed(g, K, tol=tol, seed=1, precision="mixed")
    print(f"[gpu] fp32 product {name} K={K}: status {info['status_name']} "
          f"rho {info['max_residual']:.3e} iterations {info['iterations']} "
          f"(FP64 product {i64['iterations']})", flush=True)
    assert not np.array_equal(_np(X64), _np(X))
    if name == "square_2k":
        assert info["status"] == 0, info
    if info["status"] != 0:
        assert info["status"] == 1 and info["max_residual"] > tol, info
        return
    X, lam = _np(X), _np(lam)
    np.testing.assert_array_less(np.abs(lam - lam_o[:K]) / np.abs(lam_o[:K]), 1e-6)
    assert oracle.sin_principal_angle_b(X, V_o[:, :K], ops["b"]) <= 1e-5
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    assert np.all(oracle.relative_residuals(ops["A"], ops["b"], X, lam) <= tol * 1.01 + 1e-12)


def test_option_errors(me):
    g = GRAPHS["tri_mesh"]()
    with pytest.raises(me.MembedError):
        me.embed(g, 3, precision="fp64", product="fp32")  # FP32 product needs ME_MIXED
    with pytest.raises(me.MembedError):
        me.embed(g, 3, cholqr_passes=3)


def test_embed_without_halos(me):
    """A wheel (a hub joined to 598 of 600 ring nodes, random weights): the
    hub's tile has some 600 distinct neighbours, more than the width-16 step
    stages in LDS, and every ring node has some 600 two-hop neighbours, more
    than the halo build sorts per tile, so both solves' preconditioners run
    the gathering kernels instead of the halo-staged ones.  Parity with the
    oracle at the usual bars, and bit for bit with the 64-bit-address form."""
    m = 600
    rng = np.random.default_rng(21)
    hub = 1 + np.arange(2, m)
    i = np.concatenate([np.zeros(hub.size, dtype=np.int64), 1 + np.arange(m)])
    j = np.concatenate([hub, 1 + (np.arange(m) + 1) % m])
    g = sg.from_edges(m + 1, i, j, rng.uniform(0.5, 2.0, i.size))
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    K = 16
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol = min(1e-6, 1e-5 * relgap / 4)
    print(f"[gpu] wheel n={g.n} nnz={g.nnz} relgap={relgap:.3g}", flush=True)
    X, lam, info = me.embed(g, K, tol=tol, seed=1, precision="mixed")
    assert info["status"] == 0, info
    Xn, lamn = _np(X), _np(lam)
    np.testing.assert_array_less(np.abs(lamn - lam_o[:K]) / np.abs(lam_o[:K]), 1e-6)
    assert oracle.sin_principal_angle_b(Xn, V_o[:, :K], ops["b"]) <= 1e-5
    X2, lam2, info2 = me.embed(g, K, tol=tol, seed=1, precision="mixed", addressing="global")
    assert torch.equal(X, X2) and torch.equal(lam, lam2)


def test_step_form_tuning_leaves_results_unchanged(me):
    """The run-time tuner times the halo-staged and the gathering forms of
    the preconditioner step in the first iteration of a kind of solve and
    keeps the faster: the first solve (mixed forms), the next (the kept
    form) and the 64-bit-address form agree bit for bit, and both kinds of
    the solve (the embedding's one-hop steps, the eps solve's two-hop
    steps) get a choice.  A 40 000-node square: above the size whose
    rounds replay as a HIP graph."""
    g = sg.manifold_graph("square", 40000, 8, 11)
    me.step_form_reset()
    assert me.step_form(8, 1, g.n) == -1
    h = me.build_graph_ops(g, precision="mixed")
    X1, l1, i1 = me.embed(h, 8, tol=1e-6, seed=0, precision="mixed")
    f_embed, f_eps = me.step_form(8, 1, g.n), me.step_form(4, 2, g.n)
    print(f"[gpu] step forms: embedding {f_embed}, eps {f_eps}", flush=True)
    assert f_embed in (0, 1) and f_eps in (0, 1)
    X2, l2, i2 = me.embed(h, 8, tol=1e-6, seed=0, precision="mixed")
    assert i1["status"] == 0 and i1["iterations"] == i2["iterations"]
    assert torch.equal(X1, X2) and torch.equal(l1, l2)
    h3 = me.build_graph_ops(g, precision="mixed", addressing="global")
    assert h3.eps == h.eps
    X3, l3, _ = me.embed(h3, 8, tol=1e-6, seed=0, precision="mixed", addressing="global")
    assert torch.equal(X1, X3) and torch.equal(l1, l3)
    h.close()
    h3.close()
