"""GPU kNN graph construction (me_knn_graph) against the CPU oracle
(oracle/knn.py) through the C ABI.

Bars: the row pointers and column indices (the neighbour sets after the
union) are bit-exact; sigma is bit-exact (the same order statistic, a
correctly rounded square root and the same mean); weights agree to FP64
rounding: the argument -d^2 / sigma^2 is the same on both sides and only
the exp implementations differ (numpy's and the device library's were
measured up to 8 units in the last place apart on these graphs), so at most
16 ulps (3.6e-15 relative).  Sizes span several 256-point tiles with a ragged tail,
dimensions 1, 2, 3 (compiled instances) and 7 (the run-time form), and
exact ties (duplicated points, an integer grid)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import knn as KN
import synthgraphs as sg

pytestmark = pytest.mark.gpu

MAXULP = 16


@pytest.fixture(scope="module")
def me():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2112_07862_amd as pkg
    pkg.load()
    return pkg


def _np(t):
    return t.detach().cpu().numpy()


def _compare(me, x, k, **kw):
    pts = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    csr, sigma = me.knn_graph(pts, k, **kw)
    rp, col, val, sig_o = KN.knn_graph(x, k)
    assert np.array_equal(_np(csr.rowptr), rp)
    assert np.array_equal(_np(csr.col), col)
    assert sigma == sig_o, (sigma, sig_o)
    np.testing.assert_array_max_ulp(_np(csr.val), val, maxulp=MAXULP)
    return csr


def _grid_points(nx, ny):
    a, b = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                       indexing="ij")
    return np.stack([a.ravel(), b.ravel()], axis=1)


CASES = {
    "square_2000_k8": (lambda: sg.sample_points("square", 2000, np.random.default_rng(1)), 8),
    "sphere_3001_k12": (lambda: sg.sample_points("sphere", 3001, np.random.default_rng(2)), 12),
    "swiss_1537_k10": (lambda: sg.sample_points("swiss_roll", 1537, np.random.default_rng(3)), 10),
    "torus_700_k16": (lambda: sg.sample_points("torus", 700, np.random.default_rng(4)), 16),
    "gauss7d_1000_k5": (lambda: np.random.default_rng(5).standard_normal((1000, 7)), 5),
    "line_300_k3": (lambda: np.random.default_rng(6).random((300, 1)), 3),
    "grid_40x50_k4": (lambda: _grid_points(40, 50), 4),    # ties at 1, sqrt 2, 2
    "grid_17x13_k9": (lambda: _grid_points(17, 13), 9),
    "dups_900_k6": (lambda: np.repeat(np.random.default_rng(7).random((300, 3)), 3, axis=0), 6),
    "k32_600": (lambda: sg.sample_points("sphere", 600, np.random.default_rng(8)), 32),
    "complete_20": (lambda: np.random.default_rng(9).random((20, 3)), 19),
    "pair": (lambda: np.array([[0.0, 0.0], [3.0, 4.0]]), 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_knn_matches_oracle(me, name):
    make, k = CASES[name]
    x = make()
    print(f"[gpu] knn {name} n={len(x)} dim={x.shape[1]} k={k}", flush=True)
    _compare(me, x, k)


def test_knn_swiss_roll_100k(me):
    """The 100k-point Swiss roll of the 10-NN workload: the oracle takes the
    k-d tree route (pinned equal to brute force)."""
    x = sg.sample_points("swiss_roll", 100_000, np.random.default_rng(0))
    print("[gpu] knn swiss roll 100k", flush=True)
    csr = _compare(me, x, 10)
    # the same graph as the input generator's, which the embedding tests use
    g = sg.knn_graph(x, 10)
    assert np.array_equal(_np(csr.rowptr), g.rowptr) and np.array_equal(_np(csr.col), g.col)
    np.testing.assert_allclose(_np(csr.val), g.val, rtol=1e-13)


def test_knn_graph_feeds_the_embedding(me):
    """Points -> kNN graph -> embedding, all on the GPU, against the oracle's
    embedding of the oracle's graph (eigenvalues relative 1e-6)."""
    x = sg.sample_points("square", 2000, np.random.default_rng(0))
    pts = torch.as_tensor(x, device="cuda")
    csr, _ = me.knn_graph(pts, 8)
    X, lam, info = me.embed(csr, 4, tol=1e-8, seed=0)
    assert info["status"] == 0
    rp, col, val, _ = KN.knn_graph(x, 8)
    lam_o = oracle.embed(len(x), rp, col, val, 4)[1]
    assert np.max(np.abs(_np(lam) - lam_o) / lam_o) <= 1e-6


def test_knn_workspace_and_errors(me):
    x = sg.sample_points("sphere", 1000, np.random.default_rng(3))
    pts = torch.as_tensor(x, device="cuda")
    need = me.knn_workspace_bytes(1000, 3, 10)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    a, sa = me.knn_graph(pts, 10, workspace=ws)
    b, sb = me.knn_graph(pts, 10)
    assert sa == sb and torch.equal(a.rowptr, b.rowptr) and torch.equal(a.col, b.col)
    assert torch.equal(a.val, b.val)
    with pytest.raises(me.MembedError) as e:
        me.knn_graph(pts, 10, workspace=ws[:need - 1])
    assert e.value.name == "ME_ERR_WORKSPACE"
    with pytest.raises(me.MembedError) as e:
        me.knn_graph(pts, 1000)
    assert e.value.name == "ME_ERR_K_RANGE"
    with pytest.raises(me.MembedError) as e:
        me.knn_graph(pts, 33)
    assert e.value.name == "ME_ERR_K_RANGE"
    bad = pts.clone()
    bad[17, 1] = float("nan")
    with pytest.raises(me.MembedError) as e:
        me.knn_graph(bad, 5)
    assert e.value.name == "ME_ERR_INVALID_ARG"
    dup = torch.as_tensor(np.array([[0.0], [0.0], [1.0], [1.0], [5.0]]), device="cuda")
    with pytest.raises(me.MembedError) as e:
        me.knn_graph(dup, 1)  # sigma = 0
    assert e.value.name == "ME_ERR_BAD_WEIGHT"
    huge = torch.as_tensor(np.array([[0.0], [1e200], [-1e200]]), device="cuda")
    with pytest.raises(me.MembedError) as e:
        me.knn_graph(huge, 2)  # (2e200)^2 overflows
    assert e.value.name == "ME_ERR_INVALID_ARG"
