"""GPU clustering of an embedding (me_kmeans, me_gmm) and its criteria
(me_cluster_scores) against the CPU oracle (oracle/cluster.py) through the C
ABI.

Bars: k-means seeds and labels bit-exact; centres to relative 1e-12 (the
means are summed in another order); GMM labels bit-exact, weights, means and
covariances to 1e-9 and the log-likelihood to 1e-12 relative after the same
number of EM steps; the contingency-table criteria to 1e-12.  Labels decided
by floating point are compared exactly only where the oracle's decision has
a margin far above rounding (checked in the test).  Inputs: Gaussian blobs
in 2 to 16 dimensions, and the embedding of a labelled manifold graph (C
separated squares joined into one kNN graph) computed on the GPU."""
import numpy as np
import pytest
import torch

from oracle import cluster as CL
import synthgraphs as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def me():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2112_07862_amd as pkg
    pkg.load()
    return pkg


def _np(t):
    return t.detach().cpu().numpy()


def _blobs(seed, C, K, n_per, spread=6.0):
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((C, K)) * spread
    x = np.concatenate([c + rng.standard_normal((n_per + 7 * q, K)) for q, c in enumerate(centres)])
    y = np.concatenate([np.full(n_per + 7 * q, q) for q in range(C)])
    return x, y


def _margin(x, centres, labels):
    d = CL.sq_dists(x, centres)
    srt = np.sort(d, axis=1)
    return np.min((srt[:, 1] - srt[:, 0]) / np.maximum(srt[:, 1], 1e-300))


@pytest.mark.parametrize("C,K,n_per", [(3, 2, 400), (8, 4, 300), (12, 16, 150), (40, 3, 60)])
def test_kmeans_matches_oracle(me, C, K, n_per):
    x, y = _blobs(C * 10 + K, C, K, n_per)
    u = np.random.default_rng(C + K).random(C)
    print(f"[gpu] kmeans C={C} K={K} n={len(x)}", flush=True)
    lab_o, cen_o, it_o = CL.kmeans(x, C, u)
    assert _margin(x, cen_o, lab_o) > 1e-9  # every decision far from a tie
    X = torch.as_tensor(x, device="cuda")
    lab, cen, it = me.kmeans(X, C, u)
    assert it == it_o
    assert np.array_equal(_np(lab), lab_o)
    np.testing.assert_allclose(_np(cen), cen_o, rtol=1e-12, atol=1e-12)


def test_kmeans_seeds_match(me):
    """One update: the centres are the means of the partition the k-means++
    seeds induce, so the seeds, the first assignment and the update all
    match the oracle's."""
    x, _ = _blobs(5, 6, 3, 200)
    u = np.random.default_rng(9).random(6)
    seeds = CL.kmeanspp_seeds(x, 6, u)
    X = torch.as_tensor(x, device="cuda")
    lab, cen, it = me.kmeans(X, 6, u, max_iter=1)
    lab0 = CL.assign(x, x[seeds])
    cen1 = CL.update(x, lab0, x[seeds])
    np.testing.assert_allclose(_np(cen), cen1, rtol=1e-12, atol=1e-12)


def test_kmeans_degenerate_cases(me):
    """One cluster (its centre is the mean), as many clusters as points (each
    point its own centre, in k-means++ order) and identical points (every
    D^2 weight is zero, and both sides then take the last point; ties of
    the assignment go to the lower centre index on both sides)."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal((257, 3))
    cases = [(x, 1, [0.3]), (x[:6], 6, list(rng.random(6))),
             (np.ones((50, 2)), 3, [0.2, 0.5, 0.7])]
    for xx, C, u in cases:
        lab_o, cen_o, it_o = CL.kmeans(xx, C, u)
        lab, cen, it = me.kmeans(torch.as_tensor(xx, device="cuda"), C, u)
        assert it == it_o
        assert np.array_equal(_np(lab), lab_o)
        np.testing.assert_allclose(_np(cen), cen_o, rtol=1e-12, atol=1e-12)


def test_gmm_one_component(me):
    """C = 1: the weight is 1, the mean is the sample mean and the covariance
    the sample's maximum-likelihood covariance plus the ridge both sides add
    (1e-6 times the mean variance of the coordinates)."""
    x, _ = _blobs(31, 1, 3, 400)
    lab0 = np.zeros(len(x), dtype=np.int64)
    lab_o, w_o, mu_o, cov_o, ll_o, it_o = CL.gmm(x, 1, lab0)
    lab, w, mu, cov, ll, it = me.gmm(torch.as_tensor(x, device="cuda"), 1,
                                     torch.as_tensor(lab0, device="cuda"))
    assert it == it_o
    assert ll == pytest.approx(ll_o, rel=1e-12)
    assert np.array_equal(_np(lab), lab_o)
    np.testing.assert_allclose(_np(w), [1.0], rtol=1e-15)
    np.testing.assert_allclose(_np(mu), mu_o, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(_np(cov), cov_o, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(mu_o[0], x.mean(axis=0), rtol=1e-12)
    ridge = 1e-6 * np.mean(np.var(x, axis=0))
    np.testing.assert_allclose(cov_o[0], np.cov(x.T, bias=True) + ridge * np.eye(3),
                               rtol=1e-10, atol=1e-15)


@pytest.mark.parametrize("C,K,n_per,steps", [(3, 2, 400, 100), (5, 4, 250, 100), (4, 8, 200, 7)])
def test_gmm_matches_oracle(me, C, K, n_per, steps):
    x, y = _blobs(100 + C, C, K, n_per, spread=4.0)
    u = np.random.default_rng(C).random(C)
    lab0, _, _ = CL.kmeans(x, C, u)
    print(f"[gpu] gmm C={C} K={K} n={len(x)} steps<={steps}", flush=True)
    lab_o, w_o, mu_o, cov_o, ll_o, it_o = CL.gmm(x, C, lab0, max_iter=steps)
    X = torch.as_tensor(x, device="cuda")
    lab, w, mu, cov, ll, it = me.gmm(X, C, torch.as_tensor(lab0, device="cuda"), max_iter=steps)
    assert it == it_o
    assert ll == pytest.approx(ll_o, rel=1e-12)
    np.testing.assert_allclose(_np(w), w_o, rtol=1e-9)
    np.testing.assert_allclose(_np(mu), mu_o, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(_np(cov), cov_o, rtol=1e-9, atol=1e-12)
    assert np.array_equal(_np(lab), lab_o)


@pytest.mark.parametrize("seed", [0, 1])
def test_scores_match_oracle(me, seed):
    rng = np.random.default_rng(seed)
    y = rng.integers(0, 7, 5000)
    z = np.where(rng.random(5000) < 0.8, y, rng.integers(0, 9, 5000))
    s = me.cluster_scores(torch.as_tensor(y, device="cuda"), torch.as_tensor(z, device="cuda"),
                          7, 9)
    o = CL.criteria(y, z)
    for k in ("RI", "Precision", "Purity", "NMI"):
        assert s[k] == pytest.approx(o[k], rel=1e-12), k


def test_embedding_clustering_end_to_end(me):
    """Three unit squares side by side (one connected 10-NN graph): embed
    with K = 3 on the GPU, cluster, score against the squares."""
    rng = np.random.default_rng(3)
    parts = [rng.random((700, 2)) + np.array([1.0 * q, 0.0]) for q in range(3)]
    x = np.concatenate(parts)
    y = np.repeat(np.arange(3), 700)
    g = sg.knn_graph(x, 10)
    X, lam, info = me.embed(g, 3, tol=1e-8, seed=0)
    assert info["status"] in (0, 2)
    u = [0.2, 0.5, 0.8]
    lab, cen, it = me.kmeans(X, 3, u)
    lab_o, cen_o, it_o = CL.kmeans(_np(X), 3, u)
    labg, *_ = me.gmm(X, 3, lab)
    s_k = me.cluster_scores(torch.as_tensor(y, device="cuda"), lab, 3, 3)
    s_g = me.cluster_scores(torch.as_tensor(y, device="cuda"), labg, 3, 3)
    if _margin(_np(X), cen_o, lab_o) > 1e-9:  # every decision far from a tie
        assert np.array_equal(_np(lab), lab_o)
        o = CL.criteria(y, lab_o)
        assert s_k["NMI"] == pytest.approx(o["NMI"], rel=1e-12)
    print(f"[gpu] squares: kmeans {s_k} gmm {s_g}", flush=True)
    assert s_k["Purity"] > 0.8


def test_errors(me):
    X = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(me.MembedError):
        me.kmeans(X, 11, [0.1] * 11)  # C > n
    with pytest.raises(me.MembedError):
        me.kmeans(X, 2, [0.1, 1.0])  # u outside [0, 1)
    with pytest.raises(me.MembedError):
        me.cluster_scores(torch.zeros(10, dtype=torch.int32, device="cuda"),
                          torch.full((10,), 5, dtype=torch.int32, device="cuda"), 1, 3)
