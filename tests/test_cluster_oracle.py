"""Pins of the clustering oracle (oracle/cluster.py): the four criteria by
hand and against scikit-learn's library routines, k-means++ seeding by hand,
Lloyd iterations against scikit-learn's k-means from the same seeds, EM
against scikit-learn's Gaussian mixture after the same number of steps, and
the Gaussian log-density against scipy.  CPU only."""
import math

import numpy as np
import pytest

from oracle import cluster as CL


def test_criteria_by_hand():
    """classes 0,0,0,1,1,1 vs clusters 0,0,1,1,1,1: table [[2,1],[0,3]];
    TP = 1 + 0 + 3 = 4, Ppred = 1 + 6 = 7, Ptrue = 3 + 3 = 6, Tot = 15:
    RI = 10/15, Precision = 4/7, Purity = 5/6; MI = ln2/6 + ln(3/2)/2,
    H(U) = ln 2, H(V) = ln 3 - (2/3) ln 2."""
    s = CL.criteria([0, 0, 0, 1, 1, 1], [0, 0, 1, 1, 1, 1])
    assert s["RI"] == pytest.approx(10 / 15, rel=1e-15)
    assert s["Precision"] == pytest.approx(4 / 7, rel=1e-15)
    assert s["Purity"] == pytest.approx(5 / 6, rel=1e-15)
    mi = math.log(2) / 6 + math.log(1.5) / 2
    hu, hv = math.log(2), math.log(3) - 2 / 3 * math.log(2)
    assert s["NMI"] == pytest.approx(mi / math.sqrt(hu * hv), rel=1e-14)


def test_criteria_of_a_perfect_and_a_trivial_clustering():
    y = np.repeat(np.arange(4), 25)
    perm = np.array([2, 0, 3, 1])[y]  # relabelled clusters
    s = CL.criteria(y, perm)
    assert s == {"RI": 1.0, "Precision": 1.0, "Purity": 1.0, "NMI": 1.0}
    t = CL.criteria(y, np.zeros_like(y))  # one cluster
    assert t["NMI"] == 0.0 and t["Purity"] == 0.25
    assert t["Precision"] == pytest.approx(4 * 300 / 4950)


def test_criteria_against_scikit_learn():
    from sklearn.metrics import normalized_mutual_info_score, rand_score
    from sklearn.metrics.cluster import contingency_matrix
    rng = np.random.default_rng(0)
    y = rng.integers(0, 6, 500)
    z = np.where(rng.random(500) < 0.7, y, rng.integers(0, 5, 500))
    s = CL.criteria(y, z)
    assert s["RI"] == pytest.approx(rand_score(y, z), rel=1e-13)
    assert s["NMI"] == pytest.approx(
        normalized_mutual_info_score(y, z, average_method="geometric"), rel=1e-12)
    t = contingency_matrix(y, z)
    assert np.array_equal(CL.contingency(y, z), t)
    assert s["Purity"] == pytest.approx(t.max(axis=0).sum() / 500, rel=1e-15)


def test_kmeanspp_seeding_by_hand():
    """Points 0, 1, 10, 11 on a line.  u0 = 0.3 picks floor(1.2) = point 1.
    D^2 = 1, 0, 81, 100; cumulative 1, 1, 82, 182: u1 = 0.5 (target 91)
    picks point 3; then D^2 = 1, 0, 1, 0, cumulative 1, 1, 2, 2: u2 = 0.6
    (target 1.2) picks point 2."""
    x = np.array([[0.0], [1.0], [10.0], [11.0]])
    assert CL.kmeanspp_seeds(x, 3, [0.3, 0.5, 0.6]).tolist() == [1, 3, 2]


def test_lloyd_matches_scikit_learn_from_the_same_seeds():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(1)
    centres = rng.standard_normal((5, 3)) * 4
    x = np.concatenate([c + rng.standard_normal((200, 3)) for c in centres])
    u = rng.random(5)
    labels, cen, it = CL.kmeans(x, 5, u)
    seeds = CL.kmeanspp_seeds(x, 5, u)
    km = KMeans(5, init=x[seeds], n_init=1, algorithm="lloyd", tol=0.0, max_iter=100).fit(x)
    assert np.array_equal(labels, km.labels_)
    np.testing.assert_allclose(cen, km.cluster_centers_, rtol=1e-12, atol=1e-12)


def test_log_density_against_scipy():
    from scipy.stats import multivariate_normal
    rng = np.random.default_rng(2)
    a = rng.standard_normal((4, 4))
    cov = a @ a.T + np.eye(4)
    mu = rng.standard_normal(4)
    x = rng.standard_normal((50, 4))
    np.testing.assert_allclose(CL._log_gauss(x, mu, cov),
                               multivariate_normal(mu, cov).logpdf(x), rtol=1e-12)


def test_em_matches_scikit_learn_step_for_step():
    """Five EM steps from the k-means partition equal scikit-learn's five
    steps from the same parameters (its reg_covar is the same diagonal
    term)."""
    from sklearn.mixture import GaussianMixture
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.multivariate_normal(m, c, 300) for m, c in [
        ([0, 0], [[1, 0.5], [0.5, 1]]), ([4, 1], [[0.5, 0], [0, 2]]),
        ([1, 5], [[1, -0.3], [-0.3, 0.6]])]])
    labels0, _, _ = CL.kmeans(x, 3, rng.random(3))
    lab, w, mu, cov, ll, it = CL.gmm(x, 3, labels0, max_iter=5, tol=0.0)
    assert it == 5
    reg = 1e-6 * float(np.mean(np.var(x, axis=0)))
    w0, mu0, cov0 = [], [], []
    for c in range(3):
        m = labels0 == c
        w0.append(m.mean())
        mu0.append(x[m].mean(axis=0))
        xc = x[m] - mu0[-1]
        cov0.append(xc.T @ xc / m.sum() + reg * np.eye(2))
    gm = GaussianMixture(3, covariance_type="full", reg_covar=reg, max_iter=5, tol=0.0,
                         weights_init=np.array(w0), means_init=np.array(mu0),
                         precisions_init=np.array([np.linalg.inv(c) for c in cov0]))
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gm.fit(x)
    np.testing.assert_allclose(w, gm.weights_, rtol=1e-10)
    np.testing.assert_allclose(mu, gm.means_, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(cov, gm.covariances_, rtol=1e-9, atol=1e-12)
    assert np.array_equal(lab, gm.predict(x))


def test_em_recovers_separated_blobs():
    """Far-apart blobs: EM converges to each blob's sample mean and
    covariance (plus the regularisation), with weights the blob fractions."""
    rng = np.random.default_rng(4)
    blobs = [rng.standard_normal((n, 2)) * s + m
             for n, s, m in [(400, 0.5, (0, 0)), (200, 1.0, (20, 0)), (100, 0.3, (0, 20))]]
    x = np.concatenate(blobs)
    truth = np.repeat(np.arange(3), [400, 200, 100])
    labels0, _, _ = CL.kmeans(x, 3, [0.1, 0.5, 0.9])
    lab, w, mu, cov, ll, it = CL.gmm(x, 3, labels0)
    assert CL.criteria(truth, lab)["NMI"] == 1.0
    reg = 1e-6 * float(np.mean(np.var(x, axis=0)))
    for b in blobs:
        c = int(np.argmin(np.linalg.norm(mu - b.mean(axis=0), axis=1)))
        np.testing.assert_allclose(mu[c], b.mean(axis=0), rtol=1e-8, atol=1e-9)
        bc = b - b.mean(axis=0)
        np.testing.assert_allclose(cov[c], bc.T @ bc / len(b) + reg * np.eye(2), rtol=1e-7)
        assert w[c] == pytest.approx(len(b) / len(x), rel=1e-8)
