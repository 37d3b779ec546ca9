"""Pins of the kNN-graph oracle (oracle/knn.py) against values worked by hand,
brute force in plain Python, the k-d tree of scipy, and the host input
generator.  CPU only."""
import math

import numpy as np
import pytest

from oracle import knn as KN
import synthgraphs as sg


def _rows(rowptr, col):
    return [list(col[rowptr[i]:rowptr[i + 1]]) for i in range(len(rowptr) - 1)]


def test_line_by_hand():
    """Five points 0..4 on a line, k = 2.  Node 1 has neighbours 0 and 2 at
    the same distance (both kept); node 2 has 1 and 3; node 0 takes 1 and 2;
    node 4 takes 3 and 2.  k-th distances 2, 1, 1, 1, 2: sigma = 1.  Union
    edges 0-1, 0-2, 1-2, 2-3, 2-4, 3-4 with w = exp(-d^2)."""
    x = np.arange(5.0)[:, None]
    idx, d2 = KN.knn_brute(x, 2)
    assert idx.tolist() == [[1, 2], [0, 2], [1, 3], [2, 4], [3, 2]]
    assert d2.tolist() == [[1, 4], [1, 1], [1, 1], [1, 1], [1, 4]]
    rp, col, val, sigma = KN.knn_graph(x, 2)
    assert sigma == 1.0
    assert _rows(rp, col) == [[1, 2], [0, 2], [0, 1, 3, 4], [2, 4], [2, 3]]
    e1, e4 = math.exp(-1.0), math.exp(-4.0)
    assert val.tolist() == [e1, e4, e1, e1, e4, e1, e1, e4, e1, e1, e4, e1]


def test_ties_go_to_the_smaller_index():
    """k = 1 on the line: node 2 is equally far from 1 and 3 and takes 1;
    node 1 is equally far from 0 and 2 and takes 0."""
    idx, _ = KN.knn_brute(np.arange(5.0)[:, None], 1)
    assert idx[:, 0].tolist() == [1, 0, 1, 2, 3]


def test_two_points_by_hand():
    """(0, 0) and (3, 4): d^2 = 25, sigma = 5, w = exp(-25 / 25) = 1/e."""
    rp, col, val, sigma = KN.knn_graph(np.array([[0.0, 0.0], [3.0, 4.0]]), 1)
    assert sigma == 5.0 and rp.tolist() == [0, 1, 2] and col.tolist() == [1, 0]
    assert val.tolist() == [math.exp(-1.0)] * 2


def test_even_count_median_is_the_mean_of_the_middle_pair():
    """Points 0, 1, 3, 7 with k = 1: k-th distances 1, 1, 2, 4, median
    (1 + 2) / 2 = 1.5."""
    _, _, _, sigma = KN.knn_graph(np.array([[0.0], [1.0], [3.0], [7.0]]), 1)
    assert sigma == 1.5


def test_underflowing_weight_is_clamped():
    """A far point's only edge has d^2 / sigma^2 near 1e10: exp underflows
    and the weight is the smallest normal number."""
    x = np.array([[0.0], [0.001], [0.002], [100.0]])
    rp, col, val, sigma = KN.knn_graph(x, 1)
    assert sigma == pytest.approx(0.001, rel=1e-12)
    far = dict(zip(_rows(rp, col)[3], val[rp[3]:rp[4]]))
    assert far == {2: KN.TINY}


def test_duplicate_points_and_zero_sigma():
    """Duplicated points are at distance 0 and tie with each other (smaller
    index first); if every k-th distance is 0 the weights are undefined."""
    x = np.array([[0.0], [0.0], [1.0], [1.0], [5.0]])
    idx, d2 = KN.knn_brute(x, 1)
    assert idx[:, 0].tolist() == [1, 0, 3, 2, 2]  # node 4: 2 and 3 tie at 16
    assert d2[:, 0].tolist() == [0, 0, 0, 0, 16]
    with pytest.raises(KN.KnnInputError):
        KN.knn_graph(x, 1)  # median of 0, 0, 0, 0, 4 is 0


def test_input_errors():
    with pytest.raises(KN.KnnInputError):
        KN.knn_graph(np.zeros((4, 2)) + np.arange(4)[:, None], 4)  # k = n
    with pytest.raises(KN.KnnInputError):
        KN.knn_graph(np.array([[0.0], [np.nan], [1.0]]), 1)


def _plain_python_knn(x, k):
    n, dim = x.shape
    out_i, out_d = [], []
    for i in range(n):
        cand = []
        for j in range(n):
            if j == i:
                continue
            s = 0.0
            for d in range(dim):
                t = float(x[i, d]) - float(x[j, d])
                s = s + t * t
            cand.append((s, j))
        cand.sort()
        out_i.append([j for _, j in cand[:k]])
        out_d.append([s for s, _ in cand[:k]])
    return out_i, out_d


@pytest.mark.parametrize("dim,k", [(1, 3), (3, 5), (7, 4)])
def test_brute_force_matches_plain_python(dim, k):
    x = np.random.default_rng(dim).standard_normal((37, dim))
    # a few exact ties: duplicated points
    x[5] = x[9]
    x[20] = x[9]
    idx, d2 = KN.knn_brute(x, k, block=8)
    pi, pd = _plain_python_knn(x, k)
    assert idx.tolist() == pi
    assert d2.tolist() == pd


def test_tree_route_matches_brute_force():
    x = sg.sample_points("sphere", 3000, np.random.default_rng(3))
    ib, db = KN.knn_brute(x, 12)
    it, dt = KN.knn_tree(x, 12)
    assert np.array_equal(ib, it) and np.array_equal(db, dt)


def test_distances_agree_with_the_kd_tree():
    from scipy.spatial import cKDTree
    x = sg.sample_points("swiss_roll", 2000, np.random.default_rng(4))
    idx, d2 = KN.knn_brute(x, 10)
    dist, cidx = cKDTree(x).query(x, k=11)
    np.testing.assert_allclose(np.sqrt(d2), dist[:, 1:], rtol=1e-13)
    assert np.array_equal(idx, cidx[:, 1:])


@pytest.mark.parametrize("kind,n,k", [("square", 2000, 8), ("sphere", 3000, 12),
                                      ("torus", 1500, 8)])
def test_graph_equals_the_input_generator(kind, n, k):
    """The generator (k-d tree, then the same union and weights) builds the
    same graph: identical pattern, weights equal to rounding."""
    rng = np.random.default_rng(11)
    x = sg.sample_points(kind, n, rng)
    g = sg.knn_graph(x, k)
    rp, col, val, sigma = KN.knn_graph(x, k)
    assert np.array_equal(rp, g.rowptr) and np.array_equal(col, g.col)
    np.testing.assert_allclose(val, g.val, rtol=1e-13)
