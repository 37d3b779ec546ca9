"""k-nearest-neighbour graphs of points, built as Section 5.1 describes them.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5.1 builds the kNN graphs of its face datasets from Euclidean
distances and gives no further detail.  The workloads here add the weighting recipe of
their configurations.  Readings:

K1  Distance: the squared Euclidean distance computed in FP64 as
    sum_{d = 0..D-1} (x_id - x_jd)^2, the terms added in coordinate order,
    each difference squared by a plain product (no fused multiply-add).  The
    same arithmetic gives d2(i, j) = d2(j, i) bit for bit.
K2  Neighbours: N_k(i) = the k points j != i of smallest d2(i, j); equal
    distances are ordered by the smaller index j.
K3  Symmetrisation: the union, (i, j) is an edge when j in N_k(i) or
    i in N_k(j).
K4  Scale: sigma = the median over the nodes of sqrt(d2(i, k-th neighbour))
    (for an even number of nodes, the mean of the two middle values).
K5  Weights: w_ij = exp(-d2(i, j) / sigma^2), with sigma^2 = sigma * sigma,
    raised to the smallest normal FP64 number if exp underflows (so that no
    edge gets a zero weight, which Section 3.1 excludes).  sigma = 0 leaves
    the weights undefined and is an input error.
"""
from __future__ import annotations

import numpy as np

TINY = np.finfo(np.float64).tiny


class KnnInputError(ValueError):
    pass


def _check(points, k):
    x = np.ascontiguousarray(points, dtype=np.float64)
    if x.ndim != 2 or x.shape[0] < 2 or x.shape[1] < 1:
        raise KnnInputError("points must be n x D with n >= 2, D >= 1")
    if not (1 <= k < x.shape[0]):
        raise KnnInputError("need 1 <= k < n")
    if not np.all(np.isfinite(x)):
        raise KnnInputError("non-finite coordinate")
    return x


def sq_dist(x, i, j):
    """K1 for index arrays i, j (broadcast): the terms in coordinate order."""
    acc = np.zeros(np.broadcast(np.asarray(i), np.asarray(j)).shape, dtype=np.float64)
    for d in range(x.shape[1]):
        t = x[i, d] - x[j, d]
        acc = acc + t * t
    return acc


def knn_brute(points, k, block: int = 512):
    """K1-K2 by brute force over all pairs: (idx, d2), each n x k, a row in
    increasing (d2, j) order."""
    x = _check(points, k)
    n = x.shape[0]
    idx = np.empty((n, k), dtype=np.int64)
    dd = np.empty((n, k), dtype=np.float64)
    allj = np.arange(n)
    for s in range(0, n, block):
        rows = np.arange(s, min(n, s + block))
        d2 = sq_dist(x, rows[:, None], allj[None, :])
        d2[np.arange(rows.size), rows] = np.inf  # j != i
        # order by (d2, j): lexsort's last key is the primary one
        part = np.argpartition(d2, k - 1, axis=1)[:, :k]
        kth = np.take_along_axis(d2, part, axis=1).max(axis=1)
        for r in range(rows.size):
            cand = np.nonzero(d2[r] <= kth[r])[0]  # every j tied at the k-th distance too
            order = np.lexsort((cand, d2[r, cand]))[:k]
            idx[s + r] = cand[order]
            dd[s + r] = d2[r, cand[order]]
    return idx, dd


def knn_tree(points, k, margin: int = 8):
    """K1-K2 for large n: a k-d tree (scipy cKDTree, a library search) only
    proposes k + margin candidates per point; they are re-ranked with the
    distance of K1 and the tie rule of K2.  Equal to knn_brute whenever the
    true k nearest are among the candidates (pinned against it)."""
    from scipy.spatial import cKDTree
    x = _check(points, k)
    n = x.shape[0]
    m = min(n, k + 1 + margin)
    _, cand = cKDTree(x).query(x, k=m)
    rows = np.repeat(np.arange(n), m).reshape(n, m)
    d2 = sq_dist(x, rows, cand)
    d2[cand == rows] = np.inf
    order = np.lexsort((cand, d2), axis=1)[:, :k]
    idx = np.take_along_axis(cand, order, axis=1).astype(np.int64)
    dd = np.take_along_axis(d2, order, axis=1)
    return idx, dd


def knn_lists(points, k, brute_max: int = 20_000):
    return knn_brute(points, k) if len(points) <= brute_max else knn_tree(points, k)


def kth_sigma(kth_d2):
    """K4: median of the k-th neighbour distances."""
    return float(np.median(np.sqrt(np.asarray(kth_d2, dtype=np.float64))))


def union_pattern(n, idx):
    """K3: sorted unique undirected pairs (lo, hi), lo < hi."""
    rows = np.repeat(np.arange(n, dtype=np.int64), idx.shape[1])
    cols = idx.reshape(-1).astype(np.int64)
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    key = np.unique(lo * n + hi)
    return key // n, key % n


def knn_graph(points, k, brute_max: int = 20_000):
    """The symmetric weighted kNN graph (K1-K5): (rowptr int64[n+1],
    col int32[nnz] sorted in each row, val float64[nnz], sigma)."""
    x = _check(points, k)
    n = x.shape[0]
    idx, dd = knn_lists(x, k, brute_max)
    sigma = kth_sigma(dd[:, k - 1])
    if not sigma > 0.0:
        raise KnnInputError("sigma = 0: the k-th neighbour distance has median 0")
    lo, hi = union_pattern(n, idx)
    d2 = sq_dist(x, lo, hi)
    w = np.maximum(np.exp(-d2 / (sigma * sigma)), TINY)
    r = np.concatenate([lo, hi])
    c = np.concatenate([hi, lo])
    v = np.concatenate([w, w])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, c.astype(np.int32), v, sigma
