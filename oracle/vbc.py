"""Betweenness centrality and its variance, the manifold-graph check of
Section 3.3 (eq. (3), Table 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.3 defines C_B(i) = sum over s, t != i of sigma_st(i) / sigma_st,
sigma_st the number of shortest paths from s to t and sigma_st(i) the
number of those through i, and uses the variance of C_B over the nodes
(VBC) to accept a graph as a manifold graph.  Readings:

V1  Shortest paths count edges (hop distance); edge weights do not enter.
V2  The sum runs over ordered pairs (s, t) with s != t, s != i, t != i;
    pairs in different components have no shortest path and add nothing.
V3  VBC = (1/N) sum_i (C_B(i) - mean C_B)^2 (the population variance).

``betweenness_definition`` evaluates eq. (3) literally from all-pairs hop
distances and path counts (sigma_st(i) = sigma_si sigma_it when
d(s, i) + d(i, t) = d(s, t)); ``betweenness`` is Brandes' accumulation
(U. Brandes, "A faster algorithm for betweenness centrality", 2001), level
by level for all sources at once.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _adjacency(n, rowptr, col):
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    return sp.csr_matrix((np.ones(col.size), col, rowptr), shape=(n, n))


def hop_counts(n, rowptr, col):
    """All-pairs hop distances D (inf if unreachable) and shortest-path
    counts S (S[s, s] = 1), by breadth-first levels from every source."""
    A = _adjacency(n, rowptr, col)
    D = np.full((n, n), np.inf)
    S = np.zeros((n, n))
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(S, 1.0)
    frontier = np.eye(n)  # frontier[s, v] = paths from s to v on the current level
    lev = 0
    while frontier.any():
        nxt = np.asarray((sp.csr_matrix(frontier) @ A).todense())
        new = (nxt > 0) & np.isinf(D)
        lev += 1
        D[new] = lev
        S[new] = nxt[new]
        frontier = np.where(new, nxt, 0.0)
    return D, S


def betweenness_definition(n, rowptr, col):
    """Eq. (3) evaluated term by term (small graphs)."""
    D, S = hop_counts(n, rowptr, col)
    cb = np.zeros(n)
    for i in range(n):
        through = (D[:, i][:, None] + D[i, :][None, :] == D) & np.isfinite(D)
        through[i, :] = False
        through[:, i] = False
        np.fill_diagonal(through, False)
        ratio = np.where(through, (S[:, i][:, None] * S[i, :][None, :]) / np.where(S > 0, S, 1),
                         0.0)
        cb[i] = ratio.sum()
    return cb


def betweenness(n, rowptr, col):
    """Brandes' accumulation for every source at once: delta_s(v) =
    sum over w one level below v with (v, w) an edge of
    sigma_sv / sigma_sw (1 + delta_s(w)), and C_B(v) = sum_s delta_s(v)
    (v != s).  Dense n x n state (moderate n)."""
    A = _adjacency(n, rowptr, col)
    D, S = hop_counts(n, rowptr, col)
    finite = np.isfinite(D)
    maxd = int(D[finite].max()) if finite.any() else 0
    delta = np.zeros((n, n))
    for lev in range(maxd - 1, -1, -1):
        below = (D == lev + 1)
        coef = np.where(below, (1.0 + delta) / np.where(S > 0, S, 1.0), 0.0)
        acc = np.asarray((sp.csr_matrix(coef) @ A).todense())  # sum over neighbours w of v
        at = (D == lev)
        delta = np.where(at, S * acc, delta)
    np.fill_diagonal(delta, 0.0)
    return delta.sum(axis=0)


def vbc(cb):
    """V3: population variance of the centralities."""
    cb = np.asarray(cb, dtype=np.float64)
    return float(np.mean((cb - cb.mean()) ** 2))
