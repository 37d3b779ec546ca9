"""Seeded synthetic graph generators (inputs only).

This module is shared by the oracle, the tests and the benchmark.  It holds
no arithmetic of the embedding method itself: it only samples points on a
manifold, builds symmetric k-nearest-neighbour graphs with Gaussian edge
weights, and writes a few small named graphs (rings, lines, meshes) as CSR.

The manifold-graph inputs follow the paper's setting of graphs interpreted as
uniform samples of a continuous manifold (Section 3.3) and its kNN graphs
built from Euclidean distances (Section 5.1).  The paper's own datasets are not
available; these samplers stand in for them.

CSR convention used everywhere: ``rowptr`` int64[N+1], ``col`` int32[nnz]
(strictly increasing inside a row), ``val`` float64[nnz], symmetric, no
self loops, all weights > 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "from_edges", "sample_points", "knn_graph", "manifold_graph",
    "ring", "line", "complete", "star", "tri_mesh", "grid", "complete_bipartite",
    "random_graph", "disjoint_union", "initial_block", "batch_specs",
    "serve_arrivals", "CONFIGS", "periodic_lattice", "lattice_stencil", "sparse_random_graph",
]


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64[n+1]
    col: np.ndarray     # int32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def degrees_count(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def from_edges(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray) -> CSR:
    """Symmetric CSR from an undirected edge list (each pair listed once or
    twice; duplicates must carry the same weight).  Self loops are dropped."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    keep = i != j
    i, j, w = i[keep], j[keep], w[keep]
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    key = lo * n + hi
    order = np.argsort(key, kind="stable")
    key, w = key[order], w[order]
    uniq, first = np.unique(key, return_index=True)
    w = w[first]
    lo = uniq // n
    hi = uniq % n
    r = np.concatenate([lo, hi])
    c = np.concatenate([hi, lo])
    v = np.concatenate([w, w])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int64)
    return CSR(n, rowptr, c.astype(np.int32), v.astype(np.float64))


# ----------------------------------------------------------------------------
# Manifold samplers
# ----------------------------------------------------------------------------

def sample_points(kind: str, n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform samples of a manifold.

    square      : [0,1]^2
    swiss_roll  : t ~ U[1.5pi, 4.5pi], h ~ U[0, 20], (t cos t, h, t sin t)
                  (uniform in the (t, h) chart, not area-uniform)
    sphere      : unit 2-sphere in R^3 (normalised Gaussians) plus isotropic
                  Gaussian noise of standard deviation 1e-3
    torus       : R = 2, r = 0.5, area-uniform (rejection on the minor angle
                  with acceptance (R + r cos v) / (R + r))
    """
    if kind == "square":
        return rng.random((n, 2))
    if kind == "swiss_roll":
        t = rng.uniform(1.5 * math.pi, 4.5 * math.pi, n)
        h = rng.uniform(0.0, 20.0, n)
        return np.stack([t * np.cos(t), h, t * np.sin(t)], axis=1)
    if kind == "sphere":
        g = rng.standard_normal((n, 3))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        return g + 1e-3 * rng.standard_normal((n, 3))
    if kind == "torus":
        R, r = 2.0, 0.5
        vs = np.empty(0)
        while vs.size < n:
            m = 2 * (n - vs.size) + 16
            v = rng.uniform(0.0, 2 * math.pi, m)
            acc = rng.random(m) < (R + r * np.cos(v)) / (R + r)
            vs = np.concatenate([vs, v[acc]])
        v = vs[:n]
        u = rng.uniform(0.0, 2 * math.pi, n)
        return np.stack([(R + r * np.cos(v)) * np.cos(u),
                         (R + r * np.cos(v)) * np.sin(u),
                         r * np.sin(v)], axis=1)
    raise ValueError(f"unknown manifold {kind!r}")


def knn_graph(points: np.ndarray, k: int) -> CSR:
    """Union-symmetrised kNN graph with w_ij = exp(-|p_i - p_j|^2 / sigma^2),
    sigma = median over nodes of the distance to the k-th nearest neighbour.
    Each undirected pair's squared distance is computed once, so W is exactly
    symmetric.  Point order is kept as sampled (no spatial sort)."""
    from scipy.spatial import cKDTree
    n = points.shape[0]
    tree = cKDTree(points)
    dist, idx = tree.query(points, k=k + 1)
    # drop self: the query returns the point itself first except on exact ties
    rows = np.repeat(np.arange(n, dtype=np.int64), k + 1)
    cols = idx.reshape(-1).astype(np.int64)
    keep = rows != cols
    rows, cols = rows[keep], cols[keep]
    # at most k neighbours per row (ties with duplicates could leave k+1)
    sigma = float(np.median(dist[:, k]))
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    d2 = np.sum((points[lo] - points[hi]) ** 2, axis=1)
    w = np.exp(-d2 / (sigma * sigma))
    # exp underflow would make a zero weight: clamp to the smallest normal
    w = np.maximum(w, np.finfo(np.float64).tiny)
    return from_edges(n, lo, hi, w)


def manifold_graph(kind: str, n: int, k: int, seed: int) -> CSR:
    rng = np.random.default_rng(seed)
    return knn_graph(sample_points(kind, n, rng), k)


# ----------------------------------------------------------------------------
# Small named graphs
# ----------------------------------------------------------------------------

def ring(n: int, k: int = 1, w: float = 1.0) -> CSR:
    """Circulant ring C_n(1..k): node i joined to i +- 1..k (mod n)."""
    i = np.repeat(np.arange(n), k)
    s = np.tile(np.arange(1, k + 1), n)
    return from_edges(n, i, (i + s) % n, np.full(i.size, w))


def line(n: int, w: float = 1.0) -> CSR:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, np.full(n - 1, w))


def complete(n: int, w: float = 1.0) -> CSR:
    i, j = np.triu_indices(n, 1)
    return from_edges(n, i, j, np.full(i.size, w))


def star(n: int, w: float = 1.0) -> CSR:
    """Node 0 joined to nodes 1..n-1."""
    j = np.arange(1, n)
    return from_edges(n, np.zeros(n - 1, dtype=np.int64), j, np.full(n - 1, w))


def complete_bipartite(a: int, b: int, w: float = 1.0) -> CSR:
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, i.ravel(), j.ravel(), np.full(a * b, w))


def tri_mesh(side: int = 3, w: float = 1.0) -> CSR:
    """Triangular lattice filling an equilateral triangle with `side` edges per
    side: (side+1)(side+2)/2 nodes, 3 side (side+1)/2 equal edges.  side = 3
    gives the 10-node, 18-edge mesh of the paper's Section 5.2."""
    nodes = {}
    for a in range(side + 1):
        for b in range(side + 1 - a):
            nodes[(a, b)] = len(nodes)
    ei, ej = [], []
    for (a, b), u in nodes.items():
        for da, db in ((1, 0), (0, 1), (-1, 1)):
            v = nodes.get((a + da, b + db))
            if v is not None:
                ei.append(u)
                ej.append(v)
    n = len(nodes)
    return from_edges(n, np.array(ei), np.array(ej), np.full(len(ei), w))


def grid(nx: int, ny: int, w: float = 1.0) -> CSR:
    idx = np.arange(nx * ny).reshape(nx, ny)
    i = np.concatenate([idx[:-1, :].ravel(), idx[:, :-1].ravel()])
    j = np.concatenate([idx[1:, :].ravel(), idx[:, 1:].ravel()])
    return from_edges(nx * ny, i, j, np.full(i.size, w))


def random_graph(n: int, p: float, seed: int, wlo: float = 0.25, whi: float = 2.0,
                 connect: bool = True) -> CSR:
    """Erdos-Renyi G(n, p) with uniform random weights; with `connect`, a
    random spanning path is added so no node is isolated."""
    rng = np.random.default_rng(seed)
    i, j = np.triu_indices(n, 1)
    m = rng.random(i.size) < p
    i, j = i[m], j[m]
    if connect:
        perm = rng.permutation(n)
        i = np.concatenate([i, perm[:-1]])
        j = np.concatenate([j, perm[1:]])
    w = rng.uniform(wlo, whi, i.size)
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    key, first = np.unique(lo * n + hi, return_index=True)
    return from_edges(n, key // n, key % n, w[first])


def sparse_random_graph(n: int, avg_degree: float, seed: int, wlo: float = 0.25,
                        whi: float = 2.0) -> CSR:
    """About n * avg_degree / 2 uniformly random edges plus a random spanning
    path (no isolated node), uniform random weights: an expander, whose
    breadth-first levels grow geometrically."""
    rng = np.random.default_rng(seed)
    m = int(n * avg_degree / 2)
    i = rng.integers(0, n, m)
    j = rng.integers(0, n, m)
    perm = rng.permutation(n)
    i = np.concatenate([i, perm[:-1]])
    j = np.concatenate([j, perm[1:]])
    keep = i != j
    i, j = i[keep], j[keep]
    w = rng.uniform(wlo, whi, i.size)
    lo = np.minimum(i, j).astype(np.int64)
    hi = np.maximum(i, j).astype(np.int64)
    key, first = np.unique(lo * n + hi, return_index=True)
    return from_edges(n, key // n, key % n, w[first])


def lattice_stencil(name: str, sigma2: float = 2.0):
    """Offsets and weights of a symmetric lattice stencil.  Weights are
    Gaussian in the Euclidean length of the offset, exp(-|s|^2 / sigma2),
    in the lattice's own geometry.

    cross       : (+-1, 0), (0, +-1)                       (square lattice)
    king        : cross plus (+-1, +-1)                    (square lattice)
    triangular  : (+-1, 0), (0, +-1), +-(1, -1), all of length 1
                  (the triangular lattice in a 60-degree basis)
    """
    if name == "cross":
        offs = [(1, 0), (-1, 0), (0, 1), (0, -1)]
        lens2 = [1.0] * 4
    elif name == "king":
        offs = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]
        lens2 = [1.0] * 4 + [2.0] * 4
    elif name == "triangular":
        offs = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1)]
        lens2 = [1.0] * 6
    else:
        raise ValueError(f"unknown stencil {name!r}")
    return offs, [math.exp(-l2 / sigma2) for l2 in lens2]


def periodic_lattice(n1: int, n2: int, offsets, weights) -> CSR:
    """Graph on Z_n1 x Z_n2 (node (x, y) has id x * n2 + y) joining (x, y) to
    ((x + a) mod n1, (y + b) mod n2) with weight w for each offset (a, b)
    and weight w of the stencil.  The stencil must be symmetric (each offset's
    negation listed with the same weight) and small enough for the lattice
    that no two offsets land on the same node."""
    offs = np.asarray(offsets, dtype=np.int64)
    w = np.asarray(weights, dtype=np.float64)
    n = n1 * n2
    x, y = np.divmod(np.arange(n, dtype=np.int64), n2)
    nb = ((x[:, None] + offs[None, :, 0]) % n1) * n2 + (y[:, None] + offs[None, :, 1]) % n2
    order = np.argsort(nb, axis=1, kind="stable")
    col = np.take_along_axis(nb, order, axis=1)
    val = np.broadcast_to(w, nb.shape)
    val = np.take_along_axis(val, order, axis=1)
    if np.any(np.diff(col, axis=1) == 0) or np.any(col == np.arange(n)[:, None]):
        raise ValueError("lattice too small for the stencil")
    rowptr = np.arange(n + 1, dtype=np.int64) * offs.shape[0]
    return CSR(n, rowptr, col.ravel().astype(np.int32), np.ascontiguousarray(val.ravel()))


def disjoint_union(graphs) -> CSR:
    rows, cols, vals = [], [], []
    off = 0
    for g in graphs:
        r = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr))
        rows.append(r + off)
        cols.append(g.col.astype(np.int64) + off)
        vals.append(g.val)
        off += g.n
    return from_edges(off, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


# ----------------------------------------------------------------------------
# Random starting block and workload mixes
# ----------------------------------------------------------------------------

def initial_block(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded Gaussian N x k starting block (row-major float64)."""
    return np.random.default_rng(seed).standard_normal((n, k))


CONFIGS = {
    # name: (manifold, N, kNN k, K, tol)
    "square_2k": ("square", 2000, 8, 4, 1e-8),
    "swiss_roll_100k": ("swiss_roll", 100_000, 10, 8, 1e-6),
    "sphere_1m": ("sphere", 1_000_000, 12, 16, 1e-6),
}


def batch_specs(count: int = 512, seed: int = 1000, nmin: int = 500, nmax: int = 20_000):
    """The batched mix: N log-uniform in [nmin, nmax], manifold uniform in
    {square, swiss_roll, torus}, 8-NN, K uniform in {4, 8, 16}.  Graph g uses
    seed `seed + g`.  Returns a list of (kind, N, k, K, seed)."""
    out = []
    for g in range(count):
        rng = np.random.default_rng(seed + g)
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        kind = ("square", "swiss_roll", "torus")[int(rng.integers(3))]
        K = (4, 8, 16)[int(rng.integers(3))]
        out.append((kind, n, 8, K, seed + g))
    return out


def serve_arrivals(count: int, rate: float = 200.0, seed: int = 7, nmin: int = 1000,
                   nmax: int = 200_000):
    """Poisson arrivals at `rate` per second; N log-uniform in [nmin, nmax];
    manifold uniform in {square, swiss_roll, sphere}; 10-NN, K = 8.
    Returns a list of (t_arrival_s, kind, N, k, K, graph_seed)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for q in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        kind = ("square", "swiss_roll", "sphere")[int(rng.integers(3))]
        out.append((float(t[q]), kind, n, 10, 8, 10_000 + q))
    return out
