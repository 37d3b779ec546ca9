"""Clustering of the embedding and its four criteria (Section 5.1, Table 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5.1 clusters the rows of the embedding into C clusters with k-means
and with a Gaussian mixture model (GMM), and scores each clustering against
the known classes with the Rand index (RI), Precision, Purity and
normalised mutual information (NMI); Table 3 reports the average of the
k-means and GMM scores.  The paper names the algorithms only.  Readings:

C1  k-means: Lloyd iterations.  Seeding by k-means++: the first centre is
    the point floor(u_0 n); centre t is the first point i whose cumulative
    sum of D(x)^2 (squared distance to the nearest centre chosen so far,
    summed in point order) exceeds u_t times the total.  The uniforms u_t
    are inputs.
C2  Squared distances are summed over the coordinates in order, each
    difference squared by a plain product.  A point joins the nearest
    centre, ties to the lower index.  A centre is the mean of its points;
    an empty cluster keeps its centre.  Iterate until no point changes
    cluster, at most 100 iterations.
C3  GMM: full covariances, EM started from the k-means partition (weights
    = cluster fractions, means = centres, covariances = within-cluster
    covariances).  Each covariance gets reg * I added, reg = 1e-6 times the
    mean per-coordinate variance of the data (the embedding's scale shrinks
    like n^(-1/2)).  EM stops when the log-likelihood changes by at most
    1e-6 of its magnitude, at most 100 iterations.  A point's cluster is
    its most responsible component (ties to the lower index).
C4  Criteria from the contingency table n_ij (class i, cluster j), with
    a_i, b_j its sums and pairs(x) = x (x - 1) / 2:
      TP = sum_ij pairs(n_ij), Ppred = sum_j pairs(b_j),
      Ptrue = sum_i pairs(a_i), Tot = pairs(n);
      RI = (Tot - Ppred - Ptrue + 2 TP) / Tot,  Precision = TP / Ppred,
      Purity = sum_j max_i n_ij / n,
      NMI = I(U; V) / sqrt(H(U) H(V)) (1 if both entropies are 0, 0 if
      only one is).
"""
from __future__ import annotations

import numpy as np

MAX_ITER = 100


def sq_dists(x, c):
    """C2: n x C squared distances, the terms in coordinate order."""
    d = np.zeros((x.shape[0], c.shape[0]))
    for k in range(x.shape[1]):
        t = x[:, k][:, None] - c[:, k][None, :]
        d = d + t * t
    return d


def kmeanspp_seeds(x, C, u):
    """C1: indices of the C seeds from the uniforms u[0..C-1]."""
    n = x.shape[0]
    seeds = [min(int(np.floor(u[0] * n)), n - 1)]
    d2 = sq_dists(x, x[seeds])[:, 0]
    for t in range(1, C):
        cs = np.cumsum(d2)  # sequential, in point order
        target = u[t] * cs[-1]
        i = int(np.searchsorted(cs, target, side="right"))
        seeds.append(min(i, n - 1))
        d2 = np.minimum(d2, sq_dists(x, x[[seeds[-1]]])[:, 0])
    return np.array(seeds)


def assign(x, centres):
    """C2: nearest centre, ties to the lower index (argmin's rule)."""
    return np.argmin(sq_dists(x, centres), axis=1)


def update(x, labels, centres):
    """C2: means of the clusters; an empty cluster keeps its centre."""
    out = centres.copy()
    for c in range(centres.shape[0]):
        m = labels == c
        if m.any():
            out[c] = x[m].sum(axis=0) / m.sum()
    return out


def kmeans(x, C, u, max_iter: int = MAX_ITER):
    x = np.asarray(x, dtype=np.float64)
    centres = x[kmeanspp_seeds(x, C, u)].copy()
    labels = assign(x, centres)
    it = 0
    for it in range(1, max_iter + 1):
        centres = update(x, labels, centres)
        new = assign(x, centres)
        if np.array_equal(new, labels):
            break
        labels = new
    return labels, centres, it


def _log_gauss(x, mu, cov):
    """log N(x | mu, cov) for every row of x (Cholesky of cov)."""
    K = x.shape[1]
    L = np.linalg.cholesky(cov)
    y = np.linalg.solve(L, (x - mu).T)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    return -0.5 * (K * np.log(2.0 * np.pi) + logdet + np.sum(y * y, axis=0))


def gmm(x, C, labels0, max_iter: int = MAX_ITER, tol: float = 1e-6):
    """C3: EM for a full-covariance mixture from the partition labels0.
    Returns (labels, weights, means, covs, log-likelihood, iterations)."""
    x = np.asarray(x, dtype=np.float64)
    n, K = x.shape
    reg = 1e-6 * float(np.mean(np.var(x, axis=0)))
    w = np.zeros(C)
    mu = np.zeros((C, K))
    cov = np.zeros((C, K, K))
    for c in range(C):
        m = labels0 == c
        nc = max(int(m.sum()), 1)
        w[c] = m.sum() / n
        mu[c] = x[m].mean(axis=0) if m.any() else x.mean(axis=0)
        xc = x[m] - mu[c]
        cov[c] = xc.T @ xc / nc + reg * np.eye(K)
    w = np.maximum(w, 1e-300)
    prev = None
    ll = -np.inf
    it = 0
    for it in range(1, max_iter + 1):
        lg = np.stack([_log_gauss(x, mu[c], cov[c]) + np.log(w[c]) for c in range(C)], axis=1)
        mx = lg.max(axis=1, keepdims=True)
        s = np.log(np.exp(lg - mx).sum(axis=1)) + mx[:, 0]
        ll = float(s.sum())
        r = np.exp(lg - s[:, None])
        if prev is not None and abs(ll - prev) <= tol * abs(ll):
            break
        prev = ll
        nk = r.sum(axis=0)
        w = np.maximum(nk / n, 1e-300)
        for c in range(C):
            if nk[c] <= 0:
                continue
            mu[c] = (r[:, c] @ x) / nk[c]
            xc = x - mu[c]
            cov[c] = (xc.T * r[:, c]) @ xc / nk[c] + reg * np.eye(K)
    lg = np.stack([_log_gauss(x, mu[c], cov[c]) + np.log(w[c]) for c in range(C)], axis=1)
    return np.argmax(lg, axis=1), w, mu, cov, ll, it


def contingency(classes, clusters):
    classes = np.asarray(classes, dtype=np.int64)
    clusters = np.asarray(clusters, dtype=np.int64)
    t = np.zeros((classes.max() + 1, clusters.max() + 1), dtype=np.int64)
    np.add.at(t, (classes, clusters), 1)
    return t


def criteria(classes, clusters):
    """C4: dict of RI, Precision, Purity, NMI."""
    t = contingency(classes, clusters)
    n = int(t.sum())
    pairs = lambda v: v * (v - 1) / 2.0  # noqa: E731
    a = t.sum(axis=1)
    b = t.sum(axis=0)
    tp = float(pairs(t).sum())
    ppred = float(pairs(b).sum())
    ptrue = float(pairs(a).sum())
    tot = pairs(float(n))
    ri = (tot - ppred - ptrue + 2.0 * tp) / tot
    precision = tp / ppred if ppred > 0 else 0.0
    purity = float(t.max(axis=0).sum()) / n
    pij = t / n
    pa = a / n
    pb = b / n
    nz = t > 0
    mi = float(np.sum(pij[nz] * np.log(pij[nz] / np.outer(pa, pb)[nz])))
    ha = float(-np.sum(pa[pa > 0] * np.log(pa[pa > 0])))
    hb = float(-np.sum(pb[pb > 0] * np.log(pb[pb > 0])))
    if ha == 0.0 and hb == 0.0:
        nmi = 1.0
    elif ha == 0.0 or hb == 0.0:
        nmi = 0.0
    else:
        nmi = mi / np.sqrt(ha * hb)
    return {"RI": ri, "Precision": precision, "Purity": purity, "NMI": nmi}
