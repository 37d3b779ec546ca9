"""Closed forms of every operator for periodic lattices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A periodic lattice is the graph on Z_{n1} x Z_{n2} (node (x, y) has id
x * n2 + y) in which (x, y) is joined to ((x + a) mod n1, (y + b) mod n2) for
every offset s = (a, b) of a stencil S, with weight w_s.  The stencil is
symmetric (s in S implies -s in S, w_{-s} = w_s), so W is symmetric (Section
3.1), and the graph is translation invariant: every quantity the method
defines is the same at every node, and every operator is diagonalised by the
lattice's Fourier modes.  That gives each of them in closed form, from the
definitions alone and with no linear algebra, valid at any size (the
two-dimensional form of the circulant-ring closed form):

* degree d = sum_s w_s; the Laplacian L = D - W (Section 3.1) has, for the
  mode theta = (2 pi m1 / n1, 2 pi m2 / n2), the eigenvalue
  lambda_L = sum_s w_s (1 - cos(s . theta)).
* The disconnected two-hop set (Section 4.1.1) of every node is the offset
  set U = (S + S) minus S minus {0}, so T_i = |U| =: t for all i.
* Under reading R1 of eq. (Q), Q is the Laplacian of the two-hop graph with
  weights 1/T_i + 1/T_j = 2/t: Q_ii = 2 and
  lambda_Q = sum_{u in U} (2/t) (1 - cos(u . theta)).
* eps = lambda_2(Q) (Section 4.2) is the smallest lambda_Q over the modes
  other than theta = 0 (0 exactly when the two-hop graph is disconnected,
  reading R4).
* The denominator of eq. (mu) is Q_ii - sum_{j != i} Q_ij = 4 at every node,
  so mu = eps / 4.
* r_i = d + mu * 2 (Section 4.3, reading R6) is the same at every node, so
  b = 1 and B = I.
* A = L - mu Q + eps I (eq. (obj2)) has lambda_A = lambda_L - mu lambda_Q + eps
  for each mode, with the real eigenvectors cos(theta . (x, y)) and
  sin(theta . (x, y)); theta and -theta give the same eigenvalue.

All of this needs the offsets {0} + S + (S + S) to stay distinct modulo
(n1, n2) (no wrap-around identifies two of them); ``check_lattice`` enforces
that.  Graph inputs of this shape come from ``synthgraphs.periodic_lattice``.
"""
from __future__ import annotations

import itertools

import numpy as np


def _canon(s, n1, n2):
    return (s[0] % n1, s[1] % n2)


def two_hop_offsets(stencil):
    """U = (S + S) minus S minus {0}: the offsets of the disconnected two-hop
    set of every node (Section 4.1.1), as a sorted list."""
    S = set(map(tuple, stencil))
    sums = {(a[0] + b[0], a[1] + b[1]) for a, b in itertools.product(S, S)}
    return sorted(sums - S - {(0, 0)})


def check_lattice(n1: int, n2: int, stencil, weights) -> None:
    """Raise ValueError unless the stencil is symmetric with symmetric
    positive weights and {0}, S and S + S stay distinct modulo (n1, n2)."""
    S = [tuple(s) for s in stencil]
    if len(set(S)) != len(S) or (0, 0) in S:
        raise ValueError("stencil offsets must be distinct and nonzero")
    w = dict(zip(S, weights))
    for s in S:
        neg = (-s[0], -s[1])
        if neg not in w or w[neg] != w[s] or not w[s] > 0:
            raise ValueError("stencil must be symmetric with equal positive weights")
    allo = {(0, 0)} | set(S) | set(two_hop_offsets(S))
    if len({_canon(o, n1, n2) for o in allo}) != len(allo):
        raise ValueError("lattice too small: offsets wrap around")


def _mode_grid(n1, n2):
    m1, m2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    return m1.ravel(), m2.ravel()


def _symbol(n1, n2, offsets, coef, m1, m2):
    """sum_o coef_o (1 - cos(o . theta)) for the modes (m1, m2), with exact
    zeros where every o . theta is a multiple of 2 pi (integer test)."""
    out = np.zeros(m1.size)
    exact_zero = np.ones(m1.size, dtype=bool)
    for (a, b), c in zip(offsets, coef):
        # o . theta / (2 pi) = (a m1 n2 + b m2 n1) / (n1 n2)
        num = a * m1.astype(np.int64) * n2 + b * m2.astype(np.int64) * n1
        whole = (num % (n1 * n2)) == 0
        exact_zero &= whole
        phase = 2.0 * np.pi * (a * m1 / n1 + b * m2 / n2)
        term = 1.0 - np.cos(phase)
        term[whole] = 0.0
        out += c * term
    out[exact_zero] = 0.0
    return out


def lattice_spectrum(n1: int, n2: int, stencil, weights) -> dict:
    """Every operator of the method on the periodic lattice, in closed form.
    Returns a dict with the per-node values (d, t, qdiag, den, r, b), the
    scalars eps and mu, and per mode (arrays over the n1 * n2 modes, mode q =
    (m1[q], m2[q])) lambda_L, lambda_Q and lambda_A."""
    check_lattice(n1, n2, stencil, weights)
    S = [tuple(s) for s in stencil]
    w = np.asarray(weights, dtype=np.float64)
    U = two_hop_offsets(S)
    t = len(U)
    m1, m2 = _mode_grid(n1, n2)
    lam_l = _symbol(n1, n2, S, w, m1, m2)
    q = 2.0 / t if t else 0.0
    lam_q = _symbol(n1, n2, U, np.full(t, q), m1, m2)
    nonzero_mode = (m1 != 0) | (m2 != 0)
    eps = float(lam_q[nonzero_mode].min()) if nonzero_mode.any() else 0.0
    qdiag = t * q                    # = 2 (0 when U is empty)
    den = 2.0 * qdiag                # Q_ii - sum_{j != i} Q_ij
    mu = eps / den if den > 0 and eps > 0 else 0.0
    d = float(w.sum())
    r = d + mu * qdiag
    lam_a = lam_l - mu * lam_q + eps
    return dict(n=n1 * n2, d=d, t=t, two_hop_offsets=U, qdiag=qdiag, den=den, eps=eps, mu=mu,
                r=r, b=1.0, m1=m1, m2=m2, lam_l=lam_l, lam_q=lam_q, lam_a=lam_a)


def smallest(spec: dict, count: int):
    """The `count` smallest generalized eigenvalues (B = I) and their modes,
    ascending (ties by mode index)."""
    order = np.lexsort((np.arange(spec["lam_a"].size), spec["lam_a"]))[:count]
    return spec["lam_a"][order], list(zip(spec["m1"][order].tolist(), spec["m2"][order].tolist()))


def cluster_ends(lam, rtol: float = 1e-10):
    """Indices K (1-based counts) at which the sorted values `lam` close a
    cluster of equal eigenvalues: lam[K] exceeds lam[K - 1] by more than
    rtol relative."""
    lam = np.asarray(lam)
    return [k for k in range(1, lam.size)
            if lam[k] - lam[k - 1] > rtol * max(abs(lam[k]), abs(lam[k - 1]))]


def mode_basis(n1: int, n2: int, modes) -> np.ndarray:
    """Orthonormal real basis (n1 n2 x len(modes)) of the span of the modes:
    for each pair {theta, -theta} in the list, cos and sin of theta . (x, y)
    (node (x, y) in row x * n2 + y); a self-conjugate mode (2 theta = 0)
    gives its cosine only.  The list must hold both members of each pair."""
    ms = {(m1 % n1, m2 % n2) for m1, m2 in modes}
    x, y = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    x, y = x.ravel(), y.ravel()
    cols, seen = [], set()
    for m in sorted(ms):
        if m in seen:
            continue
        neg = ((-m[0]) % n1, (-m[1]) % n2)
        if neg not in ms:
            raise ValueError(f"mode {m} without its conjugate {neg}")
        seen.update({m, neg})
        ph = 2.0 * np.pi * (m[0] * x / n1 + m[1] * y / n2)
        c = np.cos(ph)
        cols.append(c / np.linalg.norm(c))
        if neg != m:
            s = np.sin(ph)
            cols.append(s / np.linalg.norm(s))
    return np.stack(cols, axis=1)
