"""Operators of the generalized eigenproblem, built as the paper defines them.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings taken where the paper is silent, ambiguous or inconsistent:

R1  Theta_i (eq. (Q)).  The printed matrix puts 1/T_i at the (i, i) entry.
    With that entry Q is not a Laplacian: it is indefinite on manifold graphs,
    contradicting "Laplacian has lambda_1(Q) = 0" and eps > 0 (Section 4.2).
    We read Theta_i = (1/T_i) sum_{j in T_i} (e_i - e_j)(e_i - e_j)^T, whose
    (i, i) entry is 1.  ``reading="literal"`` builds the printed form, only to
    show that it breaks the method.
R2  The two-hop term of eq. (contri) carries no 1/T_i; eq. (Q) does.  We
    follow eq. (Q) and read eq. (contri) as explanatory.
R3  T_i = nodes j != i reachable from i by a path of exactly two edges with
    (i, j) not an edge; unweighted; symmetric because W is.
R4  T_i = 0: Theta_i := 0 (row i of the two-hop term is empty) and row i takes
    no part in the minimum over mu_i.  With Q = 0 or a disconnected two-hop
    graph, lambda_2(Q) = 0: then eps = mu = 0 and A = L (status "eps_zero").
R5  mu = min over rows with a positive denominator of eq. (mu).
R6  r_i = sum_{j != i} |A_ij| (the diagonal, which holds eps, is excluded).
R7  b_1 = r_1 / (prod_j r_j)^(1/N), b_i = r_i b_1 / r_1, with the geometric
    mean taken through logarithms so that it cannot overflow.  r_i = 0 (an
    isolated node) is an input error.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class OracleInputError(ValueError):
    """Invalid graph; ``code`` is one of invalid_arg, self_loop, bad_weight,
    not_symmetric, isolated_node (checked in that order)."""

    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


# ----------------------------------------------------------------------------
# Section 3.1: the graph G(V, E, W)
# ----------------------------------------------------------------------------

def validate(n, rowptr, col, val):
    """Check that (rowptr, col, val) is the adjacency of a graph as Section 3.1
    defines it: W_ij > 0 exactly on the edges, symmetric, no self loops; plus
    the storage rules (sorted unique columns) and no isolated node (Section
    4.3 needs r_i > 0)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    if n < 1 or rowptr.shape != (n + 1,) or rowptr[0] != 0:
        raise OracleInputError("invalid_arg", "bad n or rowptr")
    if np.any(np.diff(rowptr) < 0) or rowptr[-1] != col.size or col.size != val.size:
        raise OracleInputError("invalid_arg", "rowptr not monotone or sizes differ")
    if col.size and (col.min() < 0 or col.max() >= n):
        raise OracleInputError("invalid_arg", "column out of range")
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    if col.size > 1:
        same_row = rows[1:] == rows[:-1]
        if np.any(same_row & (col[1:] <= col[:-1])):
            raise OracleInputError("invalid_arg", "columns not strictly increasing")
    if np.any(rows == col):
        raise OracleInputError("self_loop", "W_ii != 0")
    if not np.all(np.isfinite(val)) or np.any(val <= 0):
        raise OracleInputError("bad_weight", "weights must be finite and > 0")
    Wm = sp.csr_matrix((val, col, rowptr), shape=(n, n))
    diff = Wm - Wm.T
    if diff.nnz and np.any(diff.data != 0):
        raise OracleInputError("not_symmetric", "W != W^T")
    if np.any(np.diff(rowptr) == 0):
        raise OracleInputError("isolated_node", "a node has no edge")
    return Wm


def degrees(W: sp.csr_matrix) -> np.ndarray:
    """D_ii = sum_j W_ij (Section 3.1)."""
    return np.asarray(W.sum(axis=1)).ravel()


def laplacian(W: sp.csr_matrix) -> sp.csr_matrix:
    """L = D - W (Section 3.1)."""
    return (sp.diags(degrees(W)) - W).tocsr()


# ----------------------------------------------------------------------------
# Section 4.1.1: disconnected two-hop neighbours and Q
# ----------------------------------------------------------------------------

def two_hop(W: sp.csr_matrix):
    """T_i = {j : j != i, (i, j) not in E, j reachable from i in two hops}
    (reading R3).  Returns (rowptr int64, col int32 sorted, counts int64).

    The pattern is (P P > 0) and not P and not I, with P the 0/1 pattern of
    W; the boolean product is one library sparse matrix product."""
    n = W.shape[0]
    P = sp.csr_matrix((np.ones(W.nnz), W.indices, W.indptr), shape=(n, n))
    P2 = (P @ P).tocsr()
    P2.sum_duplicates()
    P2.data[:] = 1.0
    # remove the diagonal and the one-hop pattern
    T = (P2 - P2.multiply(P)).tocsr()
    T = (T - sp.diags(T.diagonal())).tocsr()
    T.eliminate_zeros()
    T.sort_indices()
    counts = np.diff(T.indptr).astype(np.int64)
    return T.indptr.astype(np.int64), T.indices.astype(np.int32), counts


def two_hop_rows(n, rowptr, col, rows):
    """T_i for the listed rows only, straight from the definition (reading
    R3): the neighbours of the neighbours of i, minus i and its own
    neighbours.  For checking sampled rows of graphs too large for the
    whole pattern.  Returns a list of sorted int arrays."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col)
    out = []
    for i in rows:
        nbr = set(col[rowptr[i]:rowptr[i + 1]].tolist())
        two = set()
        for k in nbr:
            two.update(col[rowptr[k]:rowptr[k + 1]].tolist())
        two.discard(int(i))
        two.difference_update(nbr)
        out.append(np.array(sorted(two), dtype=np.int64))
    return out


def q_diag_rows(n, rowptr, col, rows):
    """Q_ii for the listed rows under reading R1: sum over j in T_i of
    (1/T_i + 1/T_j) = 1 + sum_j 1/T_j (0 when T_i is empty)."""
    out = []
    for i, ti in zip(rows, two_hop_rows(n, rowptr, col, rows)):
        if ti.size == 0:
            out.append(0.0)
            continue
        tj = two_hop_rows(n, rowptr, col, ti.tolist())
        out.append(sum(1.0 / ti.size + 1.0 / t.size for t in tj))
    return np.array(out)


def operator_a_rows(n, rowptr, col, val, rows, mu: float, eps: float, X):
    """(A X)_i for the listed rows from the definitions, A = L - mu Q + eps I
    (eq. (obj2), reading R1 for Q): d_i x_i - sum_j w_ij x_j
    - mu (Q_ii x_i - sum_{j in T_i} (1/T_i + 1/T_j) x_j) + eps x_i."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((len(rows), X.shape[1]))
    trows = two_hop_rows(n, rowptr, col, rows)
    for q, (i, ti) in enumerate(zip(rows, trows)):
        cols = np.asarray(col[rowptr[i]:rowptr[i + 1]], dtype=np.int64)
        w = np.asarray(val[rowptr[i]:rowptr[i + 1]], dtype=np.float64)
        y = w.sum() * X[i] - w @ X[cols]
        if ti.size:
            tj = np.array([t.size for t in two_hop_rows(n, rowptr, col, ti.tolist())], float)
            qij = 1.0 / ti.size + 1.0 / tj
            y -= mu * (qij.sum() * X[i] - qij @ X[ti])
        out[q] = y + eps * X[i]
    return out


def theta_sum_q(n, t_rowptr, t_col, reading: str = "R1") -> sp.csr_matrix:
    """Q = sum_i Theta_i (eq. (Q)).  Each Theta_i is added entry by entry:
    for j in T_i, +1/T_i at (j, j), -1/T_i at (i, j) and (j, i); at (i, i)
    +1 per member of T_i under reading R1 (i.e. T_i * 1/T_i = 1), or the printed
    single 1/T_i under ``reading="literal"``."""
    t_rowptr = np.asarray(t_rowptr, dtype=np.int64)
    cnt = np.diff(t_rowptr)
    i_of = np.repeat(np.arange(n), cnt)
    j_of = np.asarray(t_col, dtype=np.int64)
    inv = np.zeros(n)
    nz = cnt > 0
    inv[nz] = 1.0 / cnt[nz]
    c = inv[i_of]  # 1/T_i for each member j of T_i
    rows = [j_of, i_of, j_of]
    cols = [j_of, j_of, i_of]
    vals = [c, -c, -c]
    if reading == "R1":
        rows.append(i_of)
        cols.append(i_of)
        vals.append(c)
    elif reading == "literal":
        rows.append(np.arange(n)[nz])
        cols.append(np.arange(n)[nz])
        vals.append(inv[nz])
    else:
        raise ValueError(reading)
    Q = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    Q.sum_duplicates()
    return Q


def two_hop_components(n, t_rowptr, t_col) -> int:
    """Number of connected components of the two-hop graph (nodes with an
    empty T_i count as components of their own).  Q is the Laplacian of that
    graph under R1, so lambda_2(Q) = 0 exactly when this exceeds 1."""
    from scipy.sparse.csgraph import connected_components
    G = sp.csr_matrix((np.ones(len(t_col)), np.asarray(t_col), np.asarray(t_rowptr)),
                      shape=(n, n))
    ncomp, _ = connected_components(G, directed=False)
    return int(ncomp)


def fiedler_value(Q: sp.csr_matrix, components: int | None = None,
                  dense_max: int = 3000, method: str = "shift_invert") -> float:
    """eps = lambda_2(Q), the second smallest eigenvalue (Section 4.2).

    Dense symmetric eigenvalues for N <= dense_max; otherwise ARPACK, either
    shift-invert about a small negative shift (Q is singular; needs a sparse
    LU of Q) or, with ``method="smallest"``, plain Lanczos for the smallest
    algebraic eigenvalues of Q itself (matrix-vector products only: slower to
    converge, but no factorisation, so it reaches graphs whose LU does not
    fit).  When the two-hop graph has more than one component the value is
    exactly 0 (R4)."""
    n = Q.shape[0]
    if components is not None and components > 1:
        return 0.0
    if n <= dense_max:
        return float(np.linalg.eigvalsh(Q.toarray())[1]) if n > 1 else 0.0
    if method == "smallest":
        vals = spla.eigsh(Q.tocsr(), k=6, which="SA", return_eigenvectors=False,
                          tol=1e-13, ncv=48)
        return float(np.sort(vals)[1])
    if method != "shift_invert":
        raise ValueError(method)
    scale = float(abs(Q.diagonal()).max())
    vals = spla.eigsh(Q.tocsc(), k=3, sigma=-1e-3 * scale, which="LM",
                      return_eigenvectors=False, tol=1e-14)
    return float(np.sort(vals)[1])


def mu_from_q(Q: sp.csr_matrix, eps: float) -> float:
    """mu_i = eps / (Q_ii - sum_{j != i} Q_ij) (eq. (mu)); mu = min_i mu_i over
    rows with a positive denominator (R5)."""
    Q = Q.tocsr()
    diag = Q.diagonal()
    off = np.asarray(Q.sum(axis=1)).ravel() - diag
    den = diag - off
    pos = den > 0
    if eps == 0.0 or not np.any(pos):
        return 0.0
    return float(np.min(eps / den[pos]))


def operator_a(L, Q, mu: float, eps: float) -> sp.csr_matrix:
    """A = L - mu Q + eps I (eq. (obj2))."""
    n = L.shape[0]
    A = (L - mu * Q + eps * sp.identity(n, format="csr")).tocsr()
    A.sum_duplicates()
    return A


def gershgorin_radii(A: sp.csr_matrix) -> np.ndarray:
    """r_i = sum_{j != i} |A_ij| (Section 3.2, reading R6)."""
    absA = abs(A).tocsr()
    return np.asarray(absA.sum(axis=1)).ravel() - abs(A.diagonal())


def b_from_radii(r: np.ndarray) -> np.ndarray:
    """r_1/b_1 = ... = r_N/b_N with prod b_i = 1 (Section 4.3):
    b_1 = r_1 / (prod r)^(1/N), b_i = r_i b_1 / r_1 (reading R7)."""
    r = np.asarray(r, dtype=np.float64)
    if np.any(r <= 0):
        raise OracleInputError("isolated_node", "a Gershgorin radius is zero")
    geo = np.exp(np.mean(np.log(r)))
    b1 = r[0] / geo
    return r * (b1 / r[0])


def build_ops(n, rowptr, col, val, reading: str = "R1",
              eps_method: str = "shift_invert") -> dict:
    """All operators of the problem for one graph (``eps_method``: the
    ARPACK route of ``fiedler_value`` for large graphs)."""
    W = validate(n, rowptr, col, val)
    d = degrees(W)
    L = laplacian(W)
    t_rowptr, t_col, t_cnt = two_hop(W)
    Q = theta_sum_q(n, t_rowptr, t_col, reading=reading)
    ncomp = two_hop_components(n, t_rowptr, t_col)
    eps = fiedler_value(Q, components=ncomp if reading == "R1" else None,
                        method=eps_method)
    mu = mu_from_q(Q, eps)
    A = operator_a(L, Q, mu, eps)
    r = gershgorin_radii(A)
    b = b_from_radii(r)
    return dict(W=W, d=d, L=L, t_rowptr=t_rowptr, t_col=t_col, t_count=t_cnt, Q=Q,
                components=ncomp, eps=eps, mu=mu, A=A, r=r, b=b,
                eps_zero=(eps == 0.0))
