"""The first K generalized eigenpairs of (A, B) and checks on them.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.3 asks for the first K generalized eigenvectors q_k of the pair
(A, B = diag(b)), A q = lambda B q, with q_i^T B q_j = delta_ij.  That result
has a plain definition, so the oracle computes it directly instead of
iterating:

* N <= dense_max: B is diagonal, so B^(1/2) = diag(sqrt(b)); the pairs are
  (lambda, B^(-1/2) y) for the symmetric eigenpairs (lambda, y) of
  B^(-1/2) A B^(-1/2) (dense LAPACK eigh).
* larger N: ARPACK shift-invert Lanczos for the pair (A, B) about a shift just
  below zero, with K + 1 pairs so that the gap after lambda_K is known.

Readings: the constraint printed as "P B P^T = I" is read P^T B P = I_K
(the only dimensionally consistent form); "first K" means the K smallest
generalized eigenvalues in ascending order, the first included; the
Rayleigh quotient of the pair is v^T A v / v^T B v.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .graph_ops import build_ops


def dense_generalized_eigs(A, b, K: int):
    """K + 1 smallest pairs via eigh of B^-1/2 A B^-1/2 (all of them computed)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    s = 1.0 / np.sqrt(np.asarray(b, dtype=np.float64))
    C = s[:, None] * Ad * s[None, :]
    C = 0.5 * (C + C.T)
    n = C.shape[0]
    m = min(K + 1, n)
    lam, Y = np.linalg.eigh(C)
    return lam[:m], s[:, None] * Y[:, :m]


def sparse_generalized_eigs(A, b, K: int, tol: float = 1e-13, method: str = "shift_invert"):
    """K + 1 smallest pairs by ARPACK: shift-invert on (A, B) about a shift
    just below zero (needs a sparse LU of A), or with ``method="smallest"``
    plain Lanczos for the smallest algebraic eigenvalues of the symmetric
    C = B^-1/2 A B^-1/2 (products only), the pairs (lambda, B^-1/2 y)."""
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    if method == "smallest":
        s = 1.0 / np.sqrt(b)
        C = sp.diags(s) @ A @ sp.diags(s)
        C = ((C + C.T) * 0.5).tocsr()
        lam, Y = spla.eigsh(C, k=K + 1, which="SA", tol=tol, ncv=max(4 * (K + 1), 64))
        order = np.argsort(lam)
        return lam[order], s[:, None] * Y[:, order]
    if method != "shift_invert":
        raise ValueError(method)
    shift = -1e-3 * float(np.mean(A.diagonal()))
    lam, V = spla.eigsh(A.tocsc(), k=K + 1, M=sp.diags(b).tocsc(), sigma=shift,
                        which="LM", tol=tol)
    order = np.argsort(lam)
    return lam[order], V[:, order]


def generalized_eigs(A, b, K: int, dense_max: int = 4000, method: str = "shift_invert"):
    n = A.shape[0]
    if n <= dense_max:
        lam, V = dense_generalized_eigs(A, b, K)
    else:
        lam, V = sparse_generalized_eigs(A, b, K, method=method)
    V = b_orthonormalize(V, b)
    return lam, V


def b_orthonormalize(V, b):
    """V (V^T B V)^(-1/2): B-orthonormal, same span."""
    G = V.T @ (np.asarray(b)[:, None] * V)
    w, U = np.linalg.eigh(0.5 * (G + G.T))
    return V @ (U / np.sqrt(w)) @ U.T


def relative_residuals(A, b, X, lam):
    """rho_j = |A x_j - lambda_j B x_j|_2 / (|lambda_j| |B x_j|_2)."""
    b = np.asarray(b, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    BX = b[:, None] * X
    R = A @ X - BX * lam[None, :]
    return np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(BX, axis=0))


def b_orthonormality_error(X, b) -> float:
    """max |X^T B X - I|."""
    X = np.asarray(X, dtype=np.float64)
    G = X.T @ (np.asarray(b)[:, None] * X)
    return float(np.max(np.abs(G - np.eye(G.shape[0]))))


def sin_principal_angle_b(X, Y, b) -> float:
    """Sine of the largest principal angle between span(X) and span(Y) in the
    B inner product: the B-norm of (I - X X^T B) Y with X, Y B-orthonormal."""
    b = np.asarray(b, dtype=np.float64)
    Xo = b_orthonormalize(np.asarray(X, dtype=np.float64), b)
    Yo = b_orthonormalize(np.asarray(Y, dtype=np.float64), b)
    Z = Yo - Xo @ (Xo.T @ (b[:, None] * Yo))
    s = np.sqrt(b)[:, None] * Z
    return float(sla.svdvals(s)[0]) if s.size else 0.0


def fix_signs(X):
    """Each column's entry of largest magnitude (lowest index on ties) made
    positive.  Only a convention for reproducible output."""
    X = np.array(X, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(X), axis=0)
    sgn = np.sign(X[idx, np.arange(X.shape[1])])
    sgn[sgn == 0] = 1.0
    return X * sgn[None, :]


def embed(n, rowptr, col, val, K: int, dense_max: int = 4000):
    """Operators of the graph, then the K smallest generalized eigenpairs.
    Returns (X N x K, lambda[K], info dict with operators, lambda_{K+1} and the
    relative gap (lambda_{K+1} - lambda_K) / lambda_K)."""
    ops = build_ops(n, rowptr, col, val)
    lam, V = generalized_eigs(ops["A"], ops["b"], K, dense_max=dense_max)
    X = fix_signs(V[:, :K])
    info = dict(ops)
    if lam.size > K:
        info["lam_next"] = float(lam[K])
        info["relgap"] = float((lam[K] - lam[K - 1]) / abs(lam[K - 1])) if lam[K - 1] else np.inf
    return X, lam[:K].copy(), info
