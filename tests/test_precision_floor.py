"""Why the eigenvector block X stays FP64: the lambda-relative residual
target (1e-6) is below what an FP32 copy of X can represent.

Rounding an exact generalized eigenvector x_j (oracle, FP64) to FP32 and
applying A in FP64 leaves rho_j = |A x - lam B x| / (|lam| |B x|) of order
2^-24 max_i A_ii / lam_j: the FP32 copy differs from x by relative 2^-24 in
every entry, and A amplifies that error by up to its norm while the true
residual is lam_j small.  The tests measure the floor on the 2000-node
square (K = 4) and the 20 000-node Swiss roll (K = 8) and check it lies
above 1e-6 and within the model's order.  (The correction block W is a
different matter: its rounding reaches X only through Rayleigh-Ritz
coefficients that shrink as the block converges, which the FP32 product
option exploits.)  CPU only (oracle)."""
import numpy as np
import pytest

import oracle
import synthgraphs as sg


def _floor(kind, n, k, K):
    g = sg.manifold_graph(kind, n, k, 0)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    A, b = ops["A"], ops["b"]
    lam, X = oracle.generalized_eigs(A, b, K)
    x32 = X.astype(np.float32).astype(np.float64)
    rho = oracle.relative_residuals(A, b, x32, lam)
    ratio = np.max(np.abs(A.diagonal())) / lam[-1]
    return float(np.max(rho)), float(ratio), oracle.relative_residuals(A, b, X, lam)


@pytest.mark.parametrize("kind,n,k,K,lo", [("square", 2000, 8, 4, 3e-6),
                                           ("swiss_roll", 20000, 10, 8, 1e-4)])
def test_fp32_storage_floor_exceeds_target(kind, n, k, K, lo):
    rho32, ratio, rho64 = _floor(kind, n, k, K)
    print(f"{kind} n={n} K={K}: max A_ii / lam_K = {ratio:.3g}, FP32 floor {rho32:.3g}")
    assert np.max(rho64) < 1e-9          # the FP64 eigenvectors themselves are exact
    assert rho32 > lo                    # FP32 storage alone misses the 1e-6 target
    assert rho32 < 64 * 2.0 ** -24 * ratio  # and stays within the model's order
