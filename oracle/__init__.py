"""CPU FP64 oracle for the manifold-graph embedding hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
and does not import it.

What it computes, following Chen, Cheung & Zhang, "Fast computation of
generalized eigenvectors for manifold graph embedding":

* ``graph_ops``: validation of the graph (Section 3.1), degrees and the
  combinatorial Laplacian L = D - W (Section 3.1), the disconnected two-hop
  sets T_i (Section 4.1.1), Q = sum_i Theta_i (eq. (Q)), epsilon = lambda_2(Q)
  (Section 4.2), mu = min_i mu_i (eq. (mu)), A = L - mu Q + eps I
  (eq. (obj2)), Gershgorin radii r_i and b_i (Section 4.3).
* ``solve``: the first K generalized eigenpairs of (A, B = diag(b)) with
  P^T B P = I (Section 4.3), by dense symmetric eigendecomposition of
  B^-1/2 A B^-1/2 for small N and by shift-invert Lanczos (ARPACK, a library
  eigensolver) for large N; residuals, B-orthonormality and principal angles.

* ``knn``: the k-nearest-neighbour graph of points (Section 5.1: kNN graphs
  from Euclidean distances), union-symmetrised, with Gaussian weights
  exp(-d^2 / sigma^2), sigma the median k-th neighbour distance.

* ``cluster``: k-means and Gaussian-mixture clustering of the embedding and
  the Rand index, Precision, Purity and NMI of Section 5.1 and Table 3.

* ``vbc``: betweenness centrality (eq. (3) of Section 3.3) and its variance,
  the check that accepts a graph as a manifold graph (Table 1).

Readings of passages that are silent or ambiguous are listed at the top of
``graph_ops``, ``knn``, ``cluster`` and ``vbc``.
"""
from .graph_ops import (  # noqa: F401
    OracleInputError, validate, degrees, laplacian, two_hop, theta_sum_q,
    fiedler_value, mu_from_q, operator_a, gershgorin_radii, b_from_radii,
    build_ops, two_hop_components, two_hop_rows, q_diag_rows,
    operator_a_rows,
)
from .solve import (  # noqa: F401
    generalized_eigs, dense_generalized_eigs, sparse_generalized_eigs,
    relative_residuals, b_orthonormality_error, sin_principal_angle_b,
    fix_signs, embed,
)
