"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
hand-derived two-hop sets, brute force on tiny graphs, closed forms for
circulant rings, invariants of Q, A, mu and b, and independent library routes
for the eigenpairs.  Runs on the CPU only."""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synthgraphs as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ops_of(g, **kw):
    return oracle.build_ops(g.n, g.rowptr, g.col, g.val, **kw)


def two_hop_sets_bruteforce(g):
    """Pure-Python sets: paths i - k - j of length two, minus N(i), minus i."""
    nbr = [set(g.col[g.rowptr[i]:g.rowptr[i + 1]].tolist()) for i in range(g.n)]
    out = []
    for i in range(g.n):
        s = set()
        for k in nbr[i]:
            s |= nbr[k]
        out.append(sorted(s - nbr[i] - {i}))
    return out


# ---------------------------------------------------------------------------
# T_i (Section 4.1.1)
# ---------------------------------------------------------------------------

def test_tri_mesh_two_hop_matches_hand_derivation():
    g = sg.tri_mesh(3)
    assert g.n == 10 and g.nnz == 36  # 18 undirected edges (Section 5.2)
    idx = {}
    for a in range(4):
        for b in range(4 - a):
            idx[(a, b)] = len(idx)
    want = {}
    with open(os.path.join(GOLDEN, "tri_mesh_two_hop.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            node, rest = line.split(":")
            a, b = map(int, node.split(","))
            want[idx[(a, b)]] = sorted(idx[tuple(map(int, t.split(",")))] for t in rest.split())
    rp, col, cnt = oracle.two_hop(oracle.validate(g.n, g.rowptr, g.col, g.val))
    for i in range(g.n):
        assert col[rp[i]:rp[i + 1]].tolist() == want[i]
    # corners and centre have 3, the six edge nodes 4
    assert sorted(cnt.tolist()) == [3, 3, 3, 3, 4, 4, 4, 4, 4, 4]


@pytest.mark.parametrize("seed", range(6))
def test_two_hop_bruteforce_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    g = sg.random_graph(n, float(rng.uniform(0.03, 0.3)), seed)
    rp, col, cnt = oracle.two_hop(oracle.validate(g.n, g.rowptr, g.col, g.val))
    bf = two_hop_sets_bruteforce(g)
    for i in range(g.n):
        assert col[rp[i]:rp[i + 1]].tolist() == bf[i]
    assert np.array_equal(cnt, [len(s) for s in bf])


def test_two_hop_knn_graph_bruteforce():
    g = sg.manifold_graph("square", 300, 8, 3)
    rp, col, _ = oracle.two_hop(oracle.validate(g.n, g.rowptr, g.col, g.val))
    bf = two_hop_sets_bruteforce(g)
    assert all(col[rp[i]:rp[i + 1]].tolist() == bf[i] for i in range(g.n))


def test_two_hop_rows_match_golden_and_full_pattern():
    """The per-row form (for sampled checks of large graphs) gives the hand-
    derived tri-mesh sets and the same rows as the whole pattern."""
    g = sg.tri_mesh(3)
    rp, col, _ = oracle.two_hop(oracle.validate(g.n, g.rowptr, g.col, g.val))
    rows = oracle.two_hop_rows(g.n, g.rowptr, g.col, range(g.n))
    assert [r.tolist() for r in rows] == [col[rp[i]:rp[i + 1]].tolist() for i in range(g.n)]
    g = sg.manifold_graph("torus", 400, 8, 9)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    sample = [0, 17, 123, 399]
    rows = oracle.two_hop_rows(g.n, g.rowptr, g.col, sample)
    trp, tcol = ops["t_rowptr"], ops["t_col"]
    assert all(r.tolist() == tcol[trp[i]:trp[i + 1]].tolist() for r, i in zip(rows, sample))
    # Q_ii of the per-row form equals the diagonal of the assembled Q
    np.testing.assert_allclose(oracle.q_diag_rows(g.n, g.rowptr, g.col, sample),
                               ops["Q"].diagonal()[sample], rtol=1e-14)


def test_operator_rows_match_assembled_a():
    """Row-wise A X (sampled checks of large graphs) equals the assembled
    sparse A times X on a graph small enough for both."""
    g = sg.manifold_graph("swiss_roll", 500, 10, 4)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    X = np.random.default_rng(0).standard_normal((g.n, 3))
    rows = [0, 5, 250, 499]
    got = oracle.operator_a_rows(g.n, g.rowptr, g.col, g.val, rows, ops["mu"], ops["eps"], X)
    np.testing.assert_allclose(got, (ops["A"] @ X)[rows], rtol=1e-11, atol=1e-12)


def test_two_hop_special_graphs():
    # line of 5 (Fig. 2a): ends and their neighbours have one, the middle two
    ops = ops_of(sg.line(5))
    assert ops["t_count"].tolist() == [1, 1, 2, 1, 1]
    # complete graph: every two-hop node is already a neighbour
    assert ops_of(sg.complete(6))["t_count"].sum() == 0
    # star: the hub has none, each leaf sees every other leaf
    ops = ops_of(sg.star(7))
    assert ops["t_count"].tolist() == [0] + [5] * 6


# ---------------------------------------------------------------------------
# Q (eq. (Q)) and its invariants under reading R1
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: sg.manifold_graph("square", 400, 8, 1),
    lambda: sg.manifold_graph("torus", 400, 8, 2),
    lambda: sg.random_graph(80, 0.08, 5),
    lambda: sg.tri_mesh(4),
])
def test_q_invariants(maker):
    g = maker()
    ops = ops_of(g)
    Q = ops["Q"].toarray()
    n = g.n
    assert np.allclose(Q, Q.T, rtol=0, atol=0)
    assert np.max(np.abs(Q @ np.ones(n))) < 1e-12               # Q 1 = 0 (Laplacian)
    off = Q - np.diag(np.diag(Q))
    assert np.all(off <= 0)                                    # Q_ij <= 0 (Section 4.2)
    W = ops["W"].toarray()
    assert not np.any((W != 0) & (off != 0))                    # L_ij = 0 or Q_ij = 0
    # pattern of Q off the diagonal is exactly T
    T = np.zeros((n, n), bool)
    for i in range(n):
        T[i, ops["t_col"][ops["t_rowptr"][i]:ops["t_rowptr"][i + 1]]] = True
    assert np.array_equal(off != 0, T)
    # quadratic form: x^T Q x = sum_i (1/T_i) sum_{j in T_i} (x_i - x_j)^2
    x = np.random.default_rng(0).standard_normal(n)
    cnt = ops["t_count"]
    direct = 0.0
    for i in range(n):
        for j in ops["t_col"][ops["t_rowptr"][i]:ops["t_rowptr"][i + 1]]:
            direct += (x[i] - x[j]) ** 2 / cnt[i]
    assert abs(x @ Q @ x - direct) < 1e-10 * max(1.0, abs(direct))
    assert np.linalg.eigvalsh(Q)[0] > -1e-10                    # PSD


def test_literal_theta_breaks_psd():
    """The printed Theta_i (1/T_i at (i, i)) gives an indefinite Q on a
    manifold graph, so eps = lambda_2(Q) would not make A PSD (reading R1)."""
    g = sg.manifold_graph("square", 300, 8, 4)
    W = oracle.validate(g.n, g.rowptr, g.col, g.val)
    rp, col, _ = oracle.two_hop(W)
    Ql = oracle.theta_sum_q(g.n, rp, col, reading="literal").toarray()
    assert np.linalg.eigvalsh(Ql)[0] < -0.1
    assert np.max(np.abs(Ql @ np.ones(g.n))) > 0.1


# ---------------------------------------------------------------------------
# Closed forms for circulant rings C_n(1..k) with unit weights, n >= 4k + 1:
# T_i = {i +- (k+1..2k)}, T_i = 2k, q_ij = 1/T_i + 1/T_j = 1/k, and with
# theta_m = 2 pi m / n:
#   lambda_L(theta) = sum_{s=1..k} 2 (1 - cos s theta)
#   lambda_Q(theta) = sum_{s=k+1..2k} (2/k) (1 - cos s theta)
#   eps = min_{m != 0} lambda_Q, den_i = 2 Q_ii = 4, mu = eps / 4,
#   r_i = 2k + mu * 2 (constant) so b = 1, lambda_A = lambda_L - mu lambda_Q + eps.
# ---------------------------------------------------------------------------

def ring_closed_form(n, k):
    th = 2 * math.pi * np.arange(n) / n
    lam_l = sum(2 * (1 - np.cos(s * th)) for s in range(1, k + 1))
    lam_q = sum((2.0 / k) * (1 - np.cos(s * th)) for s in range(k + 1, 2 * k + 1))
    eps = float(np.min(lam_q[1:]))
    mu = eps / 4.0
    lam_a = np.sort(lam_l - mu * lam_q + eps)
    return eps, mu, lam_a


@pytest.mark.parametrize("n,k", [(5, 1), (12, 2), (17, 3), (40, 2), (101, 4)])
def test_ring_closed_forms(n, k):
    eps, mu, lam_a = ring_closed_form(n, k)
    g = sg.ring(n, k)
    ops = ops_of(g)
    assert np.all(ops["t_count"] == 2 * k)
    assert abs(ops["eps"] - eps) < 1e-12 * max(1, eps)
    assert abs(ops["mu"] - mu) < 1e-12 * max(1, mu)
    assert np.allclose(ops["b"], 1.0, rtol=0, atol=1e-14)
    K = min(5, n - 1)
    X, lam, info = oracle.embed(g.n, g.rowptr, g.col, g.val, K)
    assert np.allclose(lam, lam_a[:K], rtol=1e-12, atol=1e-12)
    assert np.allclose(np.sort(np.linalg.eigvalsh(ops["A"].toarray())), lam_a, atol=1e-11)


def test_ring5_printed_values():
    # values of the closed form at n = 5, k = 1 to six digits
    ops = ops_of(sg.ring(5, 1))
    assert round(ops["eps"], 6) == 1.381966
    assert round(ops["mu"], 6) == 0.345492


def test_ring_closed_form_large_uses_sparse_path():
    n, k = 6000, 3
    eps, mu, lam_a = ring_closed_form(n, k)
    g = sg.ring(n, k)
    X, lam, info = oracle.embed(g.n, g.rowptr, g.col, g.val, 5)
    assert abs(info["eps"] - eps) < 1e-9 * eps
    assert np.allclose(lam, lam_a[:5], rtol=1e-9)


# ---------------------------------------------------------------------------
# eps, mu, A, b invariants (Sections 4.2 and 4.3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,n,k,seed", [("square", 500, 8, 0), ("swiss_roll", 600, 10, 1),
                                           ("sphere", 700, 12, 2), ("torus", 500, 8, 3)])
def test_operator_invariants(kind, n, k, seed):
    g = sg.manifold_graph(kind, n, k, seed)
    ops = ops_of(g)
    assert ops["components"] == 1 and ops["eps"] > 0
    Q = ops["Q"].toarray()
    assert abs(ops["eps"] - np.linalg.eigvalsh(Q)[1]) < 1e-12
    A = ops["A"].toarray()
    # A 1 = eps 1 (L 1 = Q 1 = 0)
    assert np.max(np.abs(A @ np.ones(n) - ops["eps"])) < 1e-12
    # Gershgorin left ends >= 0, equal to 0 at the row with the largest denominator
    left = np.diag(A) - (np.abs(A).sum(axis=1) - np.abs(np.diag(A)))
    assert left.min() > -1e-12
    den = np.diag(Q) - (Q.sum(axis=1) - np.diag(Q))
    assert abs(left[np.argmax(den)]) < 1e-12
    assert np.allclose(den, 2 * np.diag(Q))
    # b: prod b = 1 and r_i / b_i constant
    b, r = ops["b"], ops["r"]
    assert abs(np.sum(np.log(b))) < 1e-9
    ratio = r / b
    assert np.ptp(ratio) < 1e-12 * ratio.mean()
    assert np.allclose(r, ops["d"] + ops["mu"] * np.diag(Q), rtol=1e-13)


def test_eps_zero_cases():
    # line graph of 5 nodes (Fig. 2a) is bipartite: its two-hop graph splits
    ops = ops_of(sg.line(5))
    assert ops["components"] == 2 and ops["eps"] == 0.0 and ops["mu"] == 0.0
    # b from degrees (1,2,2,2,1) / 8^(1/5)
    assert np.allclose(ops["b"], np.array([1, 2, 2, 2, 1]) / 8 ** 0.2, rtol=1e-14)
    ops = ops_of(sg.complete(5))
    assert ops["eps"] == 0.0
    ops = ops_of(sg.complete_bipartite(3, 4))
    assert ops["eps"] == 0.0
    # a graph with T_i = 0 somewhere (star hub) also has lambda_2(Q) = 0
    assert ops_of(sg.star(6))["eps"] == 0.0
    # dense check that the value really is 0
    g = sg.grid(4, 5)  # bipartite grid
    ops = ops_of(g)
    assert ops["eps"] == 0.0 and abs(np.linalg.eigvalsh(ops["Q"].toarray())[1]) < 1e-12


# ---------------------------------------------------------------------------
# Eigenpairs (Section 4.3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,n,k,K", [("square", 800, 8, 4), ("sphere", 900, 12, 6),
                                        ("torus", 700, 8, 5)])
def test_eigenpairs_against_generalized_lapack(kind, n, k, K):
    g = sg.manifold_graph(kind, n, k, 11)
    X, lam, info = oracle.embed(g.n, g.rowptr, g.col, g.val, K)
    A, b = info["A"], info["b"]
    # an independent library route: LAPACK generalized symmetric-definite eig
    ref = sla.eigh(A.toarray(), np.diag(b), eigvals_only=True, subset_by_index=[0, K])
    assert np.allclose(lam, ref[:K], rtol=1e-11)
    assert np.all(oracle.relative_residuals(A, b, X, lam) < 1e-10)
    assert oracle.b_orthonormality_error(X, b) < 1e-12
    assert np.all(np.diff(lam) >= 0)
    # Rayleigh quotients v^T A v / v^T B v equal the eigenvalues
    rq = np.einsum("ij,ij->j", X, A @ X) / np.einsum("ij,ij->j", X, b[:, None] * X)
    assert np.allclose(rq, lam, rtol=1e-12)


def test_tiny_brute_force_characteristic_polynomial():
    """For the 10-node mesh, det(A - lambda B) vanishes at each eigenvalue."""
    g = sg.tri_mesh(3)
    X, lam, info = oracle.embed(g.n, g.rowptr, g.col, g.val, 4)
    A = info["A"].toarray()
    B = np.diag(info["b"])
    for l in lam:
        s = sla.svdvals(A - l * B)
        assert s[-1] < 1e-12 * s[0]
    # not a root in between two distinct eigenvalues
    mid = 0.5 * (lam[0] + lam[1])
    s = sla.svdvals(A - mid * B)
    assert s[-1] > 1e-6 * s[0]


def test_dense_and_sparse_paths_agree():
    g = sg.manifold_graph("square", 2500, 8, 7)
    ops = ops_of(g)
    l1, V1 = oracle.dense_generalized_eigs(ops["A"], ops["b"], 4)
    l2, V2 = oracle.sparse_generalized_eigs(ops["A"], ops["b"], 4)
    assert np.allclose(l1, l2, rtol=1e-10)
    assert oracle.sin_principal_angle_b(V1[:, :4], V2[:, :4], ops["b"]) < 1e-8


def test_principal_angle_helper():
    b = np.array([1.0, 4.0])
    # in the B inner product e1 and e2 are orthogonal: angle 90 degrees
    assert abs(oracle.sin_principal_angle_b(np.array([[1.0], [0.0]]),
                                            np.array([[0.0], [1.0]]), b) - 1.0) < 1e-14
    # x = (1, 0) and y = (1, 1)/|.|_B: cos = <x,y>_B / (|x|_B |y|_B) = 1/sqrt(5)
    s = oracle.sin_principal_angle_b(np.array([[1.0], [0.0]]), np.array([[1.0], [1.0]]), b)
    assert abs(s - math.sqrt(1 - 1 / 5)) < 1e-14
    # span is what counts: rotation inside the span gives zero
    rng = np.random.default_rng(0)
    X = rng.standard_normal((30, 3))
    M = rng.standard_normal((3, 3))
    assert oracle.sin_principal_angle_b(X, X @ M, rng.uniform(0.5, 2, 30)) < 1e-12


def test_fix_signs_convention():
    X = np.array([[0.5, -2.0], [-0.7, 2.0], [0.1, 0.0]])
    Y = oracle.fix_signs(X)
    assert Y[1, 0] > 0 and Y[0, 1] > 0   # lowest index wins a tie in magnitude


# ---------------------------------------------------------------------------
# Input validation (Section 3.1)
# ---------------------------------------------------------------------------

def _bad(g, **kw):
    d = dict(n=g.n, rowptr=g.rowptr.copy(), col=g.col.copy(), val=g.val.copy())
    d.update(kw)
    return d


@pytest.mark.parametrize("mutate,code", [
    (lambda g: _bad(g, val=np.where(np.arange(g.nnz) == 0, -1.0, g.val)), "bad_weight"),
    (lambda g: _bad(g, val=np.where(np.arange(g.nnz) == 3, np.nan, g.val)), "bad_weight"),
    (lambda g: _bad(g, val=np.where(np.arange(g.nnz) == 2, 0.5, g.val)), "not_symmetric"),
    (lambda g: _bad(g, col=np.where(np.arange(g.nnz) == 0, 0, g.col).astype(np.int32)), "self_loop"),
    (lambda g: _bad(g, col=np.where(np.arange(g.nnz) == 1, g.n + 3, g.col).astype(np.int32)),
     "invalid_arg"),
])
def test_validation_errors(mutate, code):
    g = sg.random_graph(12, 0.3, 1, wlo=1.0, whi=2.0)
    d = mutate(g)
    with pytest.raises(oracle.OracleInputError) as e:
        oracle.validate(d["n"], d["rowptr"], d["col"], d["val"])
    assert e.value.code == code


def test_isolated_node_rejected():
    g = sg.from_edges(4, np.array([0, 1]), np.array([1, 2]), np.array([1.0, 1.0]))
    with pytest.raises(oracle.OracleInputError) as e:
        oracle.validate(g.n, g.rowptr, g.col, g.val)
    assert e.value.code == "isolated_node"


def test_generators_are_symmetric_and_seeded():
    for kind in ("square", "swiss_roll", "sphere", "torus"):
        g = sg.manifold_graph(kind, 400, 10, 5)
        W = oracle.validate(g.n, g.rowptr, g.col, g.val)
        assert (W - W.T).nnz == 0
        h = sg.manifold_graph(kind, 400, 10, 5)
        assert np.array_equal(g.col, h.col) and np.array_equal(g.val, h.val)
        assert g.degrees_count().min() >= 10


# ---------------------------------------------------------------------------
# Closed forms for periodic lattices (oracle.lattice): every operator of the
# method from the Fourier modes alone, checked against the assembled sparse
# operators and LAPACK on lattices small enough for both.  The two share no
# code: one is trigonometric sums, the other sparse assembly + dense eig.
# ---------------------------------------------------------------------------

from oracle import lattice as LT  # noqa: E402

LATTICES = [("cross", 7, 9), ("king", 9, 11), ("triangular", 8, 10), ("king", 10, 13),
            ("triangular", 11, 7)]


@pytest.mark.parametrize("stencil,n1,n2", LATTICES)
def test_lattice_closed_form_matches_assembled_operators(stencil, n1, n2):
    offs, w = sg.lattice_stencil(stencil)
    g = sg.periodic_lattice(n1, n2, offs, w)
    ops = ops_of(g)
    cf = LT.lattice_spectrum(n1, n2, offs, w)
    assert np.all(ops["t_count"] == cf["t"])
    np.testing.assert_allclose(ops["d"], cf["d"], rtol=1e-15)
    np.testing.assert_allclose(ops["Q"].diagonal(), cf["qdiag"], rtol=1e-15)
    assert abs(ops["eps"] - cf["eps"]) <= 1e-12 * cf["eps"]
    assert abs(ops["mu"] - cf["mu"]) <= 1e-12 * cf["mu"]
    np.testing.assert_allclose(ops["r"], cf["r"], rtol=1e-14)
    np.testing.assert_allclose(ops["b"], 1.0, atol=1e-14)
    # the whole spectrum of A, and of L and Q
    for key, M in (("lam_a", ops["A"]), ("lam_l", ops["L"]), ("lam_q", ops["Q"])):
        dense = np.sort(np.linalg.eigvalsh(M.toarray()))
        np.testing.assert_allclose(dense, np.sort(cf[key]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("stencil,n1,n2", [("king", 9, 11), ("triangular", 8, 10)])
def test_lattice_mode_basis_spans_the_eigenvectors(stencil, n1, n2):
    """For every closed cluster of the smallest eigenvalues, the cos/sin
    basis of the modes spans the oracle's generalized eigenvectors."""
    offs, w = sg.lattice_stencil(stencil)
    g = sg.periodic_lattice(n1, n2, offs, w)
    cf = LT.lattice_spectrum(n1, n2, offs, w)
    lam, modes = LT.smallest(cf, 20)
    ends = [k for k in LT.cluster_ends(lam) if k <= 12]
    assert ends
    X, lam_o, info = oracle.embed(g.n, g.rowptr, g.col, g.val, max(ends))
    np.testing.assert_allclose(lam_o, lam[:max(ends)], rtol=1e-11)
    for k in ends:
        Vb = LT.mode_basis(n1, n2, modes[:k])
        assert Vb.shape[1] == k
        assert oracle.sin_principal_angle_b(X[:, :k], Vb, info["b"]) < 1e-9


def test_lattice_one_dimensional_is_the_ring_closed_form():
    """n2 = 1 with offsets (+-s, 0), s = 1..k is the circulant ring C_n(1..k)."""
    for n, k in [(17, 3), (40, 2), (101, 4)]:
        offs = [(s, 0) for s in range(1, k + 1)] + [(-s, 0) for s in range(1, k + 1)]
        cf = LT.lattice_spectrum(n, 1, offs, [1.0] * (2 * k))
        eps, mu, lam_a = ring_closed_form(n, k)
        assert abs(cf["eps"] - eps) <= 1e-13 * eps and abs(cf["mu"] - mu) <= 1e-13 * mu
        np.testing.assert_allclose(np.sort(cf["lam_a"]), lam_a, rtol=0, atol=1e-12)
        assert cf["t"] == 2 * k


def test_lattice_bipartite_two_hop_graph_gives_eps_zero():
    """The cross stencil on an even x even torus is bipartite: the two-hop
    graph splits into two parity classes, lambda_2(Q) = 0 exactly (reading
    R4), and the closed form says so without rounding."""
    offs, w = sg.lattice_stencil("cross")
    cf = LT.lattice_spectrum(8, 10, offs, w)
    assert cf["eps"] == 0.0 and cf["mu"] == 0.0
    g = sg.periodic_lattice(8, 10, offs, w)
    assert ops_of(g)["eps"] == 0.0


def test_lattice_rejects_wraparound():
    offs, w = sg.lattice_stencil("king")
    with pytest.raises(ValueError):
        LT.lattice_spectrum(4, 9, offs, w)


def test_lattice_headline_size_clusters():
    """The 1250 x 800 king lattice used for the million-node GPU test: the 15
    smallest eigenvalues close a cluster with a relative gap near 0.3, and
    the closed form's eigenvalues are the min-max values (each is a Rayleigh
    quotient of its own mode vector, A applied row-wise by the oracle)."""
    offs, w = sg.lattice_stencil("king")
    cf = LT.lattice_spectrum(1250, 800, offs, w)
    lam, modes = LT.smallest(cf, 17)
    assert 15 in LT.cluster_ends(lam)
    assert (lam[15] - lam[14]) / lam[14] > 0.25
    g = sg.periodic_lattice(1250, 800, offs, w)
    V = LT.mode_basis(1250, 800, modes[:3])
    rows = [0, 1, 799, 800, 123456, 999999]
    AV = oracle.operator_a_rows(g.n, g.rowptr, g.col, g.val, rows, cf["mu"], cf["eps"], V)
    for j in range(3):
        np.testing.assert_allclose(AV[:, j], lam[1] * V[rows, j] if j else lam[0] * V[rows, j],
                                   rtol=1e-9, atol=1e-15)


# ---------------------------------------------------------------------------
# relative_residuals: values worked out by hand for vectors that are NOT
# eigenvectors, so that a wrong denominator (|x| for |Bx|, a dropped |lambda|,
# lambda with its sign, |B^1/2 x|) fails.
# ---------------------------------------------------------------------------

def test_relative_residuals_hand_values():
    import scipy.sparse as sp_
    A = sp_.csr_matrix(np.array([[2.0, -1.0], [-1.0, 2.0]]))
    b = np.array([1.0, 2.0])
    # x = (0, 1), lambda = 3: A x - 3 B x = (-1, 2) - (0, 6) = (-1, -4),
    # |.| = sqrt(17); |lambda| |B x| = 3 * 2 = 6
    # x = (1, 1), lambda = -1: A x + B x = (1, 1) + (1, 2) = (2, 3), |.| = sqrt(13);
    # |lambda| |B x| = 1 * sqrt(5)
    X = np.array([[0.0, 1.0], [1.0, 1.0]])
    rho = oracle.relative_residuals(A, b, X, np.array([3.0, -1.0]))
    np.testing.assert_allclose(rho, [math.sqrt(17) / 6, math.sqrt(13) / math.sqrt(5)],
                               rtol=1e-15)


def test_relative_residuals_line5_hand_value():
    """Line of 5 (Fig. 2a): eps = mu = 0, so A = L; b = (1,2,2,2,1) / 8^(1/5).
    x = e_0, lambda = 1: A x - B x = (1 - b_0, -1, 0, 0, 0),
    rho = sqrt((1 - b_0)^2 + 1) / b_0."""
    g = sg.line(5)
    ops = ops_of(g)
    b0 = 8 ** -0.2
    x = np.zeros((5, 1))
    x[0, 0] = 1.0
    rho = oracle.relative_residuals(ops["A"], ops["b"], x, np.array([1.0]))
    assert abs(rho[0] - math.sqrt((1 - b0) ** 2 + 1) / b0) < 1e-14


# ---------------------------------------------------------------------------
# The products-only ARPACK route (used where an LU does not fit) against the
# shift-invert route and dense LAPACK.
# ---------------------------------------------------------------------------

def test_smallest_route_matches_shift_invert_and_dense():
    g = sg.manifold_graph("sphere", 1500, 12, 3)
    ops = ops_of(g)  # eps by dense eigvalsh at this size
    eps_s = oracle.fiedler_value(ops["Q"], dense_max=0, method="smallest")
    assert abs(eps_s - ops["eps"]) <= 1e-10 * ops["eps"]
    eps_i = oracle.fiedler_value(ops["Q"], dense_max=0)
    assert abs(eps_i - ops["eps"]) <= 1e-10 * ops["eps"]
    l1, V1 = oracle.sparse_generalized_eigs(ops["A"], ops["b"], 8, method="smallest")
    l2, V2 = oracle.sparse_generalized_eigs(ops["A"], ops["b"], 8)
    l3, V3 = oracle.dense_generalized_eigs(ops["A"], ops["b"], 8)
    np.testing.assert_allclose(l1, l3, rtol=1e-10)
    np.testing.assert_allclose(l2, l3, rtol=1e-10)
    assert oracle.sin_principal_angle_b(V1[:, :8], V3[:, :8], ops["b"]) < 1e-7
