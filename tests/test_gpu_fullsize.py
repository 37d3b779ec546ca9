"""Parity at full workload sizes, in the configuration bench.py times
(mixed precision, Chebyshev degree 128).

* Swiss roll, N = 1e5, 10-NN, K = 8: the oracle handles the whole graph
  (sparse products and ARPACK shift-invert), so everything is compared:
  T bit-exact, per-node scalars, eps and mu, eigenvalues (relative 1e-6),
  residuals recomputed by the oracle in FP64, X^T B X = I, and the principal
  angle at the tolerance the relative gap requires.
* Sphere, N = 1e6, 12-NN, K = 16: too large for the whole oracle; sampled
  rows are checked against the definitions (T_i, Q_ii, degrees, r_i, and
  (A X - B X Lambda)_i from the row-wise operator), b against the whole r
  vector, X^T B X = I in FP64 on the host; the same for a second solve with
  FP16 Chebyshev iterates."""
import numpy as np
import pytest
import torch

import oracle
import synthgraphs as sg

pytestmark = pytest.mark.gpu

BENCH_OPTS = dict(precision="mixed", cheb_degree=128, seed=0)


@pytest.fixture(scope="module")
def me():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2112_07862_amd as pkg
    pkg.load()
    return pkg


def _np(t):
    return t.detach().cpu().numpy()


def test_swiss_roll_100k_bench_config(me):
    kind, n, knn, K, tol = sg.CONFIGS["swiss_roll_100k"]
    print(f"[gpu] full size {kind} n={n} K={K}", flush=True)
    g = sg.manifold_graph(kind, n, knn, 0)
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    h = me.build_graph_ops(g, **BENCH_OPTS)
    ex = h.export()
    assert np.array_equal(_np(ex["t_rowptr"]), ops["t_rowptr"])
    assert np.array_equal(_np(ex["t_col"]), ops["t_col"])
    assert np.array_equal(_np(ex["t_count"]), ops["t_count"])
    np.testing.assert_allclose(_np(ex["d"]), ops["d"], rtol=1e-13)
    np.testing.assert_allclose(_np(ex["qdiag"]), ops["Q"].diagonal(), rtol=1e-13)
    assert abs(h.eps - ops["eps"]) <= 1e-9 * ops["eps"], (h.eps, ops["eps"])
    assert abs(h.mu - ops["mu"]) <= 1e-9 * ops["mu"]
    np.testing.assert_allclose(_np(ex["b"]), ops["b"], rtol=1e-8)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K, dense_max=0)
    # the bench tolerance
    X, lam, info = me.embed(h, K, tol=tol, **BENCH_OPTS)
    assert info["status"] == 0, info
    lam, X = _np(lam), _np(X)
    assert np.max(np.abs(lam - lam_o[:K]) / lam_o[:K]) <= 1e-6, (lam, lam_o[:K])
    rho = oracle.relative_residuals(ops["A"], ops["b"], X, lam)
    assert rho.max() <= tol * 1.001, rho
    assert oracle.b_orthonormality_error(X, ops["b"]) <= 1e-10
    # the principal-angle bar needs rho <= 1e-5 relgap (sin theta <= rho / relgap)
    relgap = (lam_o[K] - lam_o[K - 1]) / lam_o[K - 1]
    tol2 = min(tol, 1e-5 * relgap / 4)
    X2, lam2, info2 = me.embed(h, K, tol=tol2, **BENCH_OPTS)
    assert info2["status"] == 0, info2
    s = oracle.sin_principal_angle_b(_np(X2), V_o[:, :K], ops["b"])
    print(f"[gpu] relgap {relgap:.3e} tol {tol2:.2e} sin {s:.2e}", flush=True)
    assert s <= 1e-5
    h.close()


def test_sphere_1m_sampled(me):
    kind, n, knn, K, tol = sg.CONFIGS["sphere_1m"]
    print(f"[gpu] full size {kind} n={n} K={K}", flush=True)
    g = sg.manifold_graph(kind, n, knn, 0)
    h = me.build_graph_ops(g, **BENCH_OPTS)
    ex = {k: _np(v) for k, v in h.export().items()}
    rows = np.sort(np.random.default_rng(5).choice(n, 200, replace=False)).tolist()
    t_rows = oracle.two_hop_rows(g.n, g.rowptr, g.col, rows)
    trp, tcol = ex["t_rowptr"], ex["t_col"]
    for i, t in zip(rows, t_rows):
        assert np.array_equal(tcol[trp[i]:trp[i + 1]], t), i
        assert ex["t_count"][i] == t.size
    d = np.add.reduceat(g.val, g.rowptr[:-1])
    np.testing.assert_allclose(ex["d"][rows], d[rows], rtol=1e-13)
    qd = oracle.q_diag_rows(g.n, g.rowptr, g.col, rows)
    np.testing.assert_allclose(ex["qdiag"][rows], qd, rtol=1e-13)
    # r_i = d_i + mu Q_ii; b = r / geometric mean of r (over every node)
    np.testing.assert_allclose(ex["r"][rows], d[rows] + h.mu * qd, rtol=1e-12)
    b = np.exp(np.log(ex["r"]) - np.mean(np.log(ex["r"])))
    np.testing.assert_allclose(ex["b"], b, rtol=1e-9)
    X, lam, info = me.embed(h, K, tol=tol, **BENCH_OPTS)
    print(f"[gpu] sphere iters {info['iterations']} eps iters {info['eps_iterations']}",
          flush=True)
    assert info["status"] == 0 and info["max_residual"] <= tol, info
    X, lam = _np(X), _np(lam)
    assert np.all(np.diff(lam) >= 0)
    G = X.T @ (ex["b"][:, None] * X)
    assert np.abs(G - np.eye(K)).max() <= 1e-10
    _check_sampled_rows(g, h, ex["b"], rows, X, lam, tol)
    # FP16 Chebyshev iterates at full size: the same bars
    X16, lam16, info16 = me.embed(h, K, tol=tol, cheb_iterates="fp16", **BENCH_OPTS)
    print(f"[gpu] sphere fp16 iterates: iters {info16['iterations']}", flush=True)
    assert info16["status"] == 0 and info16["max_residual"] <= tol, info16
    X16, lam16 = _np(X16), _np(lam16)
    assert not np.array_equal(X16, X)
    np.testing.assert_allclose(lam16, lam, rtol=1e-5)
    G16 = X16.T @ (ex["b"][:, None] * X16)
    assert np.abs(G16 - np.eye(K)).max() <= 1e-10
    _check_sampled_rows(g, h, ex["b"], rows, X16, lam16, tol)
    h.close()


def _check_sampled_rows(g, h, b, rows, X, lam, tol):
    """Sampled rows of A X - B X Lambda (the oracle's row-wise operator),
    bounded by the certified norm tol |lambda_j| |B x_j|."""
    AX = oracle.operator_a_rows(g.n, g.rowptr, g.col, g.val, rows, h.mu, h.eps, X)
    R = AX - b[rows, None] * X[rows] * lam[None, :]
    bound = tol * np.abs(lam) * np.linalg.norm(b[:, None] * X, axis=0)
    assert np.all(np.abs(R) <= bound[None, :] * 1.001), np.abs(R).max(axis=0) / bound
