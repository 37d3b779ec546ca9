"""Serving loop (continuous batching) through the C ABI.

Bars: a request's result in the mix is bitwise identical to the same graph
solved alone (a batch of one); results match the CPU FP64 oracle to the
single-solve bars; a failing request is reported on its own; a memory
budget that admits one request at a time still completes every request, in
submission order."""
import numpy as np
import pytest
import torch

import oracle
import synthgraphs as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def me():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2112_07862_amd as pkg
    pkg.load()
    return pkg


def _requests():
    return [
        (sg.manifold_graph("square", 1500, 10, 31), 8),
        (sg.manifold_graph("swiss_roll", 2500, 10, 32), 8),
        (sg.manifold_graph("sphere", 1200, 10, 33), 4),
        (sg.grid(18, 22), 8),            # eps = 0
        (sg.tri_mesh(3), 3),             # dense path
        (sg.manifold_graph("square", 900, 10, 34), 16),
        (sg.manifold_graph("sphere", 3000, 10, 35), 8),
    ]


def _drive(me, reqs, tol, stagger=True, **kw):
    """Submits the requests in waves between steps; returns {ticket: result}."""
    srv = me.Server(**kw)
    out, tickets = {}, []
    waves = [reqs[:2], reqs[2:4], reqs[4:]] if stagger else [reqs]
    order = []
    for w in waves:
        for g, K in w:
            tickets.append(srv.submit(g, K, tol))
        for _ in range(2):
            srv.step()
            for t, X, lam, info in srv.poll():
                out[t] = (X, lam, info)
                order.append(t)
    guard = 0
    while len(out) < len(reqs):
        srv.step()
        for t, X, lam, info in srv.poll():
            out[t] = (X, lam, info)
            order.append(t)
        guard += 1
        assert guard < 10000, "server did not drain"
    srv.close()
    return tickets, out, order


def test_serve_mix_equals_alone(me):
    reqs = _requests()
    print(f"[gpu] serve {len(reqs)} requests", flush=True)
    tickets, out, _ = _drive(me, reqs, 1e-8, seed=4, precision="mixed")
    for (g, K), t in zip(reqs, tickets):
        X, lam, info = out[t]
        assert info["status"] in (0, 2), info
        Xa, la, ia = me.embed_batch([g], [K], tol=1e-8, seed=4, precision="mixed")[0]
        assert ia["iterations"] == info["iterations"], (t, ia["iterations"], info["iterations"])
        assert torch.equal(X, Xa), t
        assert torch.equal(lam, la), t


def test_serve_matches_oracle(me):
    reqs = _requests()[:4]
    tickets, out, _ = _drive(me, reqs, 1e-9, seed=0)
    for (g, K), t in zip(reqs, tickets):
        X, lam, info = out[t]
        ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
        lam_o, V = oracle.generalized_eigs(ops["A"], ops["b"], K)
        scale = np.maximum(np.abs(lam_o[:K]), 1e-8 * ops["A"].diagonal().max())
        assert np.max(np.abs(lam.cpu().numpy() - lam_o[:K]) / scale) <= 1e-6, t
        relgap = (lam_o[K] - lam_o[K - 1]) / max(abs(lam_o[K - 1]), 1e-300)
        if 1e-9 / relgap <= 2.5e-6:
            assert oracle.sin_principal_angle_b(X.cpu().numpy(), V[:, :K], ops["b"]) <= 1e-5, t


def test_serve_budget_one_at_a_time(me):
    """A budget below any request's footprint admits one request at a time:
    all complete, in submission order, with the same results."""
    reqs = _requests()[:4]
    tickets, out, order = _drive(me, reqs, 1e-8, stagger=False, mem_budget=1, seed=4,
                                 precision="mixed")
    assert order == tickets
    _, out2, _ = _drive(me, reqs, 1e-8, seed=4, precision="mixed")
    for t in tickets:
        assert torch.equal(out[t][0], out2[t][0]), t


def test_serve_failing_request_isolated(me):
    good = sg.manifold_graph("square", 700, 8, 41)
    bad = sg.manifold_graph("square", 600, 8, 42)
    val = bad.val.copy()
    val[3] = -1.0  # W_ij <= 0 (and asymmetric)
    bad = sg.CSR(bad.n, bad.rowptr, bad.col, val)
    tickets, out, _ = _drive(me, [(good, 4), (bad, 4), (good, 8)], 1e-8, stagger=False, seed=1)
    st = out[tickets[1]][2]["status_name"]
    assert st in ("ME_ERR_BAD_WEIGHT", "ME_ERR_NOT_SYMMETRIC"), st
    assert out[tickets[1]][0] is None
    a4 = me.embed_batch([good], [4], tol=1e-8, seed=1)[0]
    a8 = me.embed_batch([good], [8], tol=1e-8, seed=1)[0]
    assert torch.equal(out[tickets[0]][0], a4[0]) and torch.equal(out[tickets[2]][0], a8[0])


def test_serve_weight_beyond_fp32_refused_in_mixed(me):
    """A request whose weights exceed FP32's range cannot run the mixed
    preconditioner: it retires with ME_ERR_BAD_WEIGHT and its neighbours
    are served as if alone."""
    good = sg.manifold_graph("square", 700, 8, 41)
    g0 = sg.manifold_graph("square", 600, 8, 42)
    heavy = sg.CSR(g0.n, g0.rowptr, g0.col, g0.val * 1e39)
    tickets, out, _ = _drive(me, [(good, 4), (heavy, 4)], 1e-8, stagger=False, seed=1,
                             precision="mixed")
    assert out[tickets[1]][2]["status_name"] == "ME_ERR_BAD_WEIGHT"
    assert out[tickets[1]][0] is None
    a4 = me.embed_batch([good], [4], tol=1e-8, seed=1, precision="mixed")[0]
    assert torch.equal(out[tickets[0]][0], a4[0])

@pytest.mark.timeout(600)
def test_serve_recipe_mix_with_large_requests_equals_alone(me):
    """Requests drawn from the serving recipe (Poisson stream seed 7: N
    log-uniform in [1000, 200000], square / Swiss roll / sphere, 10-NN, K = 8,
    tol 1e-6), among them requests of more than 1e5 nodes, submitted while
    others run: each result is bitwise the same graph solved alone (a batch
    of one), and each eigenvalue matches the oracle to 1e-6 for the graphs it
    can factor within the test (N <= 30000)."""
    specs = sg.serve_arrivals(40)
    big = [q for q, s in enumerate(specs) if s[2] >= 100_000][:2]
    small = [q for q, s in enumerate(specs) if s[2] < 30_000][:5]
    assert len(big) == 2
    pick = sorted(big + small)
    reqs = [(sg.manifold_graph(specs[q][1], specs[q][2], specs[q][3], specs[q][5]), specs[q][4])
            for q in pick]
    print(f"[gpu] serve recipe: N = {[g.n for g, _ in reqs]}", flush=True)
    tickets, out, _ = _drive(me, reqs, 1e-6, seed=0, precision="mixed")
    for (g, K), t, q in zip(reqs, tickets, pick):
        X, lam, info = out[t]
        assert info["status"] == 0 and info["max_residual"] <= 1e-6, (q, info)
        Xa, la, ia = me.embed_batch([g], [K], tol=1e-6, seed=0, precision="mixed")[0]
        assert ia["iterations"] == info["iterations"], q
        assert torch.equal(X, Xa) and torch.equal(lam, la), q
        if g.n <= 30_000:
            ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
            lam_o, _ = oracle.generalized_eigs(ops["A"], ops["b"], K)
            assert np.max(np.abs(lam.cpu().numpy() - lam_o[:K]) / lam_o[:K]) <= 1e-6, q
