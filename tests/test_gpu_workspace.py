"""Caller-owned device memory through the C ABI: the build, the embedding,
the batch and the server each run inside a workspace the caller allocates
(a uint8 torch tensor), sized by the library's queries.

Bars: the results are bitwise those of the same call with library-allocated
memory (the arithmetic does not depend on where the arrays live); a
workspace one byte short of the
query is ME_ERR_WORKSPACE with the outputs untouched; a server region too
small for one request completes that request with ME_ERR_WORKSPACE and
serves the others."""
import ctypes

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


def _ws(nbytes):
    return torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")


def _same_export(a, b):
    ea, eb = a.export(), b.export()
    for k in ea:
        assert torch.equal(ea[k], eb[k]), k


@pytest.mark.parametrize("name,g,K", [
    ("square_2000", sg.manifold_graph("square", 2000, 8, 0), 4),
    ("swiss_3000", sg.manifold_graph("swiss_roll", 3000, 10, 3), 8),
    ("tri_mesh", sg.tri_mesh(3), 3),         # dense solves (n <= 48)
    ("grid_bipartite", sg.grid(20, 25), 4),  # eps = 0
])
def test_build_and_embed_in_caller_workspace(me, name, g, K):
    print(f"[gpu] workspace build/embed {name} n={g.n} K={K}", flush=True)
    d = me.to_device(g)
    opts = dict(precision="mixed", seed=1)
    need = me.build_workspace_bytes(d, **opts)
    assert need > 0
    ws = _ws(need)
    h_ws = me.build_graph_ops(d, workspace=ws, **opts)
    h = me.build_graph_ops(d, **opts)
    assert h_ws.eps == h.eps and h_ws.mu == h.mu and h_ws.nnz_t == h.nnz_t
    _same_export(h_ws, h)
    lib = me.load()
    eb = int(lib.me_embed_workspace_bytes(h.handle, K, ctypes.byref(me.make_opts(**opts))))
    ews = _ws(eb)
    X1, l1, i1 = me.embed(h_ws, K, tol=1e-8, workspace=ews, **opts)
    X2, l2, i2 = me.embed(h, K, tol=1e-8, **opts)
    assert i1["status"] == i2["status"] and i1["status"] in (0, 2)
    assert i1["iterations"] == i2["iterations"]
    assert torch.equal(X1, X2) and torch.equal(l1, l2)
    # and against the oracle
    ops = oracle.build_ops(g.n, g.rowptr, g.col, g.val)
    lam_o, V_o = oracle.generalized_eigs(ops["A"], ops["b"], K)
    scale = np.maximum(np.abs(lam_o[:K]), 1e-8 * ops["A"].diagonal().max())
    assert np.max(np.abs(l1.cpu().numpy() - lam_o[:K]) / scale) <= 1e-6
    h_ws.close()
    h.close()


def test_workspace_one_byte_short_is_rejected(me):
    g = sg.manifold_graph("square", 1500, 8, 2)
    d = me.to_device(g)
    need = me.build_workspace_bytes(d)
    with pytest.raises(me.MembedError) as e:
        me.build_graph_ops(d, workspace=_ws(need - 1))
    assert e.value.name == "ME_ERR_WORKSPACE"
    h = me.build_graph_ops(d)
    lib = me.load()
    eb = int(lib.me_embed_workspace_bytes(h.handle, 4, None))
    X = torch.full((g.n, 4), 7.0, dtype=torch.float64, device="cuda")
    lam = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    ws = _ws(eb - 1)
    info = me.load().me_embed(h.handle, 4, 1e-8, None, None, ctypes.c_void_p(ws.data_ptr()),
                              eb - 1, ctypes.c_void_p(X.data_ptr()),
                              ctypes.c_void_p(lam.data_ptr()), None, None)
    assert info == -7  # ME_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((X == 7.0).all()) and bool((lam == 7.0).all())  # outputs untouched
    graphs = [g, sg.manifold_graph("torus", 1200, 8, 3)]
    bneed = me.embed_batch_workspace_bytes(graphs, [4, 8])
    with pytest.raises(me.MembedError) as e:
        me.embed_batch(graphs, [4, 8], tol=1e-8, workspace=_ws(bneed - 1))
    assert e.value.name == "ME_ERR_WORKSPACE"
    h.close()


def test_batch_in_caller_workspace_bitwise(me):
    graphs = [sg.manifold_graph("square", 1500, 8, 11), sg.manifold_graph("swiss_roll", 2000, 8, 12),
              sg.manifold_graph("torus", 1200, 8, 13), sg.tri_mesh(3), sg.grid(20, 25),
              sg.disjoint_union([sg.manifold_graph("square", 400, 8, 16),
                                 sg.manifold_graph("square", 300, 8, 17)])]
    Ks = [4, 8, 16, 3, 4, 4]
    print(f"[gpu] workspace batch of {len(graphs)}", flush=True)
    need = me.embed_batch_workspace_bytes(graphs, Ks, precision="mixed")
    ws = _ws(need)
    a = me.embed_batch(graphs, Ks, tol=1e-8, seed=2, precision="mixed", workspace=ws)
    b = me.embed_batch(graphs, Ks, tol=1e-8, seed=2, precision="mixed")
    for q, ((Xa, la, ia), (Xb, lb, ib)) in enumerate(zip(a, b)):
        assert ia["status"] == ib["status"] and ia["status"] in (0, 2), (q, ia)
        assert ia["iterations"] == ib["iterations"], q
        assert torch.equal(Xa, Xb) and torch.equal(la, lb), q


def _serve(me, reqs, tol, **kw):
    srv = me.Server(**kw)
    tickets = [srv.submit(g, K, tol) for g, K in reqs]
    out, guard = {}, 0
    while len(out) < len(reqs):
        srv.step()
        for t, X, lam, info in srv.poll():
            out[t] = (X, lam, info)
        guard += 1
        assert guard < 10000, "server did not drain"
    srv.close()
    return tickets, out


def test_server_in_caller_workspace(me):
    """A server over a caller region: every request equals its batch of one
    bitwise; a region that admits about one request at a time still drains
    in order."""
    reqs = [(sg.manifold_graph("square", 1500, 10, 31), 8),
            (sg.manifold_graph("swiss_roll", 2500, 10, 32), 8),
            (sg.grid(18, 22), 8),
            (sg.tri_mesh(3), 3),
            (sg.manifold_graph("sphere", 8000, 10, 35), 16)]
    print("[gpu] workspace server", flush=True)
    region = _ws(256 << 20)
    tickets, out = _serve(me, reqs, 1e-8, seed=4, precision="mixed", workspace=region)
    for (g, K), t in zip(reqs, tickets):
        X, lam, info = out[t]
        assert info["status"] in (0, 2), info
        Xa, la, ia = me.embed_batch([g], [K], tol=1e-8, seed=4, precision="mixed")[0]
        assert ia["iterations"] == info["iterations"], t
        assert torch.equal(X, Xa) and torch.equal(lam, la), t
    # a region that holds the largest of the first four requests (with the
    # server's tables and work-list areas) but not the last one: that one
    # completes with ME_ERR_WORKSPACE, the others run one or two at a time
    foot = [me.server_request_bytes(g, K) for g, K in reqs]
    size = int(max(foot[:4]) * 1.25) + (4 << 20)
    overhead = 2 * max(size // 128, 256 << 10) + (1 << 20)
    assert size - overhead >= max(foot[:4]) and foot[4] > size, (foot, size)
    small = _ws(size)
    tickets, out = _serve(me, reqs, 1e-8, seed=4, precision="mixed", workspace=small,
                          max_active=4)
    big = out[tickets[4]][2]
    assert big["status_name"] == "ME_ERR_WORKSPACE", big
    for (g, K), t in list(zip(reqs, tickets))[:4]:
        X, lam, info = out[t]
        assert info["status"] in (0, 2), info
        Xa, la, ia = me.embed_batch([g], [K], tol=1e-8, seed=4, precision="mixed")[0]
        assert torch.equal(X, Xa) and torch.equal(lam, la), t
