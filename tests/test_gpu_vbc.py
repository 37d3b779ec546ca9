"""GPU betweenness centrality and its variance (me_betweenness) against the
CPU oracle (oracle/vbc.py) through the C ABI.

Bars: centralities and the variance agree to relative 1e-12 (path counts are
integers and exact; the accumulated ratios are summed in another order than
the oracle's); closed forms exactly where every term is an integer.  Graphs:
paths, stars, cycles, a grid, random graphs (connected or not), a union of
components, manifold kNN graphs of a few thousand nodes, and one larger
than the 256 sources in flight."""
import numpy as np
import pytest
import torch

from oracle import vbc as VB
import synthgraphs as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def me():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2112_07862_amd as pkg
    pkg.load()
    return pkg


GRAPHS = {
    "path_40": lambda: sg.line(40),
    "star_300": lambda: sg.star(300),
    "ring_301": lambda: sg.ring(301),
    "ring_64": lambda: sg.ring(64),
    "grid_20x30": lambda: sg.grid(20, 30),
    "random_200": lambda: sg.random_graph(200, 0.03, 1),
    "random_disconnected_150": lambda: sg.random_graph(150, 0.01, 2, connect=False),
    "union": lambda: sg.disjoint_union([sg.line(30), sg.ring(41), sg.star(20),
                                        sg.manifold_graph("square", 300, 8, 3)]),
    "square_2000": lambda: sg.manifold_graph("square", 2000, 8, 0),
    "swiss_2500": lambda: sg.manifold_graph("swiss_roll", 2500, 10, 1),
    # the smallest inputs: one node without edges, one edge
    "single": lambda: sg.CSR(1, np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0)),
    "pair": lambda: sg.line(2),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_betweenness_matches_oracle(me, name):
    g = GRAPHS[name]()
    print(f"[gpu] betweenness {name} n={g.n}", flush=True)
    cb, v = me.betweenness(g)
    ref = VB.betweenness(g.n, g.rowptr, g.col)
    np.testing.assert_allclose(cb.cpu().numpy(), ref, rtol=1e-12, atol=1e-9)
    assert v == pytest.approx(VB.vbc(ref), rel=1e-12)


def test_closed_forms_exact(me):
    cb, _ = me.betweenness(sg.line(50))
    assert cb.cpu().tolist() == [2.0 * i * (49 - i) for i in range(50)]
    cb, _ = me.betweenness(sg.star(100))
    assert cb[0].item() == 99 * 98 and bool((cb[1:] == 0).all())


def test_workspace_and_errors(me):
    g = sg.manifold_graph("square", 800, 8, 5)
    need = me.betweenness_workspace_bytes(g.n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    a, va = me.betweenness(g, workspace=ws)
    b, vb = me.betweenness(g)
    assert torch.equal(a, b) and va == vb  # deterministic: no order-dependent sums
    with pytest.raises(me.MembedError) as e:
        me.betweenness(g, workspace=ws[:need - 1])
    assert e.value.name == "ME_ERR_WORKSPACE"
    # one direction of an edge missing
    rp, col, val = g.rowptr.copy(), g.col.copy(), g.val.copy()
    col2 = np.delete(col, rp[0])
    val2 = np.delete(val, rp[0])
    rp2 = rp.copy()
    rp2[1:] -= 1
    with pytest.raises(me.MembedError) as e:
        me.betweenness(sg.CSR(g.n, rp2, col2, val2))
    assert e.value.name == "ME_ERR_NOT_SYMMETRIC"
