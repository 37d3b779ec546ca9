"""Pins of the betweenness oracle (oracle/vbc.py): closed forms on paths,
stars, cycles and complete graphs, the literal eq. (3) against Brandes'
accumulation on random graphs, and the variance by hand.  CPU only."""
import numpy as np
import pytest

from oracle import vbc as VB
import synthgraphs as sg


def _both(g):
    a = VB.betweenness_definition(g.n, g.rowptr, g.col)
    b = VB.betweenness(g.n, g.rowptr, g.col)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)
    return b


@pytest.mark.parametrize("n", [2, 3, 7, 20])
def test_path(n):
    """P_n: node i lies on the one path of every pair with one end on each
    side: i (n - 1 - i) unordered pairs, twice that ordered."""
    cb = _both(sg.line(n))
    assert cb.tolist() == [2.0 * i * (n - 1 - i) for i in range(n)]


def test_star():
    cb = _both(sg.star(9))
    assert cb[0] == 8 * 7 and np.all(cb[1:] == 0)


@pytest.mark.parametrize("m", [2, 3, 6])
def test_odd_cycle(m):
    """C_{2m+1}: pairs at distance d <= m have one path with d - 1 inner
    nodes: sum_{d=2..m} (d - 1) = m (m - 1) / 2 unordered per node."""
    cb = _both(sg.ring(2 * m + 1))
    np.testing.assert_allclose(cb, m * (m - 1), rtol=1e-15)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_even_cycle(m):
    """C_{2m}: as the odd cycle up to distance m - 1, plus half of each of
    the m - 1 antipodal pairs not containing the node: (m - 1)^2 ordered."""
    cb = _both(sg.ring(2 * m))
    np.testing.assert_allclose(cb, (m - 1) ** 2, rtol=1e-15)


def test_complete_graph():
    assert np.all(_both(sg.complete(8)) == 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_definition_equals_brandes_on_random_graphs(seed):
    g = sg.random_graph(40, 0.08, seed, connect=(seed != 2))  # seed 2: maybe disconnected
    _both(g)


def test_grid_and_disjoint_union():
    _both(sg.grid(5, 6))
    _both(sg.disjoint_union([sg.line(5), sg.ring(7), sg.star(4)]))


def test_variance_by_hand():
    """P_3: C_B = 0, 2, 0, mean 2/3, variance (4/9 + 16/9 + 4/9) / 3 = 8/9."""
    cb = VB.betweenness(3, sg.line(3).rowptr, sg.line(3).col)
    assert VB.vbc(cb) == pytest.approx(8 / 9, rel=1e-15)
