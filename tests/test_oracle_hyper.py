"""Pins of the hyperedge form of the oracle (oracle/hyper.py): its conflict
multigraph against graphs built independently (the inputs' conflict graph, the
rook graph), and the doubled weight of a pair in two hyperedges against the
closed form of the K2 step."""
import numpy as np
import pytest

import oracle as O
from oracle import hyper
from paper_2605_05330_amd import inputs


def test_expansion_is_conflict_graph_when_pairs_share_one_hyperedge():
    # two stops per route and many stops: find a seed with no pair in two cliques
    inst = inputs.clique_cover_instance(400, 300, 1, 2, 7)
    rp, ci = hyper.multigraph(inst.n, inst.ptr, inst.members)
    simple = all(len(set(ci[rp[i]:rp[i + 1]].tolist())) == rp[i + 1] - rp[i] for i in range(inst.n))
    assert simple
    assert np.array_equal(rp, inst.graph.row_ptr) and np.array_equal(ci, inst.graph.col_idx)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_rows_and_columns_give_the_rook_graph(N):
    ptr = np.arange(0, 2 * N * N + 1, N)
    members = np.concatenate([np.arange(N * i, N * i + N) for i in range(N)] +
                             [np.arange(j, N * N, N) for j in range(N)])
    rp, ci = hyper.multigraph(N * N, ptr, members)
    g = inputs.rook(N)
    assert np.array_equal(rp, g.row_ptr) and np.array_equal(ci, g.col_idx)


def test_pair_in_two_hyperedges_counts_twice():
    """K2 covered by the same hyperedge twice: x'_0 = y0 / (y0 + 2 gamma y1)."""
    w = np.array([0.64, 0.25])
    x = np.array([0.3, 0.8])
    g = 0.7
    xn, _ = hyper.step(2, np.array([0, 2, 4]), np.array([0, 1, 0, 1]), w, g, x)
    y = np.sqrt(w) * x
    np.testing.assert_allclose(xn, [y[0] / (y[0] + 2 * g * y[1]), y[1] / (y[1] + 2 * g * y[0])], rtol=1e-15)
    once, _ = O.step(2, np.array([0, 1, 2]), np.array([1, 0]), w, 2 * g, x)
    np.testing.assert_allclose(xn, once, rtol=1e-15)


def test_solve_selects_one_per_hyperedge():
    """A solve on a clique cover ends in a set with at most one vertex per
    hyperedge and every other vertex covered."""
    inst = inputs.clique_cover_instance(300, 60, 2, 4, 8)
    w = inputs.weights_uniform01(inst.n, 8)
    r = hyper.solve(inst.n, inst.ptr, inst.members, w, np.full(inst.n, 0.5), max_steps=3000)
    assert r.binarised and r.conflicts == 0 and r.uncovered == 0
    for e in range(inst.m):
        assert r.sel[inst.members[inst.ptr[e]:inst.ptr[e + 1]]].sum() <= 1
