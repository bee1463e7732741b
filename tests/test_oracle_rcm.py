"""Pins of the oracle's self-gated reverse Cuthill-McKee renumbering (the reordering for
cache locality that Sec. 4.2 lists): the result is a permutation; a path with a scrambled
numbering comes back as a path (every entry at index distance 1) and an already banded one is
left alone by the gate; on any graph the reversed order is a Cuthill-McKee order --
breadth first from its start node, each node's children appended by increasing (degree,
index), the start node a fixed point of the George-Liu step -- and a solve on the
renumbered hierarchy returns the caller's solution."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order, shortest_path

import oracle as O
from paper_2606_24791_amd import inputs as I


def scrambled(g, seed):
    p = np.random.default_rng(seed).permutation(g.n).astype(np.int32)
    return O.renumbered(g, p)


def path(n):
    i = np.arange(n - 1)
    return I.from_edges(n, i, i + 1, np.ones(n - 1))


def dist_sum(g, perm):
    inv = np.empty(g.n, np.int64)
    inv[perm] = np.arange(g.n)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return int(np.abs(inv[rows] - inv[g.col_idx]).sum())


def graphs():
    return [scrambled(I.grid2d(13, 8), 1), scrambled(I.random_geometric(600, seed=2), 3),
            I.random_geometric(800, seed=4), I.chung_lu(900, 2.1, 8, seed=5),
            scrambled(path(50), 6)]


@pytest.mark.parametrize("gi", range(5))
def test_result_is_a_permutation_and_the_gate_holds(gi):
    g = graphs()[gi]
    perm, kept = O.rcm(g.row_ptr, g.col_idx)
    assert np.array_equal(np.sort(perm), np.arange(g.n))
    ident = np.arange(g.n, dtype=np.int32)
    if kept:
        assert 2 * dist_sum(g, perm) <= dist_sum(g, ident)
    else:
        assert np.array_equal(perm, ident)


def test_scrambled_path_comes_back_as_a_path():
    g = scrambled(path(200), 11)
    perm, kept = O.rcm(g.row_ptr, g.col_idx)
    assert kept
    assert dist_sum(g, perm) == g.nnz  # every entry at distance 1
    # a path already in order: the renumbering cannot halve anything, the gate keeps it
    g0 = path(200)
    perm0, kept0 = O.rcm(g0.row_ptr, g0.col_idx)
    assert not kept0 and np.array_equal(perm0, np.arange(200))


def cm_properties(g, cm):
    """Checks that cm (one component) is a Cuthill-McKee order of g from cm[0]."""
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    deg = np.diff(g.row_ptr)
    pos = np.empty(g.n, np.int64)
    pos[cm] = np.arange(g.n)
    start = cm[0]
    # breadth first: distances from the start never decrease along the order
    d = shortest_path(A, unweighted=True, indices=start)
    assert np.all(np.diff(d[cm]) >= 0)
    # the parent of v is its earliest-numbered neighbour; parents' positions never decrease,
    # and the children of one parent come by increasing (degree, index)
    parent = np.array([cm[min(pos[g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]])] if v != start else -1
                       for v in range(g.n)])
    par_pos = np.array([pos[parent[v]] for v in cm[1:]])
    assert np.all(np.diff(par_pos) >= 0)
    kids = {}
    for v in cm[1:]:
        kids.setdefault(parent[v], []).append(v)
    for ch in kids.values():
        keys = [(deg[v], v) for v in ch]
        assert keys == sorted(keys)
    # George-Liu fixed point: the least-degree node of the start's last level is no farther
    # from its own farthest node
    last = np.flatnonzero(d == d.max())
    x = min(last, key=lambda u: (deg[u], u))
    assert shortest_path(A, unweighted=True, indices=x).max() <= d.max()
    # and the start was reached from the component's least-degree node by such steps: its
    # eccentricity is at least that node's
    r0 = min(range(g.n), key=lambda u: (deg[u], u))
    assert d.max() >= shortest_path(A, unweighted=True, indices=r0).max()


@pytest.mark.parametrize("gi", [0, 1, 4])
def test_reversed_order_is_cuthill_mckee(gi):
    g = graphs()[gi]
    perm, kept = O.rcm(g.row_ptr, g.col_idx)
    assert kept
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    assert breadth_first_order(A, 0, return_predecessors=False).size == g.n  # connected
    cm_properties(g, perm[::-1].copy())


def test_solve_on_the_renumbered_hierarchy():
    g = scrambled(I.random_geometric(3000, seed=7), 8)
    h = O.Hierarchy(g, reorder=1)
    assert h.perm is not None
    # level 0 is the Laplacian of the renumbered graph
    gr = O.renumbered(g, h.perm)
    rp, ci, v = O.laplacian(gr)
    ex = h.export(0)
    np.testing.assert_array_equal(ex["row_ptr"], rp)
    np.testing.assert_array_equal(ex["col_idx"], ci)
    np.testing.assert_array_equal(ex["val"], v)
    b = I.rhs(g.n, 1, seed=9)[0]
    phi, st, _ = h.solve(b, 1e-8, 100)
    W = sp.csr_matrix((g.weight, g.col_idx, g.row_ptr), shape=(g.n, g.n))
    L = sp.diags(np.asarray(W.sum(1)).ravel()) - W
    bb = b - b.mean()
    assert st["converged"]
    assert np.linalg.norm(bb - L @ phi) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(bb)
    ref = np.linalg.pinv(L.toarray(), hermitian=True) @ bb
    assert np.linalg.norm(phi - ref) <= 1e-6 * np.linalg.norm(ref)
    # a grid in its own numbering: the gate leaves it, and the hierarchy is the default one
    hg = O.Hierarchy(I.grid2d(30, 20), reorder=1)
    assert hg.perm is None
