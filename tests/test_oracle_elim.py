"""Pins of the oracle's low-degree elimination (Sec. 2, "Low-degree elimination",
eq. (2.1)): the elimination set by brute force, the Schur complement against properties
that do not restate its formula (effective resistances between kept nodes are preserved,
the eliminated system's solution restricted to C, a closed form), and the cycle with an
elimination level (exact two-level solve, convergence with a multilevel hierarchy)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2606_24791_amd import inputs as I


def dense(rp, ci, v):
    n = rp.size - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


def small_graphs():
    return [
        I.grid2d(9, 7),
        I.grid2d(12, 5, 1.0, 1e-2),
        I.random_connected(120, 200, seed=3),
        I.random_connected(90, 400, seed=4),
        I.chung_lu(400, 2.1, 6, seed=5),
    ]


@pytest.mark.parametrize("gi", range(5))
def test_elimination_set_is_a_maximal_independent_set_of_low_degree_nodes(gi):
    g = small_graphs()[gi]
    rp, ci, v = O.laplacian(g)
    cid, nc = O.elim_select(rp, ci, v)
    n = g.n
    F = cid < 0
    deg = np.diff(rp) - 1
    A = dense(rp, ci, v) != 0
    np.fill_diagonal(A, False)
    assert np.all(deg[F] <= 4)
    assert not np.any(A[np.ix_(F, F)])  # independent
    for u in np.nonzero(~F & (deg <= 4))[0]:  # maximal among the candidates
        assert A[u, F].any(), u
    # C numbered by ascending fine index
    assert np.array_equal(cid[~F], np.arange(nc)) and nc == n - F.sum()
    # brute force: the greedy natural-order rule itself
    inF = np.zeros(n, bool)
    for u in range(n):
        if deg[u] <= 4 and not inF[A[u]].any():
            inF[u] = True
    assert np.array_equal(inF, F)


def test_elimination_set_empty_when_no_node_qualifies():
    g = I.grid3d(4, 4, 4)  # interior degree 6; corners 3, edges 4, faces 5
    rp, ci, v = O.laplacian(g)
    cid, nc = O.elim_select(rp, ci, v, dmax=2)
    assert nc == g.n and np.array_equal(cid, np.arange(g.n))


def test_schur_four_cycle_closed_form():
    """Unit 4-cycle 0-1-2-3: F = {0, 2}; the two kept nodes see two parallel paths of
    two unit edges each, an effective conductance of 1."""
    rp = np.array([0, 2, 4, 6, 8], np.int32)
    ci = np.array([1, 3, 0, 2, 1, 3, 0, 2], np.int32)
    g = I.Graph(4, rp, ci, np.ones(8), name="c4")
    Lrp, Lci, Lv = O.laplacian(g)
    cid, nc = O.elim_select(Lrp, Lci, Lv)
    assert list(cid) == [-1, 0, -1, 1]
    Crp, Cci, Cv = O.schur(Lrp, Lci, Lv, cid, nc)
    assert np.array_equal(dense(Crp, Cci, Cv), np.array([[1.0, -1.0], [-1.0, 1.0]]))


@pytest.mark.parametrize("gi", range(5))
def test_schur_preserves_effective_resistances_and_solutions(gi):
    g = small_graphs()[gi]
    rp, ci, v = O.laplacian(g)
    cid, nc = O.elim_select(rp, ci, v)
    Crp, Cci, Cv = O.schur(rp, ci, v, cid, nc)
    L = dense(rp, ci, v)
    Lc = dense(Crp, Cci, Cv)
    C = np.nonzero(cid >= 0)[0]
    F = np.nonzero(cid < 0)[0]
    # canonical form: ascending columns with the diagonal, exact symmetry, zero row sums
    for a in range(nc):
        cols = Cci[Crp[a]:Crp[a + 1]]
        assert np.all(np.diff(cols) > 0) and a in cols
    assert np.array_equal(Lc, Lc.T)
    assert np.all(np.abs(Lc.sum(1)) <= 1e-13 * np.abs(Lc).max())
    assert np.all(Lc[~np.eye(nc, dtype=bool)] <= 0)
    # Kron reduction keeps the effective resistance between any two kept nodes
    Lp = np.linalg.pinv(L, hermitian=True)
    Lcp = np.linalg.pinv(Lc, hermitian=True)
    rng = np.random.default_rng(gi)
    for _ in range(30):
        a, b = rng.choice(nc, 2, replace=False)
        r_f = Lp[C[a], C[a]] + Lp[C[b], C[b]] - 2 * Lp[C[a], C[b]]
        r_c = Lcp[a, a] + Lcp[b, b] - 2 * Lcp[a, b]
        assert r_c == pytest.approx(r_f, rel=1e-9)
    # the fine solution restricted to C solves the eliminated system with
    # b_c = b_C + sum over f of (w_fc / d_f) b_f
    b = rng.standard_normal(g.n)
    b -= b.mean()
    phi = Lp @ b
    bc = b[C].copy()
    for f in F:
        for j in range(rp[f], rp[f + 1]):
            t = ci[j]
            if t != f:
                bc[cid[t]] += (-v[j] / L[f, f]) * b[f]
    np.testing.assert_allclose(Lc @ phi[C], bc, atol=1e-9 * np.abs(bc).max())
    # pattern: kept edges plus fill between the neighbours of each eliminated node
    pat = L[np.ix_(C, C)] != 0
    for f in F:
        nb = [cid[t] for t in ci[rp[f]:rp[f + 1]] if t != f]
        for x in nb:
            for y in nb:
                pat[x, y] = True
    np.fill_diagonal(pat, True)
    assert np.array_equal(pat, Lc != 0)


def test_schur_matches_dense_reduction_with_mixed_weights():
    """Weights 1 and 2 in a grid: the canonical Schur CSR equals the dense reduction."""
    g = I.grid2d(6, 6)
    w = np.where(np.arange(g.nnz) % 3 == 0, 2.0, 1.0)
    # symmetric weights: take the larger of the two directions
    A = sp.csr_matrix((w, g.col_idx, g.row_ptr), shape=(g.n, g.n))
    A = A.maximum(A.T).tocsr()
    A.sort_indices()
    g2 = I.Graph(g.n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data, name="w")
    rp, ci, v = O.laplacian(g2)
    cid, nc = O.elim_select(rp, ci, v)
    Crp, Cci, Cv = O.schur(rp, ci, v, cid, nc)
    L = dense(rp, ci, v)
    C, F = cid >= 0, cid < 0
    d = np.diag(L)[F]
    ref = L[np.ix_(C, C)] - L[np.ix_(C, F)] @ np.diag(1.0 / d) @ L[np.ix_(F, C)]
    assert np.max(np.abs(dense(Crp, Cci, Cv) - ref)) <= 1e-12


def test_two_level_elimination_with_direct_coarse_is_exact():
    """Elimination onto a directly solved level: one cycle solves the system."""
    g = I.grid2d(30, 20)
    h = O.Hierarchy(g, elimination=True)
    assert h.nlevels == 2 and h.level_info(0)["elim"] and h.level_info(1)["coarsest"]
    b = I.rhs(g.n, 1, seed=2)[0]
    phi, st, _ = h.solve(b, 1e-12, 3)
    assert st["cycles"] == 1 and st["relres"] <= 1e-13
    L = dense(*O.laplacian(g))
    ref = np.linalg.pinv(L, hermitian=True) @ (b - b.mean())
    np.testing.assert_allclose(phi, ref - ref.mean(), atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("gen", [
    lambda: I.grid2d(40, 36, 1.0, 1e-3),
    lambda: I.chung_lu(3000, 2.1, 8, seed=5),
    lambda: I.random_connected(2000, 2600, seed=9),
])
def test_solve_with_elimination_levels(gen):
    g = gen()
    h = O.Hierarchy(g, elimination=True)
    info = [h.level_info(l) for l in range(h.nlevels)]
    assert any(i["elim"] for i in info)
    for l in range(h.nlevels - 1):
        if info[l]["elim"]:
            assert info[l]["gamma"] == 1.0 and not info[l + 1]["elim"]  # alternation
            ex = h.export(l)
            assert (ex["agg"] < 0).sum() >= 0.1 * info[l]["n"]
            assert info[l + 1]["n"] == info[l]["nc"]
    b = I.rhs(g.n, 1, seed=6)[0]
    phi, st, hist = h.solve(b, 1e-8, 100)
    L = dense(*O.laplacian(g))
    bb = b - b.mean()
    relres = np.linalg.norm(bb - L @ phi) / np.linalg.norm(bb)
    assert st["converged"] and relres <= 1e-8 * (1 + 1e-6)
    assert abs(relres - st["relres"]) <= 1e-12
    ref = np.linalg.pinv(L, hermitian=True) @ bb
    lam2 = np.linalg.eigvalsh(L)[1]
    assert np.linalg.norm(phi - ref) <= 1.01 * relres * np.linalg.norm(bb) / lam2


def test_elimination_skipped_below_a_tenth_leaves_hierarchy_unchanged():
    """A 3D grid has too few nodes of degree <= 4 for an elimination level: the hierarchy
    is the aggregation-only one, bit for bit."""
    g = I.grid3d(14, 12, 11, "lognormal", seed=2)
    a, b = O.Hierarchy(g), O.Hierarchy(g, elimination=False)
    assert a.nlevels == b.nlevels
    for l in range(a.nlevels):
        ea, eb = a.export(l), b.export(l)
        assert not ea["elim"] and np.array_equal(ea["val"], eb["val"])
