"""Pins of the oracle's block-Jacobi Gauss-Seidel smoother (the substitute for Gauss-Seidel
that Sec. 5 names beside polynomial smoothers, with the coupling between blocks frozen):
one sweep against triangular solves done by scipy -- a single block is the natural-order
forward Gauss-Seidel sweep, blocks of one row are a Jacobi sweep, any block size the solve
with the block-lower part of L -- and solves with the option against the pseudo-inverse
solution."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

import oracle as O
from paper_2606_24791_amd import inputs as I


def csr(rp, ci, v):
    n = rp.size - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def block_lower(L, bs):
    """D plus the entries below the diagonal whose row and column share a block of bs."""
    C = L.tocoo()
    keep = (C.row == C.col) | ((C.col < C.row) & (C.row // bs == C.col // bs))
    return sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=L.shape)


def graphs():
    return [I.grid2d(11, 9), I.random_connected(120, 300, seed=2),
            I.chung_lu(700, 2.1, 8, seed=3)]


@pytest.mark.parametrize("gi", range(3))
def test_one_block_is_the_forward_gauss_seidel_sweep(gi):
    g = graphs()[gi]
    rp, ci, v = O.laplacian(g)
    L = csr(rp, ci, v)
    rng = np.random.default_rng(gi)
    x, f = rng.standard_normal(g.n), rng.standard_normal(g.n)
    got = O.bjgs_sweep(rp, ci, v, g.n, f, x.copy())
    M = sp.tril(L, 0, format="csr")
    want = spsolve_triangular(M, f - (L - M) @ x, lower=True)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    # a block wider than the level is the same sweep
    np.testing.assert_array_equal(O.bjgs_sweep(rp, ci, v, 10 * g.n, f, x.copy()), got)


@pytest.mark.parametrize("gi", range(3))
def test_blocks_of_one_row_are_a_jacobi_sweep(gi):
    g = graphs()[gi]
    rp, ci, v = O.laplacian(g)
    L = csr(rp, ci, v)
    d = L.diagonal()
    rng = np.random.default_rng(10 + gi)
    x, f = rng.standard_normal(g.n), rng.standard_normal(g.n)
    got = O.bjgs_sweep(rp, ci, v, 1, f, x.copy())
    want = (f - (L - sp.diags(d)) @ x) / d
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("bs", [2, 7, 16, 33])
def test_any_block_size_is_the_block_lower_triangular_solve(bs):
    """Blocks of bs rows (the last one ragged): the in-block entries below the diagonal use
    the new values, every other entry the values at the start of the sweep."""
    for gi, g in enumerate(graphs()):
        rp, ci, v = O.laplacian(g)
        L = csr(rp, ci, v)
        rng = np.random.default_rng(100 * bs + gi)
        x, f = rng.standard_normal(g.n), rng.standard_normal(g.n)
        got = O.bjgs_sweep(rp, ci, v, bs, f, x.copy())
        M = block_lower(L, bs)
        want = spsolve_triangular(M, f - (L - M) @ x, lower=True)
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-12 * np.abs(want).max())
        # f = None is f = 0
        np.testing.assert_array_equal(O.bjgs_sweep(rp, ci, v, bs, None, x.copy()),
                                      O.bjgs_sweep(rp, ci, v, bs, np.zeros(g.n), x.copy()))


def test_solve_with_block_jacobi_on_dense_levels():
    g = I.chung_lu(6000, 2.1, 16, seed=5)
    h = O.Hierarchy(g, smoother=2)
    info = [h.level_info(l) for l in range(h.nlevels)]
    assert any(i["bjgs"] for i in info)
    for i in info:
        assert i["bjgs"] == (not i["coarsest"] and not i["elim"] and i["ncolors"] > 32)
        assert not i["cheb"]
    b = I.rhs(g.n, 1, seed=6)[0]
    phi, st, _ = h.solve(b, 1e-8, 100)
    W = sp.csr_matrix((g.weight, g.col_idx, g.row_ptr), shape=(g.n, g.n))
    L = sp.diags(np.asarray(W.sum(1)).ravel()) - W
    bb = b - b.mean()
    relres = np.linalg.norm(bb - L @ phi) / np.linalg.norm(bb)
    assert st["converged"] and relres <= 1e-8 * (1 + 1e-6)
    ref = np.linalg.pinv(L.toarray(), hermitian=True) @ bb
    assert np.linalg.norm(phi - ref) <= 1e-6 * np.linalg.norm(ref)
    # the smoother changes no level of the hierarchy
    h0 = O.Hierarchy(g)
    assert h0.nlevels == h.nlevels
    for l in range(h.nlevels):
        a, c = h.export(l), h0.export(l)
        np.testing.assert_array_equal(a["row_ptr"], c["row_ptr"])
        np.testing.assert_array_equal(a["col_idx"], c["col_idx"])
        np.testing.assert_array_equal(a["val"], c["val"])
    # a block spanning every level is Gauss-Seidel in natural order, which converges too
    h.set_bj_block(1 << 30)
    phi2, st2, _ = h.solve(b, 1e-8, 100)
    assert st2["converged"]
