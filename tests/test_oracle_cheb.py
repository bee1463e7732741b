"""Pins of the oracle's Chebyshev smoother (the polynomial substitute for Gauss-Seidel that
Sec. 5 names, after Adams, Brezina, Hu and Tuminaro 2003): the Gershgorin bound against a
dense eigensolve, the sweep's action on eigenvectors against the closed-form scaled
Chebyshev polynomial, and solves with the option against the pseudo-inverse solution."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2606_24791_amd import inputs as I


def dense(rp, ci, v):
    n = rp.size - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


def test_gershgorin_bounds_the_jacobi_scaled_spectrum():
    for g in (I.grid2d(12, 9), I.random_connected(150, 400, seed=2), I.chung_lu(500, 2.1, 8, seed=3)):
        rp, ci, v = O.laplacian(g)
        L = dense(rp, ci, v)
        d = np.diag(L)
        lam = np.linalg.eigvals(L / d[:, None]).real.max()
        gb = O.gershgorin(rp, ci, v)
        # a graph Laplacian with positive weights: sum_j |L_uj| = 2 L_uu (up to the rounding
        # of the two sums, which run in different orders)
        assert abs(gb - 2.0) <= 4e-15
        assert lam <= gb * (1 + 1e-12)
    # a coarse operator with positive off-diagonals (caliber-2 Galerkin): still an upper bound
    g = I.grid2d(40, 30, 1.0, 1e-2)
    h = O.Hierarchy(g, elimination=False)
    ex = h.export(1)
    L = dense(ex["row_ptr"], ex["col_idx"], ex["val"])
    lam = np.linalg.eigvals(L / np.diag(L)[:, None]).real.max()
    assert lam <= O.gershgorin(ex["row_ptr"], ex["col_idx"], ex["val"]) * (1 + 1e-12)


@pytest.mark.parametrize("degree,ratio", [(1, 5.0), (2, 5.0), (3, 5.0), (3, 30.0)])
def test_sweep_is_the_scaled_chebyshev_polynomial(degree, ratio):
    """On L x = 0 the error after one sweep is p(D^{-1} L) e0 with
    p(t) = T_m((theta - t)/delta) / T_m(theta/delta) on [a, b] = [lmax/ratio, lmax]:
    check it on eigenvectors of D^{-1} L (computed densely)."""
    g = I.random_connected(80, 200, seed=4)
    rp, ci, v = O.laplacian(g)
    L = dense(rp, ci, v)
    d = np.diag(L)
    # D^{-1} L is similar to the symmetric D^{-1/2} L D^{-1/2}
    S = L / np.sqrt(np.outer(d, d))
    lam, Q = np.linalg.eigh(S)
    lmax = 2.0
    b, a = lmax, lmax / ratio
    theta, delta = (a + b) / 2, (b - a) / 2
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    for idx in (1, len(lam) // 3, len(lam) // 2, len(lam) - 1):
        e0 = Q[:, idx] / np.sqrt(d)  # eigenvector of D^{-1} L
        x = O.cheb_sweep(rp, ci, v, lmax, None, e0.copy(), ratio=ratio, degree=degree)
        p = T((theta - lam[idx]) / delta) / T(theta / delta)
        np.testing.assert_allclose(x, p * e0, rtol=0, atol=1e-12 * np.abs(e0).max())


def test_solve_with_chebyshev_on_dense_levels():
    g = I.chung_lu(6000, 2.1, 16, seed=5)
    h = O.Hierarchy(g, smoother=1)
    info = [h.level_info(l) for l in range(h.nlevels)]
    assert any(i["cheb"] for i in info)
    for i in info:
        assert i["cheb"] == (not i["coarsest"] and not i["elim"] and i["ncolors"] > 32)
        if i["cheb"]:
            assert i["cheb_lmax"] >= 2.0 - 1e-14
    b = I.rhs(g.n, 1, seed=6)[0]
    phi, st, _ = h.solve(b, 1e-8, 100)
    L = sp.diags(np.asarray(sp.csr_matrix((g.weight, g.col_idx, g.row_ptr)).sum(1)).ravel()) - \
        sp.csr_matrix((g.weight, g.col_idx, g.row_ptr), shape=(g.n, g.n))
    bb = b - b.mean()
    relres = np.linalg.norm(bb - L @ phi) / np.linalg.norm(bb)
    assert st["converged"] and relres <= 1e-8 * (1 + 1e-6)
    ref = np.linalg.pinv(L.toarray(), hermitian=True) @ bb
    assert np.linalg.norm(phi - ref) <= 1e-6 * np.linalg.norm(ref)
    # the default (Gauss-Seidel everywhere) hierarchy is the same hierarchy
    h0 = O.Hierarchy(g)
    assert h0.nlevels == h.nlevels
    for l in range(h.nlevels):
        assert np.array_equal(h0.export(l)["val"], h.export(l)["val"])
