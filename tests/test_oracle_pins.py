"""Pins of the CPU oracle's setup steps against facts fixed by the paper and by
mathematics (closed forms, brute force, library routines, published values).

None of these tests re-types an oracle formula: each compares the oracle with an
independent route to the same quantity.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.optimize import minimize_scalar

import oracle as O
from paper_2606_24791_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_L(rp, ci, v):
    n = rp.size - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


def dense_W(g):
    return sp.csr_matrix((g.weight, g.col_idx, g.row_ptr), shape=(g.n, g.n)).toarray()


# --- counter-based RNG --------------------------------------------------------

def test_splitmix64_known_answers():
    """Published SplitMix64 reference sequences."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for row in rows:
        seed, outs = int(row[0]), [int(x) for x in row[1:]]
        assert [O.splitmix64(seed, i) for i in range(len(outs))] == outs


def test_tv_start_uniform():
    """Start values lie in [-1, 1), on the 2^-52 lattice, with mean ~0 and var ~1/3."""
    vals = np.array([O.tv_start(7, 0, k, u) for k in range(4) for u in range(2000)])
    assert vals.min() >= -1.0 and vals.max() < 1.0
    assert np.all(np.ldexp(vals + 1.0, 52) == np.round(np.ldexp(vals + 1.0, 52)))
    assert abs(vals.mean()) < 0.03 and abs(vals.var() - 1.0 / 3.0) < 0.02
    assert np.unique(vals).size == vals.size
    # level and vector index change the stream
    assert O.tv_start(7, 1, 0, 5) != O.tv_start(7, 0, 0, 5) != O.tv_start(7, 0, 1, 5)


# --- Laplacian (Sec. 1) -------------------------------------------------------

def test_laplacian_is_D_minus_W():
    g = I.random_connected(300, 900, seed=3)
    rp, ci, v = O.laplacian(g)
    W = dense_W(g)
    np.testing.assert_allclose(dense_L(rp, ci, v), np.diag(W.sum(1)) - W, rtol=0, atol=1e-12)
    for u in range(g.n):  # canonical: ascending columns, diagonal in place
        assert np.all(np.diff(ci[rp[u]:rp[u + 1]]) > 0) and u in ci[rp[u]:rp[u + 1]]


def test_laplacian_integer_weights_zero_rowsum_exact():
    rng = np.random.default_rng(4)
    base = I.random_connected(200, 600, seed=4)
    rows = np.repeat(np.arange(base.n), np.diff(base.row_ptr))
    up = rows < base.col_idx
    g = I.from_edges(base.n, rows[up], base.col_idx[up], rng.integers(1, 9, up.sum()).astype(float))
    rp, ci, v = O.laplacian(g)
    Ld = dense_L(rp, ci, v)
    assert np.all(Ld.sum(1) == 0.0)
    assert np.all(Ld == Ld.T)


# --- colouring (natural-order greedy) ------------------------------------------

def test_color_grid_parity():
    for g, shape in [(I.grid2d(17, 11), (11, 17)), (I.grid3d(6, 5, 7), (7, 5, 6))]:
        rp, ci, v = O.laplacian(g)
        col, nc = O.color(rp, ci)
        idx = np.indices(shape).sum(0).ravel() % 2
        assert nc == 2
        assert np.array_equal(col, idx)


def test_color_valid_and_greedy_bruteforce():
    g = I.random_connected(400, 2000, seed=5)
    rp, ci, v = O.laplacian(g)
    col, nc = O.color(rp, ci)
    ref = np.zeros(g.n, int)
    for u in range(g.n):
        nbr = {int(ref[t]) for t in ci[rp[u]:rp[u + 1]] if t < u}
        c = 0
        while c in nbr:
            c += 1
        ref[u] = c
    assert np.array_equal(col, ref) and nc == ref.max() + 1
    for u in range(g.n):
        for t in ci[rp[u]:rp[u + 1]]:
            assert t == u or col[t] != col[u]


# --- strength-of-connection veto (eq. (3.1)) -----------------------------------

def test_veto_grid_aligned_anisotropy():
    g = I.grid2d(20, 15, 1.0, 1e-3)
    rp, ci, v = O.laplacian(g)
    s = O.strong(rp, ci, v)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    dx = np.abs(ci - rows)
    assert np.all(s[dx == 1])  # x-neighbours (weight 1) kept
    assert not np.any(s[dx == 20])  # y-neighbours (1e-3 < 0.05) vetoed
    assert not np.any(s[dx == 0])  # diagonal never strong
    # veto disabled: only the diagonal is excluded
    s2 = O.strong(rp, ci, v, enable_veto=False)
    assert np.array_equal(s2, dx != 0)


def test_veto_bruteforce_random_weights():
    g = I.random_connected(300, 1500, seed=6, wmin=1e-3, wmax=1.0)
    rp, ci, v = O.laplacian(g)
    s = O.strong(rp, ci, v)
    for u in range(g.n):
        nb = [(t, -v[j]) for j, t in zip(range(rp[u], rp[u + 1]), ci[rp[u]:rp[u + 1]]) if t != u]
        mx = max(w for _, w in nb)
        got = {int(t) for j, t in zip(range(rp[u], rp[u + 1]), ci[rp[u]:rp[u + 1]]) if s[j]}
        assert got == {int(t) for t, w in nb if w >= 0.05 * mx}


# --- Gauss-Seidel (Sec. 2, "Relaxation") ---------------------------------------

def test_multicolor_gs_equals_forward_gs_on_colour_sorted_matrix():
    """A multicolour sweep is a forward GS sweep of the matrix permuted by colour:
    x_new = (D + L_lower)^{-1} (f - U x_old) -- solved with a triangular solve."""
    g = I.random_connected(250, 1000, seed=7)
    rp, ci, v = O.laplacian(g)
    col, nc = O.color(rp, ci)
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal(g.n)
    f = rng.standard_normal(g.n)
    x = O.gs_sweep(rp, ci, v, col, nc, x0.copy(), f)
    perm = np.lexsort((np.arange(g.n), col))
    A = dense_L(rp, ci, v)[np.ix_(perm, perm)]
    low = np.tril(A)
    up = np.triu(A, 1)
    xp = sla.solve_triangular(low, f[perm] - up @ x0[perm], lower=True)
    np.testing.assert_allclose(x[perm], xp, rtol=1e-12, atol=1e-12)


def test_test_vectors_are_three_sweeps_from_rng_start():
    g = I.grid2d(12, 9, 1.0, 0.3)
    rp, ci, v = O.laplacian(g)
    col, nc = O.color(rp, ci)
    X = O.test_vectors(rp, ci, v, col, nc, seed=11, level=2, sweeps=3)
    perm = np.lexsort((np.arange(g.n), col))
    A = dense_L(rp, ci, v)[np.ix_(perm, perm)]
    low, up = np.tril(A), np.triu(A, 1)
    for k in range(4):
        x = np.array([O.tv_start(11, 2, k, u) for u in range(g.n)])[perm]
        for _ in range(3):
            x = sla.solve_triangular(low, -up @ x, lower=True)
        np.testing.assert_allclose(X[perm, k], x, rtol=1e-12, atol=1e-14)


# --- affinity (eq. (2.2)) ------------------------------------------------------

def test_affinity_is_squared_cosine():
    g = I.grid2d(3, 1)  # path 0-1-2
    rp, ci, v = O.laplacian(g)
    t = 0.7
    X = np.array([[1.0, 0, 0, 0], [np.cos(t), np.sin(t), 0, 0], [0, 0, 3.0, 0]])
    a = O.affinity(rp, ci, X)

    def aff(u, w):
        j = rp[u] + list(ci[rp[u]:rp[u + 1]]).index(w)
        return a[j]

    assert aff(0, 1) == pytest.approx(np.cos(t) ** 2, abs=1e-15)
    assert aff(1, 0) == aff(0, 1)
    assert aff(1, 2) == 0.0  # orthogonal profiles
    X2 = np.array([[1.0, -2, 3, 0.5], [-2.0, 4, -6, -1], [1.0, 1, 1, 1]])
    a2 = O.affinity(rp, ci, X2)
    assert a2[rp[0] + 1] == pytest.approx(1.0, abs=1e-15)  # proportional profiles
    # diagonal entries carry 0
    assert all(a2[rp[u] + list(ci[rp[u]:rp[u + 1]]).index(u)] == 0 for u in range(3))


def test_affinity_range_and_symmetry_random():
    g = I.random_connected(200, 800, seed=8)
    rp, ci, v = O.laplacian(g)
    X = np.random.default_rng(1).standard_normal((g.n, 4))
    a = O.affinity(rp, ci, X)
    assert a.min() >= 0 and a.max() <= 1.0 + 1e-15
    M = sp.csr_matrix((a, ci, rp), shape=(g.n, g.n))
    assert abs(M - M.T).max() == 0.0


# --- guard and moments (eq. (2.3), App. B) -------------------------------------

def nodal_energy(ws, xs, y):
    """u's share of the energy, 1/2 sum_v w_uv (y - x_v)^2, summed edge by edge."""
    return 0.5 * sum(w * (y - x) ** 2 for w, x in zip(ws, xs))


def test_moment_closed_forms_match_bruteforce_energy():
    g = I.random_connected(120, 500, seed=9)
    rp, ci, v = O.laplacian(g)
    X = np.random.default_rng(2).standard_normal((g.n, 4))
    mom = O.moments(rp, ci, v, X)
    for u in range(0, g.n, 7):
        nb = [(int(t), -v[j]) for j, t in zip(range(rp[u], rp[u + 1]), ci[rp[u]:rp[u + 1]]) if t != u]
        ws = [w for _, w in nb]
        for s, _ in nb[:3]:
            ok, ef, em = O.guard(mom[u], X[s])
            for k in range(4):
                xk = [X[t, k] for t, _ in nb]
                emin = minimize_scalar(lambda y: nodal_energy(ws, xk, y), tol=1e-12).fun
                assert em[k] / 2 == pytest.approx(emin, rel=1e-7, abs=1e-12)
                assert ef[k] / 2 == pytest.approx(nodal_energy(ws, xk, X[s, k]), rel=1e-12, abs=1e-13)
            q = max(ef[k] / em[k] for k in range(4))
            assert ok == (q <= 2.5)


def test_guard_linear_chain_ratio_is_two():
    """On a 1-D chain with a linear test vector, forcing u onto a neighbour doubles its
    energy: q = 2, admissible under Q = 2.5 and not under Q = 1.9."""
    g = I.grid2d(5, 1)
    rp, ci, v = O.laplacian(g)
    X = np.tile(np.arange(5.0)[:, None] * 0.3, (1, 4)) + np.array([0.0, 1.0, -2.0, 5.0])
    mom = O.moments(rp, ci, v, X)
    ok, ef, em = O.guard(mom[2], X[3])
    np.testing.assert_allclose(ef / em, 2.0, rtol=1e-12)
    assert ok
    assert not O.guard(mom[2], X[3], Q=1.9)[0]


# --- aggregation (Sec. 2; Sec. 3.1) ---------------------------------------------

def replay_check(rp, ci, strong, aff, X, mom, seed, agg, Q=2.5):
    n = rp.size - 1
    is_seed = seed == np.arange(n)
    # coarse ids: seeds in ascending order
    assert np.array_equal(agg[is_seed], np.arange(is_seed.sum()))
    assert np.all(is_seed[seed])  # every aggregate is rooted at a seed
    assert np.array_equal(agg, agg[seed])
    first_joiner = np.full(n, n, dtype=np.int64)
    for u in np.nonzero(~is_seed)[0]:
        first_joiner[seed[u]] = min(first_joiner[seed[u]], u)

    def available(u, t):  # state of t at u's turn: undecided or a seed
        return t > u or is_seed[t]

    def candidates(u):
        out = []
        for j in range(rp[u], rp[u + 1]):
            t = ci[j]
            if strong[j] and t != u and available(u, t) and O.guard(mom[u], X[t], Q)[0]:
                out.append((aff[j], t))
        return out

    for u in range(n):
        if not is_seed[u]:
            s = seed[u]
            j = rp[u] + list(ci[rp[u]:rp[u + 1]]).index(s)
            assert strong[j] and O.guard(mom[u], X[s], Q)[0]
            cands = candidates(u)
            best = max(c for c, _ in cands)
            assert aff[j] == best
            assert s == min(t for c, t in cands if c == best)
        elif first_joiner[u] > u:
            # nobody before u chose it, so u was undecided at its own turn and
            # became a singleton seed: it had no admissible candidate
            assert candidates(u) == []


@pytest.mark.parametrize("gen", [
    lambda: I.grid2d(24, 20),
    lambda: I.grid2d(24, 20, 1.0, 1e-3),
    lambda: I.random_connected(500, 2000, seed=10),
    lambda: I.chung_lu(3000, 2.1, 16, seed=1),
])
def test_aggregation_replay_invariants(gen):
    g = gen()
    rp, ci, v = O.laplacian(g)
    col, nc = O.color(rp, ci)
    s = O.strong(rp, ci, v)
    X = O.test_vectors(rp, ci, v, col, nc, seed=1, level=0)
    a = O.affinity(rp, ci, X)
    m = O.moments(rp, ci, v, X)
    seed, agg, ncoarse = O.aggregate(rp, ci, s, a, X, m)
    assert 0 < ncoarse < g.n
    replay_check(rp, ci, s, a, X, m, seed, agg)


# --- caliber-2 weight (eq. (A.7)) -------------------------------------------------

def test_caliber2_weight_closed_forms():
    xa = np.array([1.0, 2.0, 3.0, 4.0])
    xb = np.array([3.0, 2.0, 1.0, 0.0])
    assert O.caliber2_weight((xa + xb) / 2, xa, xb) == 0.5
    assert O.caliber2_weight(xa, xa, xb) == 1.0
    assert O.caliber2_weight(xb, xa, xb) == 0.0
    assert np.isnan(O.caliber2_weight(xa, xb, xb))
    rng = np.random.default_rng(3)
    for _ in range(20):
        xu, xa, xb = rng.standard_normal((3, 4))
        w, *_ = np.linalg.lstsq((xa - xb)[:, None], xu - xb, rcond=None)
        assert O.caliber2_weight(xu, xa, xb) == pytest.approx(w[0], rel=1e-12)


def _setup_level(g, seed=1, **kw):
    rp, ci, v = O.laplacian(g)
    col, nc = O.color(rp, ci)
    s = O.strong(rp, ci, v)
    X = O.test_vectors(rp, ci, v, col, nc, seed=seed, level=0)
    a = O.affinity(rp, ci, X)
    m = O.moments(rp, ci, v, X)
    sd, agg, ncoarse = O.aggregate(rp, ci, s, a, X, m)
    p0, w0, p1, w1, n2 = O.interp(rp, ci, s, X, sd, agg, ncoarse, **kw)
    return dict(rp=rp, ci=ci, v=v, s=s, X=X, seed=sd, agg=agg, nc=ncoarse, p0=p0, w0=w0, p1=p1,
                w1=w1, n2=n2)


def test_interp_rows_partition_of_unity_and_gate():
    d = _setup_level(I.grid2d(32, 24, 1.0, 1e-3))
    n = d["rp"].size - 1
    P = np.zeros((n, d["nc"]))
    P[np.arange(n), d["p0"]] += d["w0"]
    two = d["p1"] >= 0
    P[np.nonzero(two)[0], d["p1"][two]] += d["w1"][two]
    np.testing.assert_allclose(P.sum(1), 1.0, rtol=0, atol=2e-16)
    is_seed = d["seed"] == np.arange(n)
    assert np.all(d["p0"][is_seed] == d["agg"][is_seed]) and not np.any(two[is_seed])
    # every upgraded row: strong entries reach exactly {A(u), p1}
    rp, ci, s, agg = d["rp"], d["ci"], d["s"], d["agg"]
    for u in np.nonzero(two)[0]:
        reach = {int(agg[t]) for j, t in zip(range(rp[u], rp[u + 1]), ci[rp[u]:rp[u + 1]]) if s[j]}
        assert reach == {int(agg[u]), int(d["p1"][u])}
        assert 0.01 < d["w0"][u] < 0.99
    # self-targeting: most members upgrade on the grid-aligned anisotropic grid ...
    members = (~is_seed).sum()
    assert two.sum() > 0.8 * members
    # ... and almost none on an isotropic grid
    iso = _setup_level(I.grid2d(32, 24))
    assert iso["n2"] < 0.05 * (iso["rp"].size - 1)
    off = _setup_level(I.grid2d(32, 24, 1.0, 1e-3), enable_caliber2=False)
    assert off["n2"] == 0


# --- Galerkin operator ------------------------------------------------------------

def _P_dense(n, nc, p0, w0, p1, w1):
    P = np.zeros((n, nc))
    P[np.arange(n), p0] += w0
    two = p1 >= 0
    P[np.nonzero(two)[0], p1[two]] += w1[two]
    return P


def test_galerkin_matches_dense_PtLP():
    d = _setup_level(I.grid2d(30, 22, 1.0, 1e-2))
    rp, ci, v = d["rp"], d["ci"], d["v"]
    Crp, Cci, Cv = O.galerkin(rp, ci, v, d["nc"], d["p0"], d["w0"], d["p1"], d["w1"])
    n = rp.size - 1
    P = _P_dense(n, d["nc"], d["p0"], d["w0"], d["p1"], d["w1"])
    ref = P.T @ dense_L(rp, ci, v) @ P
    got = dense_L(Crp, Cci, Cv)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    assert np.array_equal(got, got.T)  # exact symmetry of the edge form
    assert np.abs(got.sum(1)).max() < 1e-12 * np.abs(ref).max()
    for a in range(d["nc"]):
        assert np.all(np.diff(Cci[Crp[a]:Crp[a + 1]]) > 0)


def test_galerkin_random_caliber2_rows():
    g = I.random_connected(150, 500, seed=12)
    rp, ci, v = O.laplacian(g)
    rng = np.random.default_rng(5)
    nc = 40
    p0 = np.concatenate([np.arange(nc), rng.integers(0, nc, g.n - nc)]).astype(np.int32)
    p1 = np.where(rng.random(g.n) < 0.4, rng.integers(0, nc, g.n), -1).astype(np.int32)
    p1[:nc] = -1
    p1[p1 == p0] = -1
    w0 = np.where(p1 >= 0, rng.uniform(0.02, 0.98, g.n), 1.0)
    w1 = np.where(p1 >= 0, 1.0 - w0, 0.0)
    Crp, Cci, Cv = O.galerkin(rp, ci, v, nc, p0, w0, p1, w1)
    P = _P_dense(g.n, nc, p0, w0, p1, w1)
    ref = P.T @ dense_L(rp, ci, v) @ P
    np.testing.assert_allclose(dense_L(Crp, Cci, Cv), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_galerkin_caliber1_integer_weights_exact():
    g = I.grid2d(16, 12, 2.0, 3.0)
    d = _setup_level(g, enable_caliber2=False)
    rp, ci, v = d["rp"], d["ci"], d["v"]
    Crp, Cci, Cv = O.galerkin(rp, ci, v, d["nc"], d["p0"], d["w0"], d["p1"], d["w1"])
    n = rp.size - 1
    P = _P_dense(n, d["nc"], d["p0"], d["w0"], d["p1"], d["w1"])
    ref = P.T @ dense_L(rp, ci, v) @ P
    got = dense_L(Crp, Cci, Cv)
    assert np.array_equal(got, ref)
    # pattern = aggregate adjacency graph (plus diagonal)
    adj = (np.abs(P.T @ (np.abs(dense_L(rp, ci, v)) > 0) @ P) > 0)
    assert np.array_equal(got != 0, adj)
