"""Seeded synthetic workloads: weighted undirected graphs as adjacency CSR, and
right-hand sides.

This module serves both the HIP library's tests/benchmark and the CPU oracle's
tests. It holds none of the solver's arithmetic: it only draws graphs and random
vectors (numpy ``default_rng``), and returns them in the library's input format:
adjacency CSR with both directions stored, columns ascending within each row,
no diagonal, int32 indices and float64 positive weights.

The paper's own corpora (SuiteSparse, the approximate-Cholesky benchmark
families, SPE10) are not available; these generators produce graphs with the
shapes and weight distributions of its synthetic cases (grids, anisotropic grids,
heterogeneous weights, power-law and geometric graphs) instead.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Graph:
    """Adjacency CSR of a weighted undirected graph (both directions stored)."""

    n: int
    row_ptr: np.ndarray  # int32, n+1
    col_idx: np.ndarray  # int32, nnz, ascending per row
    weight: np.ndarray  # float64, nnz, > 0
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.nnz // 2

    @property
    def nnz_laplacian(self) -> int:
        """Stored entries of the Laplacian: both edge directions plus the diagonal."""
        return self.nnz + self.n


def from_edges(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray, name: str = "") -> Graph:
    """Symmetric CSR from an undirected edge list with i != j and no repeated pair."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    src = np.concatenate([i, j])
    dst = np.concatenate([j, i])
    ww = np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32), ww, name)


def grid2d(nx: int, ny: int, wx: float = 1.0, wy: float = 1.0, name: str | None = None) -> Graph:
    """5-point grid, node u = i + nx*j; weight wx on x-edges, wy on y-edges."""
    idx = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
    ex_i, ex_j = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    ey_i, ey_j = idx[:-1, :].ravel(), idx[1:, :].ravel()
    i = np.concatenate([ex_i, ey_i])
    j = np.concatenate([ex_j, ey_j])
    w = np.concatenate([np.full(ex_i.size, float(wx)), np.full(ey_i.size, float(wy))])
    return from_edges(nx * ny, i, j, w, name or f"grid2d_{nx}x{ny}_wy{wy:g}")


def grid3d(nx: int, ny: int, nz: int, weights: str = "unit", seed: int = 0,
           name: str | None = None) -> Graph:
    """7-point grid, node u = i + nx*(j + ny*k). ``weights='lognormal'`` draws
    lognormal(0, 1) i.i.d. per edge in edge order (x-, then y-, then z-edges)."""
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    pairs = [
        (idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()),
        (idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()),
        (idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()),
    ]
    i = np.concatenate([p[0] for p in pairs])
    j = np.concatenate([p[1] for p in pairs])
    if weights == "unit":
        w = np.ones(i.size)
    elif weights == "lognormal":
        w = np.random.default_rng(seed).lognormal(0.0, 1.0, i.size)
    else:
        raise ValueError(weights)
    return from_edges(nx * ny * nz, i, j, w, name or f"grid3d_{nx}x{ny}x{nz}_{weights}")


def largest_component(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray):
    """Restrict an edge list to its largest connected component, relabelled by
    ascending original id."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    A = sp.coo_matrix((np.ones(i.size), (i, j)), shape=(n, n))
    ncomp, lab = connected_components(A, directed=False)
    big = np.argmax(np.bincount(lab))
    keep = lab == big
    newid = np.full(n, -1, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    sel = keep[i] & keep[j]
    return int(keep.sum()), newid[i[sel]], newid[j[sel]], w[sel]


def chung_lu(n: int, beta: float, mean_deg: float, seed: int = 0, wlo: float = 1.0,
             whi: float = 2.0, name: str | None = None) -> Graph:
    """Chung-Lu power-law graph, degree exponent beta, largest connected component.

    Expected degrees w_i proportional to (i + i0)^(-1/(beta-1)), scaled to mean
    ``mean_deg``, with i0 chosen so that max w <= sqrt(sum w). sum(w)/2 endpoint
    pairs are drawn i.i.d. with probability proportional to w; self-loops and
    repeated pairs are dropped; edge weights are U[wlo, whi] i.i.d.
    """
    rng = np.random.default_rng(seed)
    expo = 1.0 / (beta - 1.0)
    total = mean_deg * n

    def weights_for(i0):
        base = (np.arange(n) + i0) ** (-expo)
        return base * (total / base.sum())

    lo, hi = 0.0, float(n)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if weights_for(mid).max() <= np.sqrt(total):
            hi = mid
        else:
            lo = mid
    wexp = weights_for(hi)
    cdf = np.cumsum(wexp)
    cdf /= cdf[-1]
    m_draw = int(round(total / 2))
    a = np.searchsorted(cdf, rng.random(m_draw), side="right")
    b = np.searchsorted(cdf, rng.random(m_draw), side="right")
    a = np.minimum(a, n - 1)
    b = np.minimum(b, n - 1)
    keep = a != b
    a, b = a[keep], b[keep]
    lo_ = np.minimum(a, b).astype(np.int64)
    hi_ = np.maximum(a, b).astype(np.int64)
    key = np.unique(lo_ * n + hi_)
    i, j = key // n, key % n
    w = rng.uniform(wlo, whi, i.size)
    n2, i, j, w = largest_component(n, i, j, w)
    return from_edges(n2, i, j, w, name or f"chunglu_{n}_b{beta:g}_d{mean_deg:g}")


def random_geometric(n: int, mean_deg: float = 10.0, seed: int = 0,
                     name: str | None = None) -> Graph:
    """n uniform points in the unit square, an edge between points closer than
    r = sqrt(mean_deg / (pi n)); unit weights; largest connected component."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = np.sqrt(mean_deg / (np.pi * n))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    i, j = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    w = np.ones(i.size)
    n2, i, j, w = largest_component(n, i, j, w)
    return from_edges(n2, i, j, w, name or f"rgg_{n}_d{mean_deg:g}")


def random_connected(n: int, extra_edges: int, seed: int = 0, wmin: float = 0.1,
                     wmax: float = 10.0, name: str | None = None) -> Graph:
    """Small test graph: a random spanning tree plus ``extra_edges`` random chords,
    log-uniform weights in [wmin, wmax]."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    parent = np.array([perm[rng.integers(0, k)] for k in range(1, n)], dtype=np.int64)
    ti, tj = perm[1:].astype(np.int64), parent
    ci = rng.integers(0, n, extra_edges)
    cj = rng.integers(0, n, extra_edges)
    i = np.concatenate([ti, ci])
    j = np.concatenate([tj, cj])
    keep = i != j
    lo_, hi_ = np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])
    key = np.unique(lo_ * n + hi_)
    i, j = key // n, key % n
    w = np.exp(rng.uniform(np.log(wmin), np.log(wmax), i.size))
    return from_edges(n, i, j, w, name or f"random_{n}_{extra_edges}")


def rhs(n: int, k: int = 1, seed: int = 0) -> np.ndarray:
    """k right-hand sides, N(0,1) i.i.d., returned as a (k, n) float64 array (row j
    is column j of the n x k block). The solver removes each column's mean itself."""
    return np.random.default_rng(seed).standard_normal((k, n))


# ---------------------------------------------------------------------------
# The measured workloads
# ---------------------------------------------------------------------------

def workload(name: str) -> Graph:
    """Named graphs of the measured configurations."""
    if name == "grid64":  # 64x64 5-point grid, unit weights (n = 4096)
        return grid2d(64, 64, 1.0, 1.0, name)
    if name == "aniso1024":  # 1024x1024, x-weight 1, y-weight 1e-3 (n = 1,048,576)
        return grid2d(1024, 1024, 1.0, 1e-3, name)
    if name == "lognormal128":  # 128^3 7-point, lognormal(0,1) weights (n = 2,097,152)
        return grid3d(128, 128, 128, "lognormal", seed=0, name=name)
    if name == "chunglu2m":  # Chung-Lu n = 2M, beta 2.1, mean degree 16, LCC
        return chung_lu(2_000_000, 2.1, 16.0, seed=0, name=name)
    if name == "rgg1m":  # random geometric, 1M points, mean degree 10, LCC; numbered in the
        # points' draw order, which is random in space
        return random_geometric(1_000_000, 10.0, seed=0, name=name)
    raise KeyError(name)
