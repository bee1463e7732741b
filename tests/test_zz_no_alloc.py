"""The allocation-free entry point lamg_solve_noalloc through the C ABI: on two calls in a
row (the second on a smaller graph with fewer columns) its results equal those of
lamg_solve on the same handles and right-hand sides, no device allocation happens during
it (every allocation of the library goes through a counting hook here), the handle's own
cached workspace is left as it was, and a solve larger than the fixed scratch is refused
with SCRATCH_TOO_SMALL before anything is written."""
import sys

import numpy as np
import pytest

from paper_2606_24791_amd import inputs as I

pytestmark = pytest.mark.gpu

SOL_TOL = 1e-6


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "a HIP device is required"
    from paper_2606_24791_amd import lamg

    return lamg


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def test_noalloc_solve_matches_lamg_solve(B):
    import torch

    dev = torch.cuda.current_device()
    counts = {"alloc": 0, "free": 0}

    def alloc(nbytes, stream, ctx):
        counts["alloc"] += 1
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
        except Exception:
            return None

    def free(ptr, stream, ctx):
        counts["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    B.lamg_set_allocator(alloc, free)
    handles = []
    try:
        cases = [  # (name, graph, columns, precision, rhs seed); the second call is smaller
            ("anisotropic grid 96x80", I.grid2d(96, 80, 1.0, 1e-3), 8, B.FP32_IR, 31),
            ("random graph n=3000", I.random_connected(3000, 9000, seed=12), 3, B.FP64, 32),
        ]
        for name, g, k, prec, seed in cases:
            note(f"noalloc vs lamg_solve: {name} n={g.n} k={k} precision={prec}")
            h = B.lamg_setup(g)
            handles.append(h)
            b = torch.tensor(I.rhs(g.n, k, seed=seed), device="cuda")
            ref = torch.empty_like(b)
            st_ref = B.lamg_solve(h, b, ref, precision=prec)
            torch.cuda.synchronize()
            phi = torch.full_like(b, 3.0)
            a0, f0 = counts["alloc"], counts["free"]
            st = B.lamg_solve_noalloc(h, b, phi, precision=prec)
            torch.cuda.synchronize()
            assert (counts["alloc"], counts["free"]) == (a0, f0), "device allocation in noalloc"
            assert st["status"] == B.OK and st["relres_max"] <= 1e-8, st
            assert st["cycles"] == st_ref["cycles"], (st["cycles"], st_ref["cycles"])
            p, r = phi.cpu().numpy(), ref.cpu().numpy()
            for c in range(k):
                err = np.linalg.norm(p[c] - r[c]) / np.linalg.norm(r[c])
                emax = np.abs(p[c] - r[c]).max() / np.abs(r[c]).max()
                assert err <= SOL_TOL and emax <= SOL_TOL, (c, err, emax)
            note(f"bitwise equal to lamg_solve: {bool(np.array_equal(p, r))}")
            # the handle's cached workspace is intact: lamg_solve again allocates nothing
            # and gives the same solution
            again = torch.empty_like(b)
            a0 = counts["alloc"]
            B.lamg_solve(h, b, again, precision=prec)
            torch.cuda.synchronize()
            assert counts["alloc"] == a0
            assert torch.equal(again, ref)
        # larger than the scratch: refused, phi untouched
        g = I.grid2d(150, 150)
        note(f"noalloc beyond the scratch: n={g.n} k=32")
        h = B.lamg_setup(g)
        handles.append(h)
        b = torch.tensor(I.rhs(g.n, 32, seed=5), device="cuda")
        phi = torch.full_like(b, 3.0)
        st = B.lamg_solve_noalloc(h, b, phi, precision=B.FP32_IR, check=False)
        assert st["status"] == B.SCRATCH_TOO_SMALL, st
        assert torch.all(phi == 3.0)
        assert "allocation-free" in B.lamg_status_string(st["status"])
    finally:
        for h in handles:
            h.close()
        B.lamg_set_allocator()


def test_noalloc_with_smoother_and_renumbering_options(B):
    """Hierarchies built with the block-Jacobi smoother (its sweeps use the level's residual
    vector as work space) and with the input renumbered (right-hand sides and solutions go
    through the composed permutation): the allocation-free solve still equals lamg_solve."""
    import torch

    dev = torch.cuda.current_device()
    counts = {"alloc": 0}

    def alloc(nbytes, stream, ctx):
        counts["alloc"] += 1
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
        except Exception:
            return None

    def free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    B.lamg_set_allocator(alloc, free)
    handles = []
    try:
        cases = [  # (name, graph, options, columns, precision, rhs seed)
            ("Chung-Lu n=10000, block-Jacobi", I.chung_lu(10000, 2.1, 24, seed=3),
             dict(smoother=2), 2, B.FP32_IR, 41),
            ("random geometric n=5000, renumbered", I.random_geometric(5000, seed=5),
             dict(reorder=1), 3, B.FP64, 42),
        ]
        for name, g, opts, k, prec, seed in cases:
            note(f"noalloc with options: {name} n={g.n} k={k} precision={prec}")
            h = B.lamg_setup(g, B.lamg_default_options(**opts))
            handles.append(h)
            info = B.lamg_hierarchy_info(h)
            assert any(info["bjgs"]) if "smoother" in opts else info["reordered"]
            b = torch.tensor(I.rhs(g.n, k, seed=seed), device="cuda")
            ref = torch.empty_like(b)
            st_ref = B.lamg_solve(h, b, ref, precision=prec)
            torch.cuda.synchronize()
            phi = torch.full_like(b, 3.0)
            a0 = counts["alloc"]
            st = B.lamg_solve_noalloc(h, b, phi, precision=prec)
            torch.cuda.synchronize()
            assert counts["alloc"] == a0, "device allocation in noalloc"
            assert st["status"] == B.OK and st["relres_max"] <= 1e-8, st
            assert st["cycles"] == st_ref["cycles"]
            p, r = phi.cpu().numpy(), ref.cpu().numpy()
            for c in range(k):
                err = np.linalg.norm(p[c] - r[c]) / np.linalg.norm(r[c])
                emax = np.abs(p[c] - r[c]).max() / np.abs(r[c]).max()
                assert err <= SOL_TOL and emax <= SOL_TOL, (c, err, emax)
    finally:
        for h in handles:
            h.close()
        B.lamg_set_allocator()
