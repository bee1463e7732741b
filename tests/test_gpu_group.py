"""lamg_solve_group: several requests (different graphs, column counts) solved together, the
coarse-tail work of every cycle of the groupable ones in one launch. Each request's result
must be exactly what lamg_solve gives for it alone on the same handle, requests that cannot
be grouped are still solved, a rejected request leaves the others untouched, and the
results agree with the CPU oracle."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2606_24791_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "a HIP device is required"
    from paper_2606_24791_amd import lamg

    return lamg


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


GRAPHS = [  # (graph, columns)
    (lambda: I.grid2d(40, 30), 1),
    (lambda: I.grid2d(64, 40, 1.0, 1e-3), 3),
    (lambda: I.random_geometric(3000, 10.0, seed=2), 8),
    (lambda: I.grid3d(12, 11, 10, "lognormal", seed=5), 2),
    (lambda: I.random_connected(1500, 4000, seed=9), 32),
    (lambda: I.grid2d(33, 31), 5),
]


def test_group_equals_solves_alone(B):
    import torch

    graphs = [(f(), k) for f, k in GRAPHS]
    opts = B.lamg_default_options(tail_finest=65535)
    hs = [B.lamg_setup(g, opts) for g, _ in graphs]
    grouped = [B.lamg_hierarchy_info(h)["tail_level"] == 0 for h in hs]
    note(f"group of {len(hs)} requests, grouped: {grouped}")
    assert sum(grouped) >= 4
    bs = [torch.tensor(I.rhs(g.n, k, seed=40 + i), device="cuda") for i, (g, k) in enumerate(graphs)]
    # a request on a handle built without the option is solved on its own inside the call
    g_extra = I.grid2d(50, 20)
    h_extra = B.lamg_setup(g_extra)
    assert B.lamg_hierarchy_info(h_extra)["tail_level"] != 0
    b_extra = torch.tensor(I.rhs(g_extra.n, 4, seed=7), device="cuda")
    handles, rhs = hs + [h_extra], bs + [b_extra]
    for prec in (B.FP32_IR, B.FP64):
        alone = []
        for h, b in zip(handles, rhs):
            phi = torch.empty_like(b)
            st = B.lamg_solve(h, b, phi, precision=prec)
            alone.append((phi, st))
        phis = [torch.full_like(b, 5.0) for b in rhs]
        sts = B.lamg_solve_group(handles, rhs, phis, precision=prec)
        for r, ((ref, st0), phi, st) in enumerate(zip(alone, phis, sts)):
            assert st["status"] == B.OK and st["relres_max"] <= 1e-8, (r, st)
            assert torch.equal(phi, ref), (prec, r, float((phi - ref).abs().max()))
            assert np.array_equal(st["col_cycles"], st0["col_cycles"]), r
            assert st["bytes"] == pytest.approx(st0["bytes"], rel=1e-12), r
    # the oracle on two of the requests
    for r in (1, 4):
        g, k = graphs[r]
        bh = bs[r].cpu().numpy()
        ph = phis[r].cpu().numpy()
        oh = O.Hierarchy(g, seed=1)
        for c in (0, k - 1):
            ref, _, _ = oh.solve(bh[c], 1e-8, 100)
            err = np.linalg.norm(ph[c] - ref) / np.linalg.norm(ref)
            assert err <= 1e-6, (r, c, err)
    for h in handles:
        h.close()


def test_group_isolates_a_bad_request(B):
    import torch

    opts = B.lamg_default_options(tail_finest=65535)
    graphs = [I.grid2d(30, 30), I.grid2d(45, 20, 1.0, 1e-2), I.random_connected(900, 2500, seed=3)]
    hs = [B.lamg_setup(g, opts) for g in graphs]
    bs = [torch.tensor(I.rhs(g.n, 2, seed=i), device="cuda") for i, g in enumerate(graphs)]
    bs[1][1, 7] = float("nan")
    note("group with a non-finite request")
    phis = [torch.full_like(b, 5.0) for b in bs]
    sts = B.lamg_solve_group(hs, bs, phis, precision=B.FP32_IR, check=False)
    assert sts[1]["status"] == B.INVALID_ARG and torch.all(phis[1] == 5.0)
    for r in (0, 2):
        ref = torch.empty_like(bs[r])
        B.lamg_solve(hs[r], bs[r], ref, precision=B.FP32_IR)
        assert sts[r]["status"] == B.OK and torch.equal(phis[r], ref), r
    with pytest.raises(B.LamgError):  # the same handle twice is an argument error
        B.lamg_solve_group([hs[0], hs[0]], [bs[0], bs[0]], [phis[0], phis[2]])
    for h in hs:
        h.close()
