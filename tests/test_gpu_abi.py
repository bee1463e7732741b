"""C-ABI contracts of lamg_solve on the device: right-hand sides that hold NaN or infinite
values are rejected before anything is written, and the residual history never exceeds
the documented buffer size."""
import ctypes as C
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("k,col", [(3, 1), (40, 37)])
def test_nonfinite_rhs_is_rejected(B, bad, k, col):
    """eq. (1.1) needs a finite b. One column with a NaN or infinite entry: INVALID_ARG and
    phi left as it was -- also when the column sits in the second 32-column chunk."""
    import torch

    g = I.grid2d(30, 20, 1.0, 1e-2)
    note(f"non-finite rhs {bad} k={k} column {col}")
    h = B.lamg_setup(g)
    bh = I.rhs(g.n, k, seed=1)
    bh[col, 11] = bad
    b = torch.tensor(bh, device="cuda")
    for prec in (B.FP64, B.FP32_IR):
        phi = torch.full_like(b, 7.0)
        st = B.lamg_solve(h, b, phi, precision=prec, check=False)
        assert st["status"] == B.INVALID_ARG, st
        assert torch.all(phi == 7.0)
    # the handle stays usable: a clean block solves
    b = torch.tensor(I.rhs(g.n, k, seed=2), device="cuda")
    phi = torch.empty_like(b)
    st = B.lamg_solve(h, b, phi, precision=B.FP32_IR)
    assert st["converged"] and st["relres_max"] <= 1e-8
    h.close()


def test_history_buffer_of_the_default_cycle_cap(B):
    """max_cycles <= 0 selects 300 cycles; the caller's history buffer then needs 301
    entries, and nothing is written past them."""
    import torch

    g = I.grid2d(24, 24)
    note("history buffer with max_cycles = 0")
    h = B.lamg_setup(g)
    b = torch.tensor(I.rhs(g.n, 1, seed=3), device="cuda")
    phi = torch.empty_like(b)
    buf = np.full(301 + 64, -5.0)
    rel = np.zeros(1)
    cyc = np.zeros(1, np.int32)
    info = B.lamg_solve_info()
    info.relres = rel.ctypes.data
    info.col_cycles = cyc.ctypes.data
    info.history = buf.ctypes.data
    st = B._lib.lamg_solve(h.ptr, b.data_ptr(), 1, 1e-8, 0, B.FP64, phi.data_ptr(),
                           C.byref(info), torch.cuda.current_stream().cuda_stream)
    assert st == B.OK
    assert 1 <= info.history_len <= 301 and info.history_len == info.cycles + 1
    assert buf[0] == 1.0 and np.all(buf[1:info.history_len] > 0)
    assert np.all(buf[301:] == -5.0)
    h.close()


def test_setup_phase_times(B):
    """lamg_hier_info.setup_phase_seconds: every phase non-negative, their sum within the
    setup's wall time, and the phases a hierarchy with aggregation and elimination levels
    runs (colouring, level kernels, aggregation, interpolation, elimination, Galerkin,
    coarsest inverse, layout, input) all positive."""
    g = I.grid2d(120, 90, 1.0, 1e-2)
    note("setup phase times")
    h = B.lamg_setup(g)
    hi = B.lamg_hierarchy_info(h)
    h.close()
    ph = hi["setup_phases"]
    assert set(ph) == set(B.SETUP_PHASE_NAMES)
    assert all(v >= 0.0 for v in ph.values()), ph
    assert sum(ph.values()) <= hi["setup_seconds"] * (1 + 1e-9) + 1e-6, (ph, hi["setup_seconds"])
    assert any(hi["elim"]) and hi["levels"] >= 3
    for name in B.SETUP_PHASE_NAMES:
        assert ph[name] > 0.0, (name, ph)
