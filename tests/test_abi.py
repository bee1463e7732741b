"""The C-ABI library on the CPU: it loads, exports every symbol include/lamg.h declares,
and rejects invalid graphs on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2606_24791_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lamg.h")
LIB = os.path.join(ROOT, "paper_2606_24791_amd", "liblamg.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="liblamg.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lamg_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert {"lamg_setup", "lamg_solve", "lamg_destroy", "lamg_hierarchy_info",
            "lamg_export_level", "lamg_set_allocator", "lamg_status_string"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_host_only_entry_points():
    from paper_2606_24791_amd import lamg as B

    assert B.lamg_status_string(B.OK) == "ok"
    assert B.lamg_status_string(B.NOT_CONVERGED) == "not converged"
    assert "gfx950" in B.lamg_version()
    o = B.lamg_default_options()
    assert (o.seed, o.n_direct, o.enable_veto, o.enable_caliber2, o.kappa) == (1, 512, 1, 1, 4)
    assert (o.elimination, o.smoother, o.tail_rows, o.build_fp32, o.graphs, o.reorder) == \
        (1, 0, 2500, 1, 0, 0)
    assert o.tail_finest == 0


def _graph(n, rows, cols, w):
    rows = np.asarray(rows)
    order = np.lexsort((cols, rows))
    rows, cols, w = rows[order], np.asarray(cols)[order], np.asarray(w, float)[order]
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return I.Graph(n, rp, np.asarray(cols, np.int32), w)


def test_input_errors_are_reported_without_device():
    from paper_2606_24791_amd import lamg as B

    good = I.grid2d(4, 3)
    # asymmetric weight
    g = I.Graph(good.n, good.row_ptr.copy(), good.col_idx.copy(), good.weight.copy())
    g.weight[0] = 2.0
    assert B.lamg_setup_status(g) == B.NOT_SYMMETRIC
    # missing reverse entry
    g = _graph(3, [0, 1, 1, 2], [1, 0, 2, 0], [1, 1, 1, 1])
    assert B.lamg_setup_status(g) == B.NOT_SYMMETRIC
    # self loop
    g = _graph(2, [0, 0, 1, 1], [0, 1, 0, 1], [1, 1, 1, 1])
    assert B.lamg_setup_status(g) == B.SELF_LOOP
    # weights: zero, negative, NaN, inf
    for bad in (0.0, -1.0, np.nan, np.inf):
        g = _graph(2, [0, 1], [1, 0], [bad, bad])
        assert B.lamg_setup_status(g) == B.BAD_WEIGHT, bad
    # disconnected
    g = _graph(4, [0, 1, 2, 3], [1, 0, 3, 2], [1, 1, 1, 1])
    assert B.lamg_setup_status(g) == B.DISCONNECTED
    # unsorted columns / out of range / inconsistent row_ptr
    g = I.Graph(good.n, good.row_ptr.copy(), good.col_idx.copy(), good.weight.copy())
    g.col_idx[[0, 1]] = g.col_idx[[1, 0]]
    assert B.lamg_setup_status(g) == B.INVALID_ARG
    g = I.Graph(good.n, good.row_ptr.copy(), good.col_idx.copy(), good.weight.copy())
    g.col_idx[0] = 99
    assert B.lamg_setup_status(g) == B.INVALID_ARG
    g = I.Graph(good.n, good.row_ptr.copy(), good.col_idx.copy(), good.weight.copy())
    g.row_ptr[1], g.row_ptr[2] = g.row_ptr[2], g.row_ptr[1] - 1  # not monotone
    assert B.lamg_setup_status(g) == B.INVALID_ARG
    # options out of range
    assert B.lamg_setup_status(good, B.lamg_default_options(n_direct=0)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(kappa=5)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(elimination=2)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(smoother=3)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(reorder=2)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(graphs=-1)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(tail_rows=-1)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(n_direct=1025)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(tail_finest=-1)) == B.INVALID_ARG
    assert B.lamg_setup_status(good, B.lamg_default_options(tail_finest=65536)) == B.INVALID_ARG
