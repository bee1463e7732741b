"""The continuous-batching service: scheduling and admission logic on the CPU, and on the
GPU a mixed stream whose every result equals the same request solved alone (within the
solver's tolerance), under a budget small enough to force evictions."""
import numpy as np
import pytest

from paper_2606_24791_amd import inputs as I


class _FakeHandle:
    closed = 0

    def close(self):
        _FakeHandle.closed += 1


def _server(budget, graphs):
    from paper_2606_24791_amd import serve as S

    return S.Server(graphs, hbm_budget=budget, slots=2, use_torch_allocator=False)


def test_batching_coalesces_same_graph_and_respects_columns():
    from paper_2606_24791_amd import serve as S

    graphs = {"a": I.grid2d(10, 10, name="a"), "b": I.grid2d(12, 12, name="b")}
    srv = _server(1e12, graphs)
    for rid, (gid, k) in enumerate([("a", 3), ("b", 2), ("a", 20), ("a", 10), ("b", 1)]):
        srv.submit(S.Request(rid, gid, np.zeros((k, graphs[gid].n))))
    with srv.lock:
        batch, cols, _ = srv._next_batch()
    assert [r.rid for r in batch] == [0, 2] and cols == 23  # 10 more would exceed 32
    assert "a" in srv.busy_graphs
    with srv.lock:
        batch, cols, _ = srv._next_batch()  # "a" is busy: next graph
    assert [r.rid for r in batch] == [1, 4] and cols == 3
    with srv.lock:
        assert srv._next_batch() is None  # both graphs busy
    assert [r.rid for r in srv.queue] == [3]


def test_grouping_takes_other_idle_groupable_graphs():
    """With grouping on, the batch a slot takes is joined by batches for other idle graphs
    whose hierarchies are cached and run their whole cycle in the coarse tail (oldest
    request first, same-graph requests coalesced), up to the group size."""
    from paper_2606_24791_amd import serve as S

    graphs = {g: I.grid2d(10 + i, 10, name=g) for i, g in enumerate("abcd")}
    srv = S.Server(graphs, hbm_budget=1e12, slots=2, use_torch_allocator=False, group=3)
    for gid in "abcd":
        srv.cache[gid] = dict(handle=_FakeHandle(), levels=[graphs[gid].n], bytes=1.0, ws=0.0,
                              groupable=gid != "c")
    for rid, (gid, k) in enumerate([("a", 2), ("b", 1), ("c", 1), ("d", 3), ("b", 2), ("a", 1)]):
        srv.submit(S.Request(rid, gid, np.zeros((k, graphs[gid].n))))
    with srv.lock:
        nb = srv._next_batch()
        extras = srv._next_group(nb)
    assert [r.rid for r in nb[0]] == [0, 5]
    assert [[r.rid for r in e[0]] for e in extras] == [[1, 4], [3]]  # "c" is not groupable
    assert srv.busy_graphs == {"a", "b", "d"} and [r.rid for r in srv.queue] == [2]
    srv2 = S.Server(graphs, hbm_budget=1e12, slots=2, use_torch_allocator=False, group=0)
    srv2.cache.update(srv.cache)
    srv2.submit(S.Request(0, "a", np.zeros((1, graphs["a"].n))))
    srv2.submit(S.Request(1, "b", np.zeros((1, graphs["b"].n))))
    with srv2.lock:
        assert srv2._next_group(srv2._next_batch()) == []  # grouping off


def test_request_wider_than_a_batch_runs_alone():
    from paper_2606_24791_amd import serve as S

    graphs = {"a": I.grid2d(10, 10, name="a")}
    srv = _server(1e12, graphs)
    srv.submit(S.Request(0, "a", np.zeros((40, 100))))
    srv.submit(S.Request(1, "a", np.zeros((1, 100))))
    with srv.lock:
        batch, cols, _ = srv._next_batch()
    assert [r.rid for r in batch] == [0] and cols == 40


def test_batch_larger_than_the_budget_is_rejected_not_queued():
    from paper_2606_24791_amd import lamg as B
    from paper_2606_24791_amd import serve as S

    graphs = {"a": I.grid2d(40, 40, name="a")}
    srv = _server(1000.0, graphs)  # far below any hierarchy
    srv.submit(S.Request(0, "a", np.zeros((2, graphs["a"].n))))
    with srv.lock:
        assert srv._next_batch() is None
    assert not srv.queue and srv.rejected == 1 and srv.results[0].status == B.OOM


def test_admission_evicts_idle_hierarchies_lru_and_never_busy_ones():
    from paper_2606_24791_amd import serve as S

    graphs = {x: I.grid2d(30, 30, name=x) for x in "abc"}
    need = S.hierarchy_estimate(graphs["c"]) + S.workspace_bytes([graphs["c"].n], 1, True)
    srv = _server(2.5 * need, graphs)
    for gid in "ab":
        srv.cache[gid] = dict(handle=_FakeHandle(), levels=[900], bytes=need, ws=0.0)
    srv.busy_graphs.add("a")
    _FakeHandle.closed = 0
    with srv.lock:
        ok, extra = srv._admit("c", 1)
    assert ok and list(srv.cache) == ["a"] and _FakeHandle.closed == 1  # "b" evicted
    srv.reserved += extra
    with srv.lock:
        ok, _ = srv._admit("b", 1)  # "a" is busy, nothing else to evict
    assert not ok


@pytest.mark.gpu
def test_stream_results_equal_solves_alone():
    import sys

    import torch

    from paper_2606_24791_amd import lamg as B
    from paper_2606_24791_amd import serve as S

    assert torch.cuda.is_available()
    graphs, reqs = S.synthetic_stream(40, rate=400.0, n_graphs=8, nmin=4000, nmax=16000, kmax=4,
                                      seed=3)
    cols = 8
    # each request solved alone; the same pass measures every graph's setup peak and its
    # device bytes with a full batch of `cols` columns resident
    alone, peak, sizes = {}, {}, {}
    for gid, g in graphs.items():
        if not any(r.graph_id == gid for r in reqs):
            continue
        print(f"[case] alone {gid} n={g.n}", flush=True)
        h = B.lamg_setup(g)
        peak[gid] = B.lamg_hierarchy_info(h)["bytes_peak"]
        b = torch.tensor(I.rhs(g.n, cols, seed=1), device="cuda")
        B.lamg_solve(h, b, torch.empty_like(b), precision=B.FP32_IR)
        sizes[gid] = B.lamg_hierarchy_info(h)["bytes_device"]
        for req in reqs:
            if req.graph_id == gid:
                b = torch.tensor(req.b, device="cuda")
                phi = torch.empty_like(b)
                st = B.lamg_solve(h, b, phi, precision=B.FP32_IR)
                assert st["relres_max"] <= 1e-8
                alone[req.rid] = phi.cpu().numpy()
        h.close()
        est = S.hierarchy_estimate(g)
        print(f"[case]   setup peak {peak[gid] / 1e6:.2f} MB (estimate {est / 1e6:.2f} MB), "
              f"with {cols} columns {sizes[gid] / 1e6:.2f} MB "
              f"(estimate {(est + S.workspace_bytes([g.n], cols, True)) / 1e6:.2f})", flush=True)
        assert peak[gid] <= est  # the default admission estimate is an upper bound
    # admission charged with the measured peaks; room for any one graph with a full batch,
    # not for all of them at once
    by_name = {g.name: gid for gid, g in graphs.items()}
    need = {gid: max(peak[gid], sizes[gid]) + S.workspace_bytes([graphs[gid].n], cols, True)
            for gid in peak}
    budget = 1.2 * max(need.values())
    assert budget < sum(sizes[gid] for gid in {r.graph_id for r in reqs})
    print(f"[case] stream of {len(reqs)} requests, budget {budget / 1e6:.1f} MB", flush=True)
    used = {gid: graphs[gid] for gid in peak}
    srv = S.Server(used, hbm_budget=budget, slots=3, max_columns=cols,
                   estimate=lambda g: peak[by_name[g.name]])
    srv.progress_every = 10
    out = srv.run(reqs, stall_timeout=60.0)
    results = {r.rid: r for r in srv.results}
    srv.close()
    print(out, file=sys.stderr, flush=True)
    assert out["requests"] == len(reqs) and out["rejected"] == 0 and out["max_relres"] <= 1e-8
    assert out["evictions"] > 0 and out["overshoots"] == 0
    assert out["max_resident_bytes"] <= budget
    assert out["p50_ms"] is not None and out["p99_ms"] >= out["p50_ms"]
    for req in reqs:
        mix = results[req.rid].phi
        for c in range(mix.shape[0]):
            ref = alone[req.rid][c]
            err = np.linalg.norm(mix[c] - ref) / np.linalg.norm(ref)
            assert err <= 1e-6, (req.rid, c, err)


@pytest.mark.gpu
def test_grouped_stream_results_equal_solves_alone():
    """Grouping on, cache preloaded: batches on different small graphs share
    lamg_solve_group calls; every result still equals the request solved alone."""
    import sys

    import torch

    from paper_2606_24791_amd import lamg as B
    from paper_2606_24791_amd import serve as S

    assert torch.cuda.is_available()
    graphs, reqs = S.synthetic_stream(36, rate=0.0, n_graphs=8, nmin=1000, nmax=5000, kmax=4,
                                      seed=5)
    alone = {}
    opts = B.lamg_default_options(tail_finest=65535)
    for gid, g in graphs.items():
        mine = [r for r in reqs if r.graph_id == gid]
        if not mine:
            continue
        print(f"[case] alone {gid} n={g.n}", flush=True)
        h = B.lamg_setup(g, opts)
        for req in mine:
            b = torch.tensor(req.b, device="cuda")
            phi = torch.empty_like(b)
            B.lamg_solve(h, b, phi, precision=B.FP32_IR)
            alone[req.rid] = phi.cpu().numpy()
        h.close()
    srv = S.Server(graphs, hbm_budget=200e9, slots=2, group=6)
    # a warm cache: only cached hierarchies are grouped, and a cold stream arriving at once
    # would meet every graph uncached
    assert srv.preload(list(graphs)) == len(graphs)
    ngroupable = sum(e["groupable"] for e in srv.cache.values())
    print(f"[case] grouped stream: {ngroupable} of {len(graphs)} graphs groupable", flush=True)
    assert ngroupable >= 2
    out = srv.run(reqs, stall_timeout=60.0)
    results = {r.rid: r for r in srv.results}
    srv.close()
    print(out, file=sys.stderr, flush=True)
    assert out["requests"] == len(reqs) and out["rejected"] == 0 and out["max_relres"] <= 1e-8
    assert out["groups"] > 0 and out["grouped_batches"] >= 2 * out["groups"]
    for req in reqs:
        mix = results[req.rid].phi
        for c in range(mix.shape[0]):
            ref = alone[req.rid][c]
            err = np.linalg.norm(mix[c] - ref) / np.linalg.norm(ref)
            assert err <= 1e-6, (req.rid, c, err)
