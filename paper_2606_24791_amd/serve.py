"""Continuous-batching solve service over the LAMG+ library.

Requests (a graph id and a block of right-hand sides) arrive over time. The server keeps
hierarchies resident on the device (an LRU cache charged against an HBM budget), admits
work only while the budget allows, and runs up to `slots` solves at once, one per HIP
stream and worker thread (the library call releases the GIL). When a slot frees, it takes
the oldest waiting request whose graph is idle and coalesces every other waiting request
for the same graph into one multi-right-hand-side solve (up to 32 columns), so requests
that arrive while others run join the next batch instead of waiting for their own turn.
Each column of a batch is solved independently inside the library (its own energy
correction, recombination and stopping), so a request's result does not depend on what
it was batched with beyond rounding.

Latency = completion time - arrival time (queueing, any setup, host/device copies and the
solve included); the summary reports p50/p99 overall and split by hierarchy-cache hit and
miss, and throughput = sum of nnz(L) * columns over the wall time.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np
import torch

from . import lamg as B


@dataclasses.dataclass
class Request:
    rid: int
    graph_id: str
    b: np.ndarray  # (k, n) right-hand sides
    arrival: float = 0.0  # seconds from the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    graph_id: str
    phi: np.ndarray
    relres: np.ndarray
    cycles: np.ndarray
    latency: float
    cache_hit: bool
    batch_columns: int
    status: int


def workspace_bytes(n_levels: list[int], k: int, fp32: bool) -> int:
    """Device bytes of a solve workspace with k columns: the finest level's FP64 state and
    recombination history (13 vectors) and six cycle vectors per level. With only the
    finest size known, the coarse levels are taken to add as much again."""
    s = 4 if fp32 else 8
    total_n = sum(n_levels) if len(n_levels) > 1 else 2 * n_levels[0]
    return int(13 * 8 * n_levels[0] * k + 6 * s * k * total_n + (1 << 16) * (k + 1))


def hierarchy_estimate(graph) -> int:
    """Device bytes a setup may hold at its peak, before the hierarchy exists: the Galerkin
    product's sort buffers (up to 12 keyed 16-byte contributions per stored entry, double
    buffered) beside the finest level's operator, test vectors and aggregation data, and the
    persistent FP64 + FP32 operators of all levels (operator complexity up to 4), plus the
    coarsest inverse."""
    nnz, n = graph.nnz_laplacian, graph.n
    return int(12 * 32 * nnz + 4 * (16 * nnz + 100 * n) + 8 * 1024 * 1024 + (1 << 20))


class Server:
    def __init__(self, graphs: dict, hbm_budget: float = 200e9, slots: int = 4,
                 precision: int = B.FP32_IR, tol: float = 1e-8, max_columns: int = 32,
                 use_torch_allocator: bool = True, estimate=None, smoother: int = 0,
                 hip_graphs: bool = False, group: int = 0, reorder: int = 0):
        self.graphs = graphs
        # setup option: 1 = Chebyshev, 2 = block-Jacobi Gauss-Seidel, on levels with many colours
        self.smoother = smoother
        self.hip_graphs = hip_graphs  # setup option: replay repeated cycles as HIP graphs
        self.reorder = reorder  # setup option: self-gated RCM renumbering of each graph
        # up to this many batches on different graphs per lamg_solve_group call (0/1: none);
        # hierarchies are then built to run the whole FP32 cycle of small graphs in the tail
        self.group = group
        self.groups = 0  # lamg_solve_group calls made
        self.grouped_batches = 0
        # device bytes charged for a graph's setup before its hierarchy exists
        self.estimate = estimate or hierarchy_estimate
        self.budget = float(hbm_budget)
        self.slots = slots
        self.precision = precision
        self.tol = tol
        self.max_columns = max_columns
        self.lock = threading.Condition()
        self.queue: collections.deque[Request] = collections.deque()
        self.cache: collections.OrderedDict[str, dict] = collections.OrderedDict()
        self.busy_graphs: set[str] = set()
        self.reserved = 0.0  # bytes of in-flight work beyond resident hierarchies
        self.results: list[Result] = []
        self.done = False
        self.t0 = 0.0
        self.max_resident = 0.0
        self.setups = 0
        self.evictions = 0
        self.rejected = 0
        self.overshoots = 0  # times the resident bytes could not be brought under the budget
        self.progress_every = 0  # print a progress line every this many results (0: never)
        self.log_batches = False  # print one line per solved batch
        if use_torch_allocator:
            self._install_allocator()

    # --- device memory through torch's stream-ordered caching allocator -------------
    def _install_allocator(self):
        dev = torch.cuda.current_device()

        def alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
            except Exception:
                return None

        def free(ptr, stream, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        B.lamg_set_allocator(alloc, free)

    # --- accounting -------------------------------------------------------------------
    def _resident(self) -> float:
        return sum(e["bytes"] for e in self.cache.values()) + self.reserved

    def _need(self, gid: str, k: int) -> tuple[float, float]:
        """(bytes the batch adds, bytes the graph holds once it has run): a cached graph adds
        only workspace growth; a new one its whole hierarchy and workspace."""
        g = self.graphs[gid]
        fp32 = self.precision == B.FP32_IR
        entry = self.cache.get(gid)
        if entry is not None:
            extra = max(0.0, workspace_bytes(entry["levels"], k, fp32) - entry["ws"])
            return extra, entry["bytes"] + extra
        extra = self.estimate(g) + workspace_bytes([g.n], k, fp32)
        return extra, extra

    def _admit(self, gid: str, k: int) -> tuple[bool, float]:
        """Called with the lock held: can a k-column batch on graph gid start now? Evicts
        idle hierarchies (least recently used first) if that makes room."""
        extra, _ = self._need(gid, k)
        while self._resident() + extra > self.budget:
            victim = next((v for v in self.cache if v not in self.busy_graphs and v != gid), None)
            if victim is None:
                return False, extra
            ev = self.cache.pop(victim)
            ev["handle"].close()
            self.evictions += 1
        return True, extra

    # --- scheduling -------------------------------------------------------------------
    def submit(self, req: Request):
        with self.lock:
            self.queue.append(req)
            self.lock.notify_all()

    def _next_batch(self):
        """Called with the lock held. Oldest waiting request on an idle graph, plus every
        other waiting request for that graph (column limit permitting). A batch that could
        not fit even alone is rejected (status OOM) instead of waiting forever."""
        for i, req in enumerate(self.queue):
            if req.graph_id in self.busy_graphs:
                continue
            batch, cols = [req], req.b.shape[0]  # a request wider than a batch runs alone
            for r in list(self.queue):
                if r is not req and r.graph_id == req.graph_id \
                        and cols + r.b.shape[0] <= self.max_columns:
                    batch.append(r)
                    cols += r.b.shape[0]
            _, alone = self._need(req.graph_id, req.b.shape[0])
            if alone > self.budget:
                self.queue.remove(req)
                self._reject(req)
                self.lock.notify_all()
                return None
            ok, extra = self._admit(req.graph_id, cols)
            if not ok:
                return None
            for r in batch:
                self.queue.remove(r)
            self.busy_graphs.add(req.graph_id)
            self.reserved += extra
            return batch, cols, extra
        return None

    def _take_graph(self, gid: str, first: Request):
        """Called with the lock held: first plus every other waiting request for gid (column
        limit permitting), if the batch fits the budget; removes them from the queue and
        marks gid busy. Returns (batch, cols, extra) or None."""
        batch, cols = [first], first.b.shape[0]
        for r in list(self.queue):
            if r is not first and r.graph_id == gid and cols + r.b.shape[0] <= self.max_columns:
                batch.append(r)
                cols += r.b.shape[0]
        ok, extra = self._admit(gid, cols)
        if not ok:
            return None
        for r in batch:
            self.queue.remove(r)
        self.busy_graphs.add(gid)
        self.reserved += extra
        return batch, cols, extra

    def _next_group(self, nb):
        """Called with the lock held, after _next_batch chose nb: with grouping on and nb's
        graph cached and groupable, more batches for other idle, cached, groupable graphs
        (oldest request first) to be solved in the same lamg_solve_group call."""
        if self.group <= 1:
            return []
        e = self.cache.get(nb[0][0].graph_id)
        if e is None or not e.get("groupable"):
            return []
        extras = []
        for req in list(self.queue):
            if len(extras) + 1 >= self.group:
                break
            if req not in self.queue or req.graph_id in self.busy_graphs:
                continue
            e2 = self.cache.get(req.graph_id)
            if e2 is None or not e2.get("groupable") or req.b.shape[0] > self.max_columns:
                continue
            got = self._take_graph(req.graph_id, req)
            if got is None:
                break
            extras.append(got)
        return extras

    def _reject(self, req: Request, status: int = B.OOM):
        """Called with the lock held: answers req with an error status and no solution."""
        now = time.perf_counter() - self.t0
        k = req.b.shape[0]
        self.results.append(Result(req.rid, req.graph_id, np.full((k, req.b.shape[1]), np.nan),
                                   np.full(k, np.nan), np.zeros(k, np.int32), now - req.arrival,
                                   False, k, status))
        self.rejected += 1

    def _worker(self, stream):
        torch.cuda.set_device(torch.cuda.current_device())
        while True:
            with self.lock:
                while True:
                    if self.done and not self.queue:
                        return
                    nb = self._next_batch()
                    if nb is not None:
                        extras = self._next_group(nb)
                        break
                    self.lock.wait(0.05)
            if extras:
                self._run_group([nb] + extras, stream)
                continue
            batch, cols, extra = nb
            gid = batch[0].graph_id
            resv = {"extra": extra}  # bytes this batch holds in `reserved`
            try:
                self._run_batch(batch, cols, gid, stream, resv)
            except B.LamgError as e:  # the batch fails, the service goes on
                with self.lock:
                    for r in batch:
                        self._reject(r, e.status)
            finally:
                with self.lock:
                    self.busy_graphs.discard(gid)
                    self.reserved -= resv["extra"]
                    self.lock.notify_all()

    def _make_room(self, gid: str):
        """Called with the lock held: evicts idle hierarchies (LRU first, never gid) while
        the resident bytes exceed the budget; counts an overshoot if that is not enough."""
        while self._resident() > self.budget:
            victim = next((v for v in self.cache if v not in self.busy_graphs and v != gid), None)
            if victim is None:
                self.overshoots += 1
                return
            self.cache.pop(victim)["handle"].close()
            self.evictions += 1

    def _build(self, gid: str, cols: int, stream, resv) -> dict:
        """Sets up gid's hierarchy on `stream` and caches it. resv["extra"] holds the bytes
        reserved for it (the estimate); on return it holds the workspace estimate of a
        cols-column batch instead."""
        g = self.graphs[gid]
        fp32 = self.precision == B.FP32_IR
        h = B.lamg_setup(g, B.lamg_default_options(
            smoother=self.smoother, graphs=int(self.hip_graphs), reorder=int(self.reorder),
            tail_finest=65535 if self.group > 1 else 0), stream=stream)
        info = B.lamg_hierarchy_info(h)
        entry = dict(handle=h, levels=info["n"], bytes=float(info["bytes_device"]), ws=0.0,
                     groupable=info["tail_level"] == 0)
        ws_est = float(workspace_bytes(info["n"], cols, fp32)) if cols else 0.0
        with self.lock:
            # the setup's high-water mark beside everything else resident
            others = self._resident() - resv["extra"]
            self.max_resident = max(self.max_resident, others + info["bytes_peak"])
            # the estimate is replaced by the measured hierarchy + the workspace
            self.reserved += ws_est - resv["extra"]
            resv["extra"] = ws_est
            self.cache[gid] = entry
            self.setups += 1
            self._make_room(gid)
        return entry

    def preload(self, gids) -> int:
        """Builds the hierarchies of gids (in that order) before a stream starts, so that
        their first requests are cache hits; stops at the first one the budget cannot hold.
        Returns how many were built."""
        stream = torch.cuda.current_stream()
        built = 0
        for gid in gids:
            with self.lock:
                if gid in self.cache:
                    continue
                ok, extra = self._admit(gid, 0)
                if not ok:
                    break
                self.reserved += extra
            resv = {"extra": extra}
            try:
                self._build(gid, 0, stream, resv)
                built += 1
            finally:
                with self.lock:
                    self.reserved -= resv["extra"]
        stream.synchronize()
        return built

    def _run_batch(self, batch, cols, gid, stream, resv):
        g = self.graphs[gid]
        with torch.cuda.stream(stream):
            with self.lock:
                entry = self.cache.get(gid)
                if entry is not None:
                    self.cache.move_to_end(gid)
            hit = entry is not None
            if not hit:
                entry = self._build(gid, cols, stream, resv)
            bh = np.concatenate([r.b for r in batch], axis=0)
            b = torch.tensor(bh, device="cuda")
            phi = torch.empty_like(b)
            ts = time.perf_counter()
            st = B.lamg_solve(entry["handle"], b, phi, tol=self.tol, precision=self.precision,
                              stream=stream)
            ph = phi.cpu().numpy()
            stream.synchronize()
            if self.log_batches:
                import sys

                print(f"[serve] batch {gid} n={g.n} cols={cols} {'hit' if hit else 'miss'} "
                      f"solve {1e3 * (time.perf_counter() - ts):.1f} ms cycles {st['cycles']}",
                      file=sys.stderr, flush=True)
            self._answer(batch, cols, gid, entry, hit, st, ph, resv)

    def _answer(self, batch, cols, gid, entry, hit, st, ph, resv):
        """The results of one solved batch: workspace accounting, one Result per request."""
        fp32 = self.precision == B.FP32_IR
        info = B.lamg_hierarchy_info(entry["handle"])
        now = time.perf_counter() - self.t0
        with self.lock:
            # the entry now holds its real workspace: drop the batch's reservation
            entry["bytes"] = float(info["bytes_device"])
            entry["ws"] = max(entry["ws"], float(workspace_bytes(entry["levels"], cols, fp32)))
            self.max_resident = max(self.max_resident, self._resident() - resv["extra"])
            self.reserved -= resv["extra"]
            resv["extra"] = 0.0
            self._make_room(gid)
            c0 = 0
            for r in batch:
                k = r.b.shape[0]
                self.results.append(Result(
                    r.rid, gid, ph[c0:c0 + k], st["relres"][c0:c0 + k].copy(),
                    st["col_cycles"][c0:c0 + k].copy(), now - r.arrival, hit, cols,
                    st["status"]))
                c0 += k

    def _run_group(self, nbs, stream):
        """Solves several batches on cached, groupable graphs with one lamg_solve_group call
        (their coarse-tail work shares one launch per cycle)."""
        entries, bs, phis = [], [], []
        with self.lock:
            for batch, _, _ in nbs:
                gid = batch[0].graph_id
                self.cache.move_to_end(gid)
                entries.append(self.cache[gid])
        try:
            with torch.cuda.stream(stream):
                for (batch, _, _) in nbs:
                    b = torch.tensor(np.concatenate([r.b for r in batch], axis=0), device="cuda")
                    bs.append(b)
                    phis.append(torch.empty_like(b))
                sts = B.lamg_solve_group([e["handle"] for e in entries], bs, phis, tol=self.tol,
                                         precision=self.precision, stream=stream, check=False)
                phs = [p.cpu().numpy() for p in phis]
                stream.synchronize()
            with self.lock:
                self.groups += 1
                self.grouped_batches += len(nbs)
            for (batch, cols, extra), e, st, ph in zip(nbs, entries, sts, phs):
                resv = {"extra": extra}
                if st["status"] in (B.OK, B.NOT_CONVERGED):
                    self._answer(batch, cols, batch[0].graph_id, e, True, st, ph, resv)
                else:
                    with self.lock:
                        for r in batch:
                            self._reject(r, st["status"])
                with self.lock:
                    self.reserved -= resv["extra"]
                    resv["extra"] = 0.0
        finally:
            with self.lock:
                for batch, _, _ in nbs:
                    self.busy_graphs.discard(batch[0].graph_id)
                self.lock.notify_all()

    # --- driving a stream --------------------------------------------------------------
    def run(self, requests: list[Request], stall_timeout: float = 120.0) -> dict:
        """Releases the requests at their arrival times (seconds from now) and returns a
        summary once all are answered. Raises RuntimeError if no request completes for
        `stall_timeout` seconds while work is pending."""
        import sys

        streams = [torch.cuda.Stream() for _ in range(self.slots)]
        self.t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(s,), daemon=True) for s in streams]
        for w in workers:
            w.start()
        for req in sorted(requests, key=lambda r: r.arrival):
            delay = req.arrival - (time.perf_counter() - self.t0)
            if delay > 0:
                time.sleep(delay)
            self.submit(req)
        with self.lock:
            self.done = True
            self.lock.notify_all()
        last, last_t, shown = -1, time.perf_counter(), 0
        while any(w.is_alive() for w in workers):
            for w in workers:
                w.join(timeout=0.5)
            with self.lock:
                nres = len(self.results)
            if nres != last:
                last, last_t = nres, time.perf_counter()
                if self.progress_every and nres // self.progress_every > shown:
                    shown = nres // self.progress_every
                    print(f"[serve] {nres}/{len(requests)} answered", file=sys.stderr, flush=True)
            elif time.perf_counter() - last_t > stall_timeout:
                with self.lock:
                    self.done = True
                    self.queue.clear()
                raise RuntimeError(f"serving stalled: {nres}/{len(requests)} answered")
        wall = time.perf_counter() - self.t0
        return self.summary(wall)

    def summary(self, wall: float) -> dict:
        ok = [r for r in self.results if r.status in (B.OK, B.NOT_CONVERGED)]
        lat = np.array([r.latency for r in ok])
        hit = np.array([r.cache_hit for r in ok], dtype=bool)
        work = sum(self.graphs[r.graph_id].nnz_laplacian * r.phi.shape[0] for r in ok)

        def pct(x, q):
            return float(np.percentile(x, q)) if x.size else None

        return dict(requests=len(self.results), answered=len(ok), rejected=self.rejected,
                    wall_s=wall,
                    throughput_nnz_rhs_per_s=work / wall if wall > 0 else None,
                    p50_ms=pct(lat, 50) * 1e3 if lat.size else None,
                    p99_ms=pct(lat, 99) * 1e3 if lat.size else None,
                    hit_p50_ms=pct(lat[hit], 50) * 1e3 if hit.any() else None,
                    hit_p99_ms=pct(lat[hit], 99) * 1e3 if hit.any() else None,
                    miss_p50_ms=pct(lat[~hit], 50) * 1e3 if (~hit).any() else None,
                    miss_p99_ms=pct(lat[~hit], 99) * 1e3 if (~hit).any() else None,
                    setups=self.setups, evictions=self.evictions, overshoots=self.overshoots,
                    groups=self.groups, grouped_batches=self.grouped_batches,
                    mean_batch_columns=float(np.mean([r.batch_columns for r in ok]))
                    if ok else None,
                    max_relres=float(max(r.relres.max() for r in ok)) if ok else None,
                    max_resident_bytes=self.max_resident, budget_bytes=self.budget)

    def close(self):
        for e in self.cache.values():
            e["handle"].close()
        self.cache.clear()
        B.lamg_set_allocator()


def _pool_graph(args):
    """One graph of the synthetic pool (top level so that worker processes can run it)."""
    from . import inputs as I

    i, n, seed = args
    fam = i % 3
    if fam == 0:
        side = max(2, int(round(np.sqrt(n))))
        return I.grid2d(side, side, name=f"g{i}_grid{side}")
    if fam == 1:
        return I.random_geometric(n, 10.0, seed=seed * 1000 + i, name=f"g{i}_rgg{n}")
    return I.chung_lu(n, 2.3, 12.0, seed=seed * 1000 + i, name=f"g{i}_cl{n}")


def graph_pool(n_graphs: int = 16, nmin: float = 1e3, nmax: float = 1e6, seed: int = 0,
               workers: int = 1) -> dict:
    """A pool of 2D grids, random geometric graphs (mean degree 10) and Chung-Lu graphs
    (exponent 2.3, mean degree 12), n log-uniform in [nmin, nmax]; generated in `workers`
    processes when above 1."""
    rng = np.random.default_rng(seed)
    specs = [(i, int(round(10 ** rng.uniform(np.log10(nmin), np.log10(nmax)))), seed)
             for i in range(n_graphs)]
    if workers > 1:
        import concurrent.futures as cf
        import multiprocessing as mp

        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            graphs = list(ex.map(_pool_graph, specs))
    else:
        graphs = [_pool_graph(sp) for sp in specs]
    return {g.name: g for g in graphs}


def request_stream(graphs: dict, n_requests: int, rate: float, kmax: int = 32, seed: int = 0,
                   shared_rhs: bool = False) -> list:
    """Poisson arrivals at `rate` requests/s (rate <= 0: all at time 0) over the pool with
    Zipf(1) popularity (in pool order); each request has U{1..kmax} right-hand sides N(0,1).
    With `shared_rhs`, a request's block is a view into one kmax x n block per graph (at a
    random offset), which keeps host memory at one block per graph for long streams."""
    rng = np.random.default_rng(seed + 7919)
    names = list(graphs)
    pop = 1.0 / np.arange(1, len(names) + 1)
    pop /= pop.sum()
    blocks = {}
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        if rate > 0:
            t += rng.exponential(1.0 / rate)
        gid = names[rng.choice(len(names), p=pop)]
        k = int(rng.integers(1, kmax + 1))
        n = graphs[gid].n
        if shared_rhs:
            if gid not in blocks:
                blocks[gid] = np.random.default_rng(seed * 31 + len(blocks)).standard_normal(
                    (2 * kmax, n))
            o = int(rng.integers(0, kmax + 1))
            b = blocks[gid][o:o + k]
        else:
            b = rng.standard_normal((k, n))
        reqs.append(Request(rid, gid, b, t))
    return reqs


def synthetic_stream(n_requests: int, rate: float, n_graphs: int = 16, nmin: float = 1e3,
                     nmax: float = 1e6, kmax: int = 32, seed: int = 0):
    """A graph pool and a request stream over it (see graph_pool, request_stream).
    Returns (graphs, requests)."""
    graphs = graph_pool(n_graphs, nmin, nmax, seed)
    return graphs, request_stream(graphs, n_requests, rate, kmax, seed)


def main(argv=None) -> int:
    """Serving benchmark: a saturation run (every request at time 0) measures the capacity
    in requests/s; then one run per offered load (a fraction of that capacity) with
    Poisson arrivals. One JSON line per run."""
    import argparse
    import json
    import os
    import sys

    ap = argparse.ArgumentParser(description="LAMG+ serving stream on one GPU")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--graphs", type=int, default=12)
    ap.add_argument("--nmin", type=float, default=1e3)
    ap.add_argument("--nmax", type=float, default=1e6)
    ap.add_argument("--kmax", type=int, default=32)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--loads", default="0.5,0.8,1.0",
                    help="offered loads as fractions of the measured capacity")
    ap.add_argument("--rate", type=float, default=None,
                    help="run one stream at this offered rate (requests/s) instead")
    ap.add_argument("--log-batches", action="store_true")
    ap.add_argument("--reorder", action="store_true",
                    help="renumber each graph by the self-gated reverse Cuthill-McKee order")
    ap.add_argument("--smoother", type=int, default=0,
                    help="0: multicolour Gauss-Seidel; 1: Chebyshev on levels with > 32 colours; "
                         "2: block-Jacobi Gauss-Seidel on those levels")
    ap.add_argument("--hip-graphs", action="store_true",
                    help="replay each cycle of repeated (precision, columns) solves as a HIP graph")
    ap.add_argument("--group", type=int, default=0,
                    help="solve up to this many batches on different small graphs per "
                         "lamg_solve_group call (0: every batch on its own)")
    ap.add_argument("--preload", action="store_true",
                    help="build every graph's hierarchy before each stream (a warm cache)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    log = lambda *x: print("[serve]", *x, file=sys.stderr, flush=True)
    t = time.perf_counter()
    graphs = graph_pool(a.graphs, a.nmin, a.nmax, a.seed, workers=a.workers)
    nnz = sorted(g.nnz_laplacian for g in graphs.values())
    log(f"{len(graphs)} graphs in {time.perf_counter() - t:.1f}s, nnz(L) {nnz[0]}..{nnz[-1]}")

    def one(rate, tag):
        reqs = request_stream(graphs, a.requests, rate, a.kmax, a.seed, shared_rhs=True)
        srv = Server(graphs, hbm_budget=a.budget_gb * 1e9, slots=a.slots, smoother=a.smoother,
                     hip_graphs=a.hip_graphs, group=a.group, reorder=int(a.reorder))
        srv.progress_every = max(1, a.requests // 10)
        srv.log_batches = a.log_batches
        if a.preload:
            srv.preload(list(graphs))
            srv.setups = 0  # count only the setups the stream itself needed
        out = srv.run(reqs)
        srv.close()
        out.update(run=tag, offered_rate=rate if rate > 0 else None, requests_total=a.requests,
                   graphs=len(graphs), slots=a.slots, kmax=a.kmax, smoother=a.smoother,
                   hip_graphs=a.hip_graphs, group=a.group, preload=a.preload, reorder=a.reorder)
        out["answered_per_s"] = out["answered"] / out["wall_s"]
        print(json.dumps(out), flush=True)
        log(f"{tag}: {out['answered_per_s']:.2f} req/s p50 {out['p50_ms']:.1f} ms "
            f"p99 {out['p99_ms']:.1f} ms")
        return out

    if a.rate is not None:
        one(a.rate, f"rate{a.rate:g}")
        return 0
    cap = one(0.0, "saturation")["answered_per_s"]
    for f in (float(x) for x in a.loads.split(",") if x):
        one(f * cap, f"load{f:g}")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
