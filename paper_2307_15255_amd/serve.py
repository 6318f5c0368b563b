"""Serving transfer queries over tables resident in HBM.

A query asks for the transfer phase over a subgraph of a resident star
schema (the fact table and one to four dimensions, each edge on its int32 or
int64 key columns, one or two range predicates). The server keeps the tables
on the GPU and runs a request loop:

  admission   queries wait in arrival order; the head is admitted when the
              memory its filters, bitmaps and task tables need fits in what
              the in-flight batches leave of the budget (a ledger of bytes);
              a query that could never fit is rejected on its own (out of
              memory) and one that waits longer than its timeout is dropped,
              without holding up the others;
  batching    every admitted query that is waiting when a launch slot is
              free goes into one batch (pt_batch: one persistent launch for
              all of its queries, whose probes of the resident fact table
              share one scan of its key columns);
  overlap     up to `slots` batches are in flight at once, each on its own
              stream: queries that arrive while others run are admitted and
              launched as soon as a slot and memory free up.

The loop is written against a small executor interface (mem_need, launch,
done, finish) so its admission and batching logic also runs, with a host
executor, where there is no GPU. The paper evaluates one query at a time;
serving is an addition.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import workloads as W


@dataclass
class Query:
    qid: int
    dims: list[int]                 # dimensions joined to the fact table
    wide: list[bool]                # per joined dimension: int64 key columns
    preds: list[tuple[int, int]]    # (dimension, threshold): attr < threshold
    arrival: float = 0.0            # seconds after the start of the stream


def random_query(rng: np.random.Generator, qid: int, n_dims: int = 4, wide_dims: tuple[int, ...] = (0, 1),
                 sel_lo: float = 0.001, sel_hi: float = 0.5) -> Query:
    """A fact table plus 1-4 distinct dimensions (2-5 tables); the int64 key
    variant on each edge that has one with probability 1/2; one or two
    predicates on joined dimensions with selectivity log-uniform on
    [sel_lo, sel_hi]."""
    k = int(rng.integers(1, n_dims + 1))
    dims = sorted(int(d) for d in rng.choice(n_dims, size=k, replace=False))
    wide = [d in wide_dims and bool(rng.integers(2)) for d in dims]
    n_pred = min(len(dims), int(rng.integers(1, 3)))
    preds = []
    for d in rng.choice(dims, size=n_pred, replace=False):
        sel = math.exp(rng.uniform(math.log(sel_lo), math.log(sel_hi)))
        preds.append((int(d), max(1, int(round(sel * 1_000_000)))))
    return Query(qid, dims, wide, sorted(preds))


def poisson_arrivals(rng: np.random.Generator, n: int, qps: float) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


class ResidentStar:
    """The star schema (fact with int32 foreign keys k0..k3, dimensions with
    primary key pk and attribute attr uniform on [0, 10^6)) plus int64 twins
    of the keys of the edges in `wide_dims`, on the host and in HBM."""

    def __init__(self, seed: int = 1, n_fact: int = 100_000_000, dims: tuple[int, ...] = W.STAR_DIMS,
                 wide_dims: tuple[int, ...] = (0, 1), device: str | None = "cuda"):
        base = W.star(seed=seed, n_fact=n_fact, dims=dims, keeps=(None,) * len(dims), payload=0)
        self.dims = dims
        self.wide_dims = wide_dims
        self.host = [dict(c) for c in base.columns]
        for d in wide_dims:
            self.host[0][f"k{d}_64"] = self.host[0][f"k{d}"].astype(np.int64)
            self.host[d + 1]["pk64"] = self.host[d + 1]["pk"].astype(np.int64)
        self.dev = None
        if device is not None:
            import torch
            self.dev = [{c: torch.from_numpy(np.ascontiguousarray(a)).to(device) for c, a in cols.items()}
                        for cols in self.host]

    def problem(self, q: Query) -> tuple[W.Problem, list | None]:
        """The query as a join problem, with the device columns in the same
        order (None without a device)."""
        names, cols, dev, edges, preds = ["F"], [{}], [{}], [], []
        for i, (d, wide) in enumerate(zip(q.dims, q.wide)):
            fk, pk = (f"k{d}_64", "pk64") if wide else (f"k{d}", "pk")
            cols[0][fk] = self.host[0][fk]
            names.append(f"D{d}")
            cols.append({pk: self.host[d + 1][pk], "attr": self.host[d + 1]["attr"]})
            if self.dev is not None:
                dev[0][fk] = self.dev[0][fk]
                dev.append({pk: self.dev[d + 1][pk], "attr": self.dev[d + 1]["attr"]})
            edges.append((0, fk, i + 1, pk))
        for d, thr in q.preds:
            preds.append((q.dims.index(d) + 1, "attr", "lt", thr, 0))
        label = f"query {q.qid}: F + {['D%d%s' % (d, '/64' if w else '') for d, w in zip(q.dims, q.wide)]}"
        return W.Problem(names, cols, edges, preds, label=label), (dev if self.dev is not None else None)


@dataclass
class Report:
    latency: dict = field(default_factory=dict)    # qid -> seconds from arrival to results ready
    service: dict = field(default_factory=dict)    # qid -> seconds from launch to results ready (alone)
    finish: dict = field(default_factory=dict)     # qid -> seconds after start
    batches: list = field(default_factory=list)    # (launch time, [qid], bytes)
    rejected: dict = field(default_factory=dict)   # qid -> reason (needs more memory than a batch may hold)
    timed_out: dict = field(default_factory=dict)  # qid -> seconds waited when it was dropped
    peak_bytes: int = 0
    wall: float = 0.0
    launch_host_s: float = 0.0  # host time spent in executor.launch (planning and enqueueing batches)

    def percentile(self, p: float) -> float:
        """Latency percentile over the queries that completed."""
        return float(np.percentile(np.array(list(self.latency.values())), p))


def serve(queries: list[Query], executor, budget_bytes: int, slots: int = 2, max_batch: int = 64,
          batch_bytes: int | None = None, timeout: float | None = None, hold: float = 0.0,
          clock=time.perf_counter, idle=lambda: time.sleep(50e-6)) -> Report:
    """Runs the request loop over `queries` (sorted by arrival) on
    `executor` and reports every query's latency. budget_bytes bounds the
    memory of all batches in flight, batch_bytes (default: the budget) that
    of one batch. A query needing more than either is rejected when it
    arrives (Report.rejected, the library's out-of-memory case); a query
    still waiting `timeout` seconds after its arrival is dropped
    (Report.timed_out). Neither stops the others. hold > 0: while another
    batch is running, a query waiting alone is held up to `hold` seconds
    after its arrival for another one to batch with."""
    rep = Report()
    cap = budget_bytes if batch_bytes is None else min(batch_bytes, budget_bytes)
    need = {q.qid: executor.mem_need(q) for q in queries}
    pending = collections.deque(sorted(queries, key=lambda q: q.arrival))
    waiting: collections.deque[Query] = collections.deque()
    inflight = []  # (handle, queries, bytes, slot)
    free_slots = list(range(slots))
    used = 0
    t0 = clock()
    while pending or waiting or inflight:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            q = pending.popleft()
            if need[q.qid] > cap:
                rep.rejected[q.qid] = f"out of memory: needs {need[q.qid]} bytes, a batch may hold {cap}"
            else:
                waiting.append(q)
        if timeout is not None:
            while waiting and now - waiting[0].arrival > timeout:
                q = waiting.popleft()
                rep.timed_out[q.qid] = now - q.arrival
        progressed = False
        for item in list(inflight):
            handle, qs, nbytes, slot = item
            if executor.done(handle):
                t = clock() - t0
                executor.finish(handle)
                for q in qs:
                    rep.finish[q.qid] = t
                    rep.latency[q.qid] = t - q.arrival
                used -= nbytes
                free_slots.append(slot)
                inflight.remove(item)
                progressed = True
        held = (hold > 0 and inflight and len(waiting) == 1 and pending
                and now - waiting[0].arrival < hold)
        if waiting and free_slots and not held:
            take, nbytes = [], 0
            while (waiting and len(take) < max_batch and used + nbytes + need[waiting[0].qid] <= budget_bytes
                   and nbytes + need[waiting[0].qid] <= cap):
                q = waiting.popleft()
                take.append(q)
                nbytes += need[q.qid]
            if take:
                slot = free_slots.pop(0)
                used += nbytes
                rep.peak_bytes = max(rep.peak_bytes, used)
                rep.batches.append((clock() - t0, [q.qid for q in take], nbytes))
                t_launch = clock()
                inflight.append((executor.launch(take, slot), take, nbytes, slot))
                rep.launch_host_s += clock() - t_launch
                progressed = True
        if not progressed:
            idle()
    rep.wall = clock() - t0
    return rep


def one_at_a_time(queries: list[Query], executor, clock=time.perf_counter,
                  idle=lambda: time.sleep(50e-6)) -> Report:
    """The baseline: queries in arrival order, each run alone once the
    previous one has finished."""
    rep = Report()
    t0 = clock()
    for q in sorted(queries, key=lambda q: q.arrival):
        while clock() - t0 < q.arrival:
            idle()
        start = clock() - t0
        h = executor.launch_single(q)
        while not executor.done(h):
            idle()
        t = clock() - t0
        executor.finish(h)
        rep.finish[q.qid] = t
        rep.latency[q.qid] = t - q.arrival
        rep.service[q.qid] = t - start
    rep.wall = clock() - t0
    return rep


class GpuExecutor:
    """Runs batches on `slots` streams: a batch's small queries as one
    pt_batch (one persistent launch), its large ones (at least large_rows
    rows in their tables, which fill the GPU by themselves) as pt_transfer
    calls one after the other on the same stream. Single queries run with
    pt_transfer on a stream of their own. Each slot owns a workspace arena of
    `arena_bytes` allocated once (the workspace of whatever runs on the slot
    is a prefix of it; serve with batch_bytes <= arena_bytes), and single
    queries share one more arena, so the loop itself allocates nothing but
    the queries' bitmaps. Keeps every query's bitmaps and counts when
    `keep`."""

    def __init__(self, resident: ResidentStar, params=None, slots: int = 2, keep: bool = False,
                 arena_bytes: int = 1 << 30, single_arena_bytes: int = 0, large_rows: int = 8_000_000):
        import torch
        from . import pt
        self.torch, self.pt = torch, pt
        self.resident = resident
        self.params = params if params is not None else pt.params()
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.single_stream = torch.cuda.Stream()
        self.arenas = [torch.empty(arena_bytes, dtype=torch.uint8, device="cuda") for _ in range(slots)]
        self.single_arena = (torch.empty(single_arena_bytes, dtype=torch.uint8, device="cuda")
                             if single_arena_bytes else None)
        self.keep = keep
        self.large_rows = large_rows
        self.results: dict[int, tuple[list, object]] = {}
        self._dp_cache: dict[int, object] = {}

    def device_problem(self, q: Query):
        dp = self._dp_cache.get(q.qid)
        if dp is None:
            prob, dev = self.resident.problem(q)
            dp = self.pt.DeviceProblem(prob, columns=dev)
            self._dp_cache[q.qid] = dp
        return dp

    def single_need(self, q: Query) -> int:
        """Workspace pt_transfer needs for the query alone."""
        return self.pt.pt_transfer_workspace_size(self.device_problem(q), self.params)

    def mem_need(self, q: Query) -> int:
        dp = self.device_problem(q)
        ws = max(self.pt.pt_batch_workspace_size([dp], [self.params]), self.single_need(q))
        bitmaps = sum(8 * self.pt.bitmap_words(n) for n in dp.n_rows) + 8 * dp.n_tables
        return ws + bitmaps

    def is_large(self, q: Query) -> bool:
        """A query whose tables hold at least large_rows rows: its own
        launches already fill the GPU, so it runs as its own transfer (the
        persistent batch kernel pays off for many small problems)."""
        return sum(self.device_problem(q).n_rows) >= self.large_rows

    def launch(self, qs: list[Query], slot: int):
        """One batch on the slot's stream: its small queries as one pt_batch,
        then its large queries one transfer after the other (the arena is
        their shared workspace: they run in stream order)."""
        torch = self.torch
        s = self.streams[slot]
        small = [q for q in qs if not self.is_large(q)]
        large = [q for q in qs if self.is_large(q)]
        parts = []
        with torch.cuda.stream(s):
            if small:
                dps = [self.device_problem(q) for q in small]
                bt = self.pt.Batch(dps, [self.params] * len(dps), stream=s, ws=self.arenas[slot])
                bt.run(stream=s, eager=True)
                parts.append(("batch", bt, small))
            for q in large:
                tr = self.pt.Transfer(self.device_problem(q), self.params, ws=self.arenas[slot])
                tr.run(stream=s)
                parts.append(("single", tr, [q]))
            ev = torch.cuda.Event()
            ev.record(s)
        return (parts, ev, qs, s)

    def launch_single(self, q: Query):
        torch = self.torch
        s = self.single_stream
        with torch.cuda.stream(s):
            tr = self.pt.Transfer(self.device_problem(q), self.params, ws=self.single_arena)
            tr.run(stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return ([("single", tr, [q])], ev, [q], s)

    def done(self, h) -> bool:
        return h[1].query()

    def finish(self, h) -> None:
        parts, _, _, stream = h
        for kind, obj, qs in parts:
            if self.keep:
                # Copied on the stream the results were made on: their blocks
                # go back to that stream's pool when `obj` is dropped, so the
                # next launch there cannot reuse them before the copies ran.
                with self.torch.cuda.stream(stream):
                    if kind == "batch":
                        for i, q in enumerate(qs):
                            self.results[q.qid] = ([b.clone() for b in obj.bitmaps[i]], obj.counts[i].clone())
                    else:
                        self.results[qs[0].qid] = ([b.clone() for b in obj.bitmaps], obj.counts.clone())
            if kind == "batch":
                obj.close()
