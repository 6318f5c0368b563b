"""The serving loop's admission and batching logic, driven by a host
executor on a simulated clock (no GPU): the memory budget is never exceeded,
queries are admitted in arrival order, no batch exceeds its size or the
number of launch slots, every query completes, and queries that arrive while
a batch runs are launched before it ends."""
import numpy as np
import pytest

import oracle
from paper_2307_15255_amd import serve as S


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def idle(self):
        self.t += 1e-4


class HostExecutor:
    """Each batch takes fixed + per-query time on the simulated clock."""

    def __init__(self, clock, fixed=2e-3, per_query=1e-3):
        self.clock, self.fixed, self.per_query = clock, fixed, per_query
        self.live = 0
        self.max_live = 0

    def mem_need(self, q):
        return 100 + 50 * len(q.dims)

    def launch(self, qs, slot):
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return [self.clock() + self.fixed + self.per_query * len(qs), qs]

    def launch_single(self, q):
        return self.launch([q], 0)

    def done(self, h):
        return self.clock() >= h[0]

    def finish(self, h):
        self.live -= 1


def make_queries(n, qps, seed=3):
    rng = np.random.default_rng(seed)
    qs = [S.random_query(rng, i) for i in range(n)]
    for q, t in zip(qs, S.poisson_arrivals(rng, n, qps)):
        q.arrival = float(t)
    return qs


@pytest.mark.parametrize("budget,slots,max_batch", [(10_000, 2, 64), (700, 3, 4), (300, 1, 8)])
def test_admission_and_batching(budget, slots, max_batch):
    clock = Clock()
    ex = HostExecutor(clock)
    qs = make_queries(300, qps=2000)
    rep = S.serve(qs, ex, budget, slots=slots, max_batch=max_batch, clock=clock, idle=clock.idle)
    assert set(rep.latency) == {q.qid for q in qs}
    assert all(v > 0 for v in rep.latency.values())
    assert rep.peak_bytes <= budget
    assert ex.max_live <= slots
    order = [qid for _, ids, _ in rep.batches for qid in ids]
    arrival = {q.qid: q.arrival for q in qs}
    assert order == sorted(order, key=lambda i: (arrival[i], i))  # FIFO admission
    assert all(len(ids) <= max_batch for _, ids, _ in rep.batches)
    assert all(nbytes <= budget for _, _, nbytes in rep.batches)
    for t, ids, _ in rep.batches:  # a batch holds only queries that had arrived
        assert all(arrival[i] <= t + 1e-12 for i in ids)


def test_batches_overlap_and_beat_one_at_a_time():
    """At a load the one-query-at-a-time loop cannot keep up with, later
    batches launch while earlier ones run, and p99 latency is lower."""
    qs = make_queries(400, qps=1500)
    c1 = Clock()
    served = S.serve(qs, HostExecutor(c1), 10_000, slots=2, max_batch=64, clock=c1, idle=c1.idle)
    c2 = Clock()
    alone = S.one_at_a_time(qs, HostExecutor(c2), clock=c2, idle=c2.idle)
    starts = [t for t, _, _ in served.batches]
    ends = sorted(served.finish[ids[-1]] for _, ids, _ in served.batches)
    assert any(s < e for s, e in zip(starts[1:], ends[:-1]))  # a launch before an earlier batch ended
    assert served.percentile(99) < alone.percentile(99)
    assert alone.percentile(50) >= 3e-3 - 1e-9  # every lone query takes fixed + per-query time


def test_hold_batches_lone_queries_while_busy():
    """With hold, a query that would launch alone beside a running batch
    waits (at most `hold` after its arrival) for company: batches grow, no
    launch of a lone query beside a running batch happens before its hold
    ran out unless another query came, and every query completes."""
    qs = make_queries(300, qps=600)
    hold = 1.5e-3
    c1 = Clock()
    plain = S.serve(qs, HostExecutor(c1), 10_000, slots=2, clock=c1, idle=c1.idle)
    c2 = Clock()
    held = S.serve(qs, HostExecutor(c2), 10_000, slots=2, hold=hold, clock=c2, idle=c2.idle)
    assert set(held.latency) == {q.qid for q in qs}
    assert len(held.batches) < len(plain.batches)
    arrival = {q.qid: q.arrival for q in qs}
    finish = [(t, held.finish[ids[0]]) for t, ids, _ in held.batches]
    for t, ids, _ in held.batches:
        busy = any(s < t < f for s, f in finish if s != t)
        if busy and len(ids) == 1:
            assert t - arrival[ids[0]] >= hold - 2e-4


def test_oversized_query_is_rejected_alone():
    """A query that can never fit the memory limit is rejected by itself;
    the others are served."""
    clock = Clock()
    qs = make_queries(40, 500)
    ex = HostExecutor(clock)
    limit = 100 + 50 * 3  # queries with four dimensions need more
    rep = S.serve(qs, ex, budget_bytes=limit, clock=clock, idle=clock.idle)
    big = {q.qid for q in qs if ex.mem_need(q) > limit}
    assert big and set(rep.rejected) == big
    assert all("out of memory" in r for r in rep.rejected.values())
    assert set(rep.latency) == {q.qid for q in qs} - big
    assert rep.peak_bytes <= limit


def test_queries_time_out_while_waiting():
    """Under an overload with one slot, queries still waiting after the
    timeout are dropped; every query is either served or dropped, and no
    served query waited past the timeout before its launch."""
    clock = Clock()
    qs = make_queries(200, qps=5000)
    rep = S.serve(qs, HostExecutor(clock, fixed=5e-3), 10_000, slots=1, max_batch=4, timeout=0.02, clock=clock,
                  idle=clock.idle)
    assert rep.timed_out and rep.latency
    assert set(rep.timed_out) | set(rep.latency) == {q.qid for q in qs}
    assert not set(rep.timed_out) & set(rep.latency)
    assert all(w > 0.02 for w in rep.timed_out.values())
    arrival = {q.qid: q.arrival for q in qs}
    for t, ids, _ in rep.batches:
        assert all(t - arrival[i] <= 0.02 + 1e-9 for i in ids)


def test_queries_are_valid_problems(oracle_lib):
    """Random queries over a small resident star are well-formed join
    problems (2-5 tables, int32 or int64 key pairs, 1-2 predicates) that the
    oracle runs."""
    res = S.ResidentStar(seed=2, n_fact=5_000, dims=(800, 300, 40, 25), device=None)
    rng = np.random.default_rng(8)
    for i in range(12):
        q = S.random_query(rng, i)
        prob, dev = res.problem(q)
        assert dev is None
        assert 2 <= prob.n_tables <= 5 and 1 <= len(prob.preds) <= 2
        for u, uc, v, vc in prob.edges:
            assert prob.columns[u][uc].dtype == prob.columns[v][vc].dtype
        ref = oracle.transfer(prob)
        assert ref.counts[0] <= 5_000
