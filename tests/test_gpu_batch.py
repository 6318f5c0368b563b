"""GPU parity of the batched transfer (pt_batch_*): every problem of a batch
ends with the bitmaps and counts the oracle computes for it alone, whether
the batch runs eagerly or as its captured graph, replayed several times with
other GPU work in between."""
import os
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_bitmaps_equal, say
from paper_2307_15255_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = ["chain", "star", "tree", "cycle", "parallel", "forest"]


@pytest.fixture(scope="module")
def pt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_15255_amd import pt as ptmod
    return ptmod


def check_against_oracle(pt, bt, probs, params, which=None, threads=1):
    counts = [c.cpu().numpy() for c in bt.counts]
    for i in (range(len(probs)) if which is None else which):
        p = params[i]
        ref = oracle.transfer(probs[i], p.block_bits, p.k, p.bits_per_key, threads=threads)
        for t in range(probs[i].n_tables):
            assert_bitmaps_equal(bt.bitmap(i, t), ref.bitmaps[t], f"problem {i} ({probs[i].label}) table {t}")
            assert counts[i][t] == ref.counts[t], (i, t)


def mixed_params(pt, n, rng):
    choices = [(512, 3, 10), (256, 3, 8), (512, 4, 12), (1024, 2, 16), (64, 3, 10)]
    return [pt.params(*choices[int(rng.integers(len(choices)))]) for _ in range(n)]


def test_tiny_graphs_every_shape(pt):
    """Thirty random graphs of every shape (cycles, forests, parallel edges)
    with mixed parameters, in one batch."""
    rng = np.random.default_rng(31)
    probs = [W.tiny_random(np.random.default_rng(70_000 + s), SHAPES[s % 6]) for s in range(30)]
    ps = mixed_params(pt, len(probs), rng)
    bt = pt.Batch([pt.DeviceProblem(p) for p in probs], ps)
    say("batch tiny eager")
    bt.run(eager=True)
    torch.cuda.synchronize()
    check_against_oracle(pt, bt, probs, ps)


def test_outer_join_edges(pt):
    """Random graphs of every shape with outer-join edges (Sec. 3.4), in one
    batch: every problem gets the oracle's bits."""
    probs = [W.tiny_random(np.random.default_rng(96_000 + s), SHAPES[s % 6], outer=0.6) for s in range(30)]
    ps = [pt.params(512, 3, 6)] * len(probs)
    bt = pt.Batch([pt.DeviceProblem(p) for p in probs], ps)
    say("batch outer")
    bt.run(eager=True)
    torch.cuda.synchronize()
    check_against_oracle(pt, bt, probs, ps)


def test_graph_replays_match_eager(pt):
    """A batch of chains and stars of 1 k to 200 k rows: the eager run and
    three replays of the captured graph (with unrelated GPU work and a
    synchronisation between them) all give the oracle's bits."""
    probs = W.batch(seed=5, n_problems=24, lo=1_000, hi=200_000)
    rng = np.random.default_rng(5)
    ps = mixed_params(pt, len(probs), rng)
    bt = pt.Batch([pt.DeviceProblem(p) for p in probs], ps)
    n_launch, rows = bt.info()
    say("batch small: launches", n_launch, "rows probed", rows)
    bt.run(eager=True)
    torch.cuda.synchronize()
    check_against_oracle(pt, bt, probs, ps)
    eager = [[b.clone() for b in bms] for bms in bt.bitmaps]
    noise = torch.ones(1 << 20, device="cuda")
    for r in range(3):
        for bms in bt.bitmaps:
            for b in bms:
                b.fill_(-1)
        bt.run()
        torch.cuda.synchronize()
        noise.mul_(1.5).add_(r)  # other work between replays
        torch.cuda.synchronize()
        for i, bms in enumerate(bt.bitmaps):
            for t, b in enumerate(bms):
                assert torch.equal(b, eager[i][t]), (r, i, t)


def test_batch_equals_single_transfers(pt):
    """Each problem of a batch gets the bits pt_transfer gives it alone."""
    probs = W.batch(seed=9, n_problems=16, lo=10_000, hi=400_000)
    dps = [pt.DeviceProblem(p) for p in probs]
    bt = pt.Batch(dps)
    bt.run()
    torch.cuda.synchronize()
    for i, dp in enumerate(dps):
        tr = pt.Transfer(dp)
        tr.run()
        torch.cuda.synchronize()
        for t in range(dp.n_tables):
            assert torch.equal(bt.bitmaps[i][t], tr.bitmaps[t]), (i, t)
        assert torch.equal(bt.counts[i], tr.counts), i


@pytest.mark.timeout(400)
def test_full_batch(pt):
    """256 problems with tables of 10 k to 5 M rows (677 M rows in all), as
    one persistent launch: every problem's bitmaps and counts against the
    oracle (its row split over the host's cores, bit-exact with one
    thread), and every problem's counts against pt_transfer on its own."""
    t0 = time.time()
    probs = W.batch(seed=1)
    say("full batch generated", round(time.time() - t0, 1), "s")
    dps = [pt.DeviceProblem(p) for p in probs]
    bt = pt.Batch(dps)
    bt.run()
    torch.cuda.synchronize()
    say("full batch ran", round(time.time() - t0, 1), "s")
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    check_against_oracle(pt, bt, probs, bt.params, threads=threads)
    say("full batch oracle ok", round(time.time() - t0, 1), "s")
    for i, dp in enumerate(dps):
        tr = pt.Transfer(dp)
        tr.run()
        torch.cuda.synchronize()
        assert torch.equal(bt.counts[i], tr.counts), i
        del tr
    say("full batch counts ok", round(time.time() - t0, 1), "s")


@pytest.mark.parametrize("sel_hi", [0.5, 0.02])
def test_shared_scans(pt, sel_hi):
    """Forty queries joining one resident 2 M-row fact table through int32
    and int64 key columns, in one batch: their fact probes run as shared
    scans (groups of at most sixteen problems and four key columns; the
    timeline shows shared items) and every problem ends with the oracle's
    bits, as it does without them. With predicates keeping
    up to 50 % some groups' filters exceed LDS (members probed one by one);
    with at most 2 % every group's filters fit (one pass for the group)."""
    from paper_2307_15255_amd import serve as S
    res = S.ResidentStar(seed=6, n_fact=2_000_000, dims=(300_000, 20_000, 1_000, 25))
    rng = np.random.default_rng(3)
    probs, dps = [], []
    for i in range(40):
        prob, dev = res.problem(S.random_query(rng, i, sel_hi=sel_hi))
        probs.append(prob)
        dps.append(pt.DeviceProblem(prob, columns=dev))
    os.environ["PT_BATCH_TIMELINE"] = "1"
    try:
        bt = pt.Batch(dps, [pt.params(flags=pt.PT_FLAG_SHARED_SCAN)] * len(dps))
    finally:
        del os.environ["PT_BATCH_TIMELINE"]
    say("shared batch")
    bt.run(eager=True)
    torch.cuda.synchronize()
    bt.check_status()
    tl, _ = bt.timeline()
    shared_kind = 10
    assert int((tl[:, 2] == shared_kind).sum()) > 0
    check_against_oracle(pt, bt, probs, bt.params)
    solo = pt.Batch(dps, [pt.params()] * len(dps))
    solo.run()
    torch.cuda.synchronize()
    for i in range(len(dps)):
        for t in range(dps[i].n_tables):
            assert torch.equal(bt.bitmaps[i][t], solo.bitmaps[i][t]), (i, t)
        assert torch.equal(bt.counts[i], solo.counts[i]), i


def test_tile_search_keeps_bits(pt, tmp_path, monkeypatch):
    """The rows-per-item search times the batch with every candidate and
    keeps the fastest (a second call reuses the saved choice); every
    candidate gives the same bits, the oracle's."""
    from paper_2307_15255_amd import autotune as A
    monkeypatch.setattr(A, "COST_DIR", str(tmp_path))
    probs = W.batch(seed=12, n_problems=24, lo=10_000, hi=400_000)
    dps = [pt.DeviceProblem(p) for p in probs]
    ps = [pt.params(512, 3, 10)] * len(probs)
    say("tile search")
    out, rec = A.tune_tiles(dps, ps, reps=3)
    assert set(rec["measured_ms"]) == set(A.TILE_ROWS)
    assert rec["tile_rows"] == min(A.TILE_ROWS, key=lambda t: (rec["measured_ms"][t], t))
    again, rec2 = A.tune_tiles(dps, ps)
    assert rec2["measured_ms"] is None and rec2["tile_rows"] == rec["tile_rows"]
    results = []
    for tr in (min(A.TILE_ROWS), max(A.TILE_ROWS)):
        bt = pt.Batch(dps, [pt.params(512, 3, 10, tile_rows=tr)] * len(dps))
        bt.run()
        torch.cuda.synchronize()
        bt.check_status()
        results.append(bt)
    for i in range(len(dps)):
        for t in range(dps[i].n_tables):
            assert torch.equal(results[0].bitmaps[i][t], results[1].bitmaps[i][t]), (i, t)
    check_against_oracle(pt, results[1], probs, [pt.params(512, 3, 10)] * len(probs), which=[0, 7, 23])
