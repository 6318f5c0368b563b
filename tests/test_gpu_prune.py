"""GPU parity of transfer path pruning (PT_FLAG_PRUNE; Sec. 3.2, "Transfer
Path Pruning", with the rule the oracle implements: a non-empty table that
still holds every row sends no filter). Every bitmap and count, and every
filter of both passes (a pruned one has a block count of zero), equal the
pruning oracle's
on random graphs of every shape, with outer-join edges, with exact filters,
on the authored worked example, on the scaled snowflake and star, and in a
batch. The snowflake shows what pruning skips: its unfiltered D4 sends
nothing, so D1 receives nothing and sends nothing either."""
import numpy as np
import pytest
import torch

import goldens
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


def check_pruned(pt, prob, B=512, k=3, bpk=10, exact=False, filters=True, threads=1):
    flags = pt.PT_FLAG_PRUNE | (pt.PT_FLAG_EXACT if exact else 0)
    dp = pt.DeviceProblem(prob)
    tr = pt.Transfer(dp, pt.params(B, k, bpk, flags))
    tr.run()
    tr.check_status()
    kind = oracle.EXACT if exact else oracle.BLOOM
    dump = filters and not exact
    ref = oracle.transfer(prob, B, k, bpk, kind=kind, dump_filters=dump, prune=True, threads=threads)
    counts = tr.counts.cpu().numpy()
    for t in range(prob.n_tables):
        assert_bitmaps_equal(tr.bitmap(t), ref.bitmaps[t], f"{prob.label} table {t}")
        assert counts[t] == ref.counts[t], (prob.label, t)
    if dump:
        for (p, e), words in ref.filters.items():
            if ref.edge_src[(p, e)] == 0xFFFFFFFF:  # an outer join blocks this direction
                continue
            g_words, g_nb, g_builder = tr.filter(p + 1, e)
            assert g_builder == ref.edge_src[(p, e)]
            assert g_nb == ref.filter_nb[(p, e)], (prob.label, p, e)
            assert np.array_equal(g_words, words), (prob.label, p, e)
    return tr, ref


@pytest.mark.parametrize("shape", SHAPES)
def test_prune_tiny_random_graphs(pt, shape):
    for s in range(20):
        prob = W.tiny_random(np.random.default_rng(120_000 + 100 * SHAPES.index(shape) + s), shape)
        say("prune tiny", shape, s)
        check_pruned(pt, prob)


@pytest.mark.parametrize("shape", SHAPES)
def test_prune_outer_and_exact(pt, shape):
    for s in range(10):
        rng = np.random.default_rng(130_000 + 100 * SHAPES.index(shape) + s)
        prob = W.tiny_random(rng, shape, outer=0.5)
        say("prune outer", shape, s)
        check_pruned(pt, prob, 512, 3, 6)
        say("prune exact", shape, s)
        check_pruned(pt, prob, exact=True)


@pytest.mark.parametrize("exact", [False, True])
def test_prune_worked_example(pt, exact):
    prob, spec = goldens.load("prune_chain.json")
    tr, _ = check_pruned(pt, prob, 512, 8, 64, exact=exact)
    for name, rows in spec["expect_pruned_final_rows_1based"].items():
        t = prob.table(name)
        bits = tr.bitmap(t)
        got = {r for r in range(prob.n_rows(t)) if (int(bits[r // 64]) >> (r % 64)) & 1}
        assert got == {r - 1 for r in rows}, name


def test_prune_snowflake_scaled(pt):
    prob = W.snowflake(seed=4, scale=0.01)
    say("prune snowflake 1%")
    tr, ref = check_pruned(pt, prob, 512, 3, 12)
    d4, d1, f = prob.table("D4"), prob.table("D1"), prob.table("F")
    fwd = {(prob.edges[e][0], prob.edges[e][2]): e for e in range(len(prob.edges))}
    e41 = fwd.get((d1, d4), fwd.get((d4, d1)))
    e1f = fwd.get((f, d1), fwd.get((d1, f)))
    # forward pass: neither D4 nor D1 lost a row, so neither sends a filter
    assert tr.filter(1, e41)[1] == 0 and tr.filter(1, e1f)[1] == 0
    # backward pass: the fact table did lose rows, so its filters go out
    assert tr.filter(2, e1f)[1] > 0


def test_prune_star_scaled(pt):
    prob = W.star(seed=5, n_fact=1_000_003, dims=(200_000, 20_000, 1_000, 25), payload=0)
    say("prune star 1M")
    check_pruned(pt, prob, 512, 3, 10)


def test_prune_in_a_batch(pt):
    """Thirty random graphs with pruning, the three-table chain and a
    200 k-row star, in one batch (an eager run, then the captured graph):
    every problem gets the pruning oracle's bits."""
    probs = [W.tiny_random(np.random.default_rng(140_000 + s), SHAPES[s % 6]) for s in range(30)]
    probs += [W.chain(seed=3), W.star(seed=6, n_fact=200_000, dims=(20_000, 2_000, 100, 25), payload=0)]
    ps = [pt.params(512, 3, 10, pt.PT_FLAG_PRUNE)] * len(probs)
    bt = pt.Batch([pt.DeviceProblem(p) for p in probs], ps)
    say("prune batch")
    bt.run(eager=True)
    bt.run()
    torch.cuda.synchronize()
    bt.check_status()
    counts = [c.cpu().numpy() for c in bt.counts]
    for i, prob in enumerate(probs):
        ref = oracle.transfer(prob, 512, 3, 10, prune=True)
        for t in range(prob.n_tables):
            assert_bitmaps_equal(bt.bitmap(i, t), ref.bitmaps[t], f"problem {i} ({prob.label}) table {t}")
            assert counts[i][t] == ref.counts[t], (i, t)
