"""GPU parity of pt_transfer against the oracle: every table's bitmap and
count, and the words of every filter of both passes, bit for bit, on random
small join graphs of every shape, the worked examples, the three-table chain
and the star schema up to its full size (100 M fact rows)."""
import time

import numpy as np
import pytest
import torch

import goldens
import oracle
import refcheck as rc
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


def check_transfer(pt, prob, B=512, k=3, bpk=10, filters=True, runs=1, flags=0, **layout):
    dp = pt.DeviceProblem(prob)
    tr = pt.Transfer(dp, pt.params(B, k, bpk, flags, **layout))
    for _ in range(runs):
        tr.run()
    tr.check_status()  # waits for the stream; no kernel reported an overflow
    ref = oracle.transfer(prob, B, k, bpk, dump_filters=filters)
    counts = tr.counts.cpu().numpy()
    for t in range(prob.n_tables):
        assert_bitmaps_equal(tr.bitmap(t), ref.bitmaps[t], f"{prob.label} table {t}")
        assert counts[t] == ref.counts[t], (prob.label, t)
    if filters:
        for (p, e), words in ref.filters.items():
            if ref.edge_src[(p, e)] == 0xFFFFFFFF:  # an outer join blocks this edge in this pass
                with pytest.raises(pt.PtError):
                    tr.filter(p + 1, e)
                continue
            g_words, g_nb, g_builder = tr.filter(p + 1, e)
            assert g_builder == ref.edge_src[(p, e)]
            assert g_nb == ref.filter_nb[(p, e)], (prob.label, p, e)
            assert np.array_equal(g_words, words), (prob.label, p, e)
    return tr, ref


@pytest.mark.parametrize("shape", SHAPES)
def test_tiny_random_graphs(pt, shape):
    for s in range(25):
        prob = W.tiny_random(np.random.default_rng(50_000 + 100 * SHAPES.index(shape) + s), shape)
        say("tiny", shape, s)
        check_transfer(pt, prob)


@pytest.mark.parametrize("B,k,bpk", [(32, 1, 2), (64, 3, 8), (1024, 8, 16), (256, 3, 10)])
def test_parameters(pt, B, k, bpk):
    for s in range(6):
        prob = W.tiny_random(np.random.default_rng(777 + s), SHAPES[s % 6], max_rows=300, domain=64)
        say("params", B, k, bpk, s)
        check_transfer(pt, prob, B, k, bpk)


@pytest.mark.parametrize("layout", [dict(probe_order=1), dict(lds_budget=64), dict(lds_budget=4096, probe_order=1),
                                    dict(hash_version=0)])
def test_layout_parameters_keep_bits(pt, layout):
    """probe order, LDS staging budget (filters read from global memory when
    they do not fit) and the hash-version alias change no bit."""
    for s in range(6):
        prob = W.tiny_random(np.random.default_rng(4242 + s), SHAPES[s % 6], max_rows=3000, domain=500)
        say("layout", layout, s)
        check_transfer(pt, prob, **layout)
    prob = W.star(seed=3, n_fact=300_000, dims=(20_000, 2_000, 100, 25))
    say("layout star", layout)
    check_transfer(pt, prob, **layout)


@pytest.mark.parametrize("name", ["fig2_transform.json", "fig3_chain.json"])
def test_worked_examples(pt, name):
    prob, spec = goldens.load(name)
    tr, _ = check_transfer(pt, prob, 512, 8, 64)
    if "expect_final_rows_1based" in spec:
        for tname, rows in spec["expect_final_rows_1based"].items():
            t = prob.table(tname)
            assert rc.bits_to_rows(tr.bitmap(t), prob.n_rows(t)) == {r - 1 for r in rows}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_chain_config(pt, seed):
    """Three-table chain R 1000 - S 10000 - T 1000, int32 keys on [0, 2000),
    10 % predicate on R, B = 512, k = 3, 10 bits per key."""
    say("chain", seed)
    check_transfer(pt, W.chain(seed), runs=2)


@pytest.mark.parametrize("n_fact", [1_000_003, 10_000_000])
def test_star_scaled(pt, n_fact):
    prob = W.star(seed=n_fact % 7 + 1, n_fact=n_fact, payload=0)
    say("star", n_fact)
    check_transfer(pt, prob)


def test_star_full_size(pt):
    """The full star schema: 100 M fact rows, 4 int32 foreign keys into
    dimensions of 2 M, 200 k, 10 k and 25 rows, predicates keeping 1 % and
    20 %; the whole of every bitmap and filter against the oracle."""
    t0 = time.time()
    prob = W.star(seed=1)
    say("star full: generated", round(time.time() - t0, 1), "s")
    tr, ref = check_transfer(pt, prob)
    say("star full: fact survivors", ref.counts[0], "after", round(time.time() - t0, 1), "s")
    assert 300_000 < ref.counts[0] < 1_000_000


def test_repeatable_and_stream_ordered(pt):
    """Two transfers on one workspace, on a side stream, give identical bits."""
    prob = W.star(seed=5, n_fact=2_000_000, payload=0)
    dp = pt.DeviceProblem(prob)
    tr = pt.Transfer(dp)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tr.run(s)
        first = [b.clone() for b in tr.bitmaps]
        tr.run(s)
    s.synchronize()
    for a, b in zip(first, tr.bitmaps):
        assert torch.equal(a, b)


@pytest.mark.parametrize("bpk", [8, 12, 16])
def test_snowflake_scaled(pt, bpk):
    """Cyclic snowflake (int64 Zipf keys, a three-table cycle) at 1 % size:
    every bitmap, count and filter word of both passes."""
    prob = W.snowflake(seed=bpk, scale=0.01)
    say("snowflake 1%", bpk)
    check_transfer(pt, prob, 512, 3, bpk)


def test_snowflake_full_size(pt):
    """The full snowflake: 200 M fact rows, 50 M-row D1 whose filter (50 M
    keys) is read from HBM, every key int64 Zipf(1.1); all bitmaps and
    counts against the oracle."""
    t0 = time.time()
    prob = W.snowflake(seed=1)
    say("snowflake full: generated", round(time.time() - t0, 1), "s")
    tr, ref = check_transfer(pt, prob, 512, 3, 12, filters=False)
    say("snowflake full: counts", ref.counts, "after", round(time.time() - t0, 1), "s")


@pytest.mark.parametrize("flags", [0, 1])
@pytest.mark.parametrize("n_fact", [20_000, 3_000_000])
def test_append_and_rescan_agree(pt, flags, n_fact):
    """Builds from keys appended during the probe (the default) and builds
    that scan the selected rows again (PT_FLAG_NO_APPEND) write the same
    filters; at 3 M fact rows the dense dimension probes overflow some
    append regions, which are then walked."""
    key64 = (True, False, False, True) if n_fact < 100_000 else ()
    prob = W.star(seed=11, n_fact=n_fact, dims=(n_fact // 3, n_fact // 20, 500, 25), keeps=(0.3, 0.9, None, None),
                  payload=0, key64=key64)
    say("append", flags, n_fact)
    check_transfer(pt, prob, flags=flags)
    for s in range(3):
        say("append tiny", flags, s)
        check_transfer(pt, W.tiny_random(np.random.default_rng(9100 + s), SHAPES[s]), flags=flags)


@pytest.mark.parametrize("path,max_entries", [("atomic", None), ("lds", None), ("part", None), ("part", "1000")])
def test_build_paths(pt, monkeypatch, path, max_entries):
    """Every build path - one workgroup for a small table (the default when
    its filters fit in LDS), per-workgroup LDS copies (the default for larger
    tables whose filters fit, and for a large table whose selected rows make
    small filters), the partitioned tile build (forced here for every size),
    and in-place atomic OR (forced, or the partitioned build's fallback when
    its entry buffer is too small) - writes the same filter words."""
    monkeypatch.setenv("PT_BUILD_PATH", path)
    if max_entries:
        monkeypatch.setenv("PT_MAX_ENTRIES", max_entries)
    for s in range(4):
        prob = W.tiny_random(np.random.default_rng(4242 + s), SHAPES[s], max_rows=400, domain=40)
        say("build path", path, max_entries, s)
        check_transfer(pt, prob)
    say("build path", path, max_entries, "star")
    check_transfer(pt, W.star(seed=9, n_fact=300_000, dims=(60_000, 7_000, 500, 25), payload=0))


@pytest.mark.parametrize("key64", [(), (True, True, False, False)])
def test_small_filters_of_large_tables(pt, key64):
    """Builds sized for the partitioned path by their table's rows: D0 keeps
    2 % of 300 k rows (its filter fits the LDS copies the partitioned
    kernels fall back to), D1 keeps 90 % of 250 k rows (partitioned), and
    the fact table's backward filters are partitioned too; a 3 000-row
    dimension takes the one-workgroup build. Every bitmap, count and filter
    word equals the oracle's, with and without transfer path pruning (int32
    keys, then int64 keys on the two large dimensions)."""
    prob = W.star(seed=21, n_fact=400_000, dims=(300_000, 250_000, 3_000, 25), keeps=(0.02, 0.9, None, None),
                  payload=0, key64=key64)
    say("small filters of large tables", key64)
    check_transfer(pt, prob)
    say("small filters of large tables, pruned", key64)
    dp = pt.DeviceProblem(prob)
    tr = pt.Transfer(dp, pt.params(512, 3, 10, pt.PT_FLAG_PRUNE))
    tr.run()
    tr.check_status()
    ref = oracle.transfer(prob, 512, 3, 10, prune=True)
    counts = tr.counts.cpu().numpy()
    for t in range(prob.n_tables):
        assert_bitmaps_equal(tr.bitmap(t), ref.bitmaps[t], f"{prob.label} table {t}")
        assert counts[t] == ref.counts[t], (prob.label, t)


@pytest.mark.parametrize("shape", SHAPES)
def test_outer_join_edges(pt, shape):
    """Random graphs whose edges are inner, left, right or full outer joins
    (Sec. 3.4): bitmaps, counts and every filter equal the oracle's, and no
    filter exists for a direction an outer join blocks."""
    for s in range(15):
        prob = W.tiny_random(np.random.default_rng(95_000 + 1000 * SHAPES.index(shape) + s), shape, outer=0.6)
        say(prob.label, s, prob.edge_flags)
        check_transfer(pt, prob, 512, 3, 4)
