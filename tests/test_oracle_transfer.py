"""Pins of the oracle's transfer phase against what the paper and brute force
fix (Sec. 2.2, Sec. 3.2, Sec. 3.5):

* soundness: the join of the pre-filtered tables equals the join of the
  unfiltered ones (a transferred filter removes only non-joining rows);
* superset: kept rows contain every participating row; Bloom kept rows
  contain precise-filter kept rows;
* a precise filter turns the schedule into semi-joins: with every edge
  pointing towards one root the two passes are exactly Yannakakis' semi-join
  phase, so the result is the full reduction on acyclic graphs;
* a Bloom join is one-hop transfer; LIP on a star is the forward pass;
* the worked examples of Fig. 2 and Fig. 3 (authored instances);
* order invariance, edge cases, orientation rule.
"""
import numpy as np
import pytest

import goldens
import oracle
import refcheck as rc
from paper_2307_15255_amd import workloads as W

SHAPES = ["chain", "star", "tree", "cycle", "parallel", "forest"]


def kept_rows(res, problem):
    return [rc.bits_to_rows(res.bitmaps[t], problem.n_rows(t)) for t in range(problem.n_tables)]


def masks_from(res, problem):
    return [rc.bitmap_to_bool(res.bitmaps[t], problem.n_rows(t)) if problem.n_rows(t) else
            np.zeros(0, bool) for t in range(problem.n_tables)]


def _problems(shape, n, base_seed=0, **kw):
    for s in range(n):
        rng = np.random.default_rng(base_seed + 1000 * SHAPES.index(shape) + s)
        yield W.tiny_random(rng, shape, **kw)


@pytest.mark.parametrize("shape", SHAPES)
def test_sound_and_superset(oracle_lib, shape):
    for prob in _problems(shape, 40):
        bloom = oracle.transfer(prob, 512, 3, 10)
        exact = oracle.transfer(prob, kind=oracle.EXACT)
        part = rc.participating_rows(prob)
        kb, ke = kept_rows(bloom, prob), kept_rows(exact, prob)
        for t in range(prob.n_tables):
            local = set(np.nonzero(rc.local_rows(prob, t))[0].tolist())
            assert part[t] <= ke[t] <= kb[t] <= local, (prob.label, t)
            assert bloom.counts[t] == len(kb[t]) and exact.counts[t] == len(ke[t])
        # the join of the reduced tables is the join of the original ones
        base = rc.join_multiset(prob)
        assert rc.join_multiset(prob, masks_from(bloom, prob)) == base
        assert rc.join_multiset(prob, masks_from(exact, prob)) == base


@pytest.mark.parametrize("shape", ["chain", "star", "tree", "forest"])
def test_exact_in_tree_is_yannakakis_full_reduction(oracle_lib, shape):
    """Edges oriented child -> parent: the forward pass semi-joins each table
    with all its children bottom-up, the backward pass each child with its
    parent top-down (Sec. 2.2), so precise-filter transfer is the full
    reducer; it equals the participating rows when no tree joins to nothing."""
    for prob in _problems(shape, 40, base_seed=7):
        root = int(np.random.default_rng(len(prob.edges)).integers(0, prob.n_tables))
        prob.orient = rc.in_tree_orientation(prob, root)
        exact = oracle.transfer(prob, kind=oracle.EXACT)
        yk = rc.yannakakis_full_reduction(prob, root)
        assert kept_rows(exact, prob) == yk, prob.label
        comps = rc.join_tuples(prob)
        if all(len(df) for df in comps):
            assert yk == rc.participating_rows(prob)
        # fixpoint: running again on the reduced tables removes nothing more
        again = W.Problem(prob.names, [
            {c: a[rc.bitmap_to_bool(exact.bitmaps[t], prob.n_rows(t))] if prob.n_rows(t) else a
             for c, a in prob.columns[t].items()} for t in range(prob.n_tables)],
            prob.edges, [], prob.orient)
        res2 = oracle.transfer(again, kind=oracle.EXACT)
        assert res2.counts == [again.n_rows(t) for t in range(again.n_tables)]


def test_exact_not_full_reduction_without_in_tree(oracle_lib):
    """A - B - C with B the smallest table orients as A <- B -> C. A is
    filtered by B's forward filter before C has filtered B, and nothing flows
    back into A afterwards, so precise transfer keeps a row of A even though
    the whole join is empty: the full-reduction equality needs an in-tree."""
    A = {"x": np.array([1, 2], np.int32)}
    B = {"x": np.array([1], np.int32), "y": np.array([10], np.int32)}
    Cc = {"y": np.array([20, 30], np.int32)}
    prob = W.Problem(["A", "B", "C"], [A, B, Cc], [(0, "x", 1, "x"), (1, "y", 2, "y")])
    exact = oracle.transfer(prob, kind=oracle.EXACT)
    assert rc.participating_rows(prob) == [set(), set(), set()]
    assert exact.counts == [1, 0, 0]


def test_bpk_large_bloom_equals_exact(oracle_lib):
    for shape in SHAPES:
        for prob in _problems(shape, 15, base_seed=99):
            bloom = oracle.transfer(prob, 512, 8, 64)
            exact = oracle.transfer(prob, kind=oracle.EXACT)
            assert kept_rows(bloom, prob) == kept_rows(exact, prob), prob.label


@pytest.mark.parametrize("shape", SHAPES)
def test_order_invariance(oracle_lib, shape):
    """Topological tie-break and incoming-probe order leave every bitmap and
    every filter word unchanged (AND and OR commute)."""
    for prob in _problems(shape, 20, base_seed=5):
        ref = oracle.transfer(prob, 512, 3, 10, dump_filters=True)
        for variant in (1, 2, 3):
            r = oracle.transfer(prob, 512, 3, 10, variant=variant, dump_filters=True)
            for t in range(prob.n_tables):
                assert np.array_equal(r.bitmaps[t], ref.bitmaps[t])
            for key in ref.filters:
                assert np.array_equal(r.filters[key], ref.filters[key])


def test_bloom_join_is_one_hop_transfer(oracle_lib):
    """Sec. 1 and Sec. 2.1: a Bloom join builds a filter on the smaller
    table's key and probes it on the other table; one forward hop of the
    transfer computes exactly that."""
    for seed in range(10):
        rng = np.random.default_rng(seed)
        small = {"k": rng.integers(0, 500, 300).astype(np.int32), "x": rng.integers(0, 100, 300).astype(np.int32)}
        big = {"k": rng.integers(0, 500, 5000).astype(np.int64)}
        prob = W.Problem(["S", "L"], [small, big], [(1, "k", 0, "k")], [(0, "x", "lt", 40, 0)])
        res = oracle.transfer(prob, 512, 3, 10, n_passes=1)
        sel, _ = oracle.local_filter([small["k"], small["x"]], [(1, "lt", 40, 0)])
        words, nb = oracle.bloom_build(small["k"], sel, 512, 3, 10)
        bm, cnt = oracle.bloom_probe(big["k"], words, nb, 512, 3)
        assert np.array_equal(res.bitmaps[1], bm) and res.counts[1] == cnt
        # and it contains every joining row of L
        allowed = set(small["k"][small["x"] < 40].tolist())
        joining = {r for r, v in enumerate(big["k"].tolist()) if v in allowed}
        assert joining <= rc.bits_to_rows(bm, len(big["k"]))


def test_star_forward_pass_is_lip(oracle_lib):
    """Sec. 2.1 (LIP): on a star every dimension's filter goes straight to
    the fact table; the forward pass of the transfer is exactly that."""
    prob = W.star(seed=3, n_fact=50_000, dims=(20_000, 2_000, 100, 25), payload=0)
    res = oracle.transfer(prob, 512, 3, 10, n_passes=1)
    fact = prob.columns[0]
    bm = oracle.all_rows_bitmap(prob.n_rows(0))
    for d in range(4):
        dim = prob.columns[d + 1]
        sel = rc.rows_to_bits(np.nonzero(rc.local_rows(prob, d + 1))[0], prob.n_rows(d + 1))
        words, nb = oracle.bloom_build(dim["pk"], sel, 512, 3, 10)
        bm, _ = oracle.bloom_probe(fact[f"k{d}"], words, nb, 512, 3, bm)
    assert np.array_equal(res.bitmaps[0], bm)


@pytest.mark.parametrize("kind,bk,bpk", [(oracle.EXACT, 3, 10), (oracle.BLOOM, 8, 64)])
def test_fig3_worked_example(oracle_lib, kind, bk, bpk):
    prob, spec = goldens.load("fig3_chain.json")
    res = oracle.transfer(prob, 512, bk, bpk, kind=kind)
    for name, rows in spec["expect_forward_rows_1based"].items():
        t = prob.table(name)
        assert rc.bits_to_rows(res.fwd_bitmaps[t], prob.n_rows(t)) == {r - 1 for r in rows}
    for name, rows in spec["expect_final_rows_1based"].items():
        t = prob.table(name)
        assert rc.bits_to_rows(res.bitmaps[t], prob.n_rows(t)) == {r - 1 for r in rows}


def test_fig2_filter_transformation(oracle_lib):
    prob, spec = goldens.load("fig2_transform.json")
    for kind, bk, bpk in [(oracle.EXACT, 3, 10), (oracle.BLOOM, 8, 64)]:
        res = oracle.transfer(prob, 512, bk, bpk, kind=kind, n_passes=1, dump_filters=True)
        R = prob.table("R")
        assert rc.bits_to_rows(res.fwd_bitmaps[R], 5) == {r - 1 for r in spec["expect_forward_rows_1based"]["R"]}
        if kind == oracle.BLOOM:
            e = 2  # edge R.c -> Z.c
            words, nb = res.filters[(0, e)], res.filter_nb[(0, e)]
            assert res.edge_src[(0, e)] == R
            for key in spec["expect_c_filter_keys"]:
                assert oracle.bloom_contains(words, nb, 512, bk, key)
            for key in (100, 200, 400, 600):
                assert not oracle.bloom_contains(words, nb, 512, bk, key)
            assert nb == oracle.filter_blocks(2, bpk, 512)


def test_orientation_rule(oracle_lib):
    """Edges point from the smaller table to the bigger one (Sec. 3.2); ties
    go from the lower table index. The result is acyclic even on a cycle."""
    t = lambda n: {"a": np.arange(n, dtype=np.int32), "b": np.arange(n, dtype=np.int32)}
    prob = W.Problem(["A", "B", "C"], [t(5), t(3), t(5)],
                     [(0, "a", 1, "a"), (1, "b", 2, "b"), (2, "a", 0, "b")])
    res = oracle.transfer(prob, 512, 3, 10, dump_filters=True)
    assert res.edge_src[(0, 0)] == 1  # B (3 rows) -> A
    assert res.edge_src[(0, 1)] == 1  # B -> C
    assert res.edge_src[(0, 2)] == 0  # A, C tie at 5 rows: lower index A first
    for e in range(3):
        assert res.edge_src[(1, e)] != res.edge_src[(0, e)]  # backward reverses
    prob.orient = [1, 1, 1]  # A -> B -> C -> A is a cycle: rejected
    with pytest.raises(ValueError):
        oracle.transfer(prob)


def test_edge_cases(oracle_lib):
    # an empty selection builds one all-zero block and rejects everything downstream
    R = {"a": np.arange(10, dtype=np.int32), "p": np.zeros(10, np.int32)}
    S = {"a": np.arange(100, dtype=np.int32)}
    prob = W.Problem(["R", "S"], [R, S], [(0, "a", 1, "a")], [(0, "p", "gt", 5, 0)])
    res = oracle.transfer(prob, 512, 3, 10, dump_filters=True)
    assert res.filter_nb[(0, 0)] == 1 and not res.filters[(0, 0)].any()
    assert res.counts == [0, 0]
    # zero-row tables
    E = {"a": np.zeros(0, np.int32)}
    prob = W.Problem(["E", "S"], [E, S], [(0, "a", 1, "a")])
    res = oracle.transfer(prob, 512, 3, 10)
    assert res.counts == [0, 0]
    # an isolated table keeps its local filter only
    I = {"x": np.arange(70, dtype=np.int32)}
    prob = W.Problem(["R", "S", "I"], [R, S, I], [(0, "a", 1, "a")], [(2, "x", "lt", 65, 0)])
    res = oracle.transfer(prob, 512, 3, 10)
    assert res.counts[2] == 65 and res.counts[0] == 10 and res.counts[1] >= 10
    assert int(res.bitmaps[2][1]) == 1  # rows 64 is kept, 65..69 are not; tail bits zero
    # parallel edges on two column pairs act as two filters
    R2 = {"a": np.array([1, 2, 3], np.int32), "b": np.array([1, 9, 3], np.int32)}
    S2 = {"a": np.array([1, 2, 3, 4], np.int32), "b": np.array([1, 2, 3, 4], np.int32)}
    prob = W.Problem(["R", "S"], [R2, S2], [(0, "a", 1, "a"), (0, "b", 1, "b")])
    res = oracle.transfer(prob, kind=oracle.EXACT)
    assert rc.bits_to_rows(res.bitmaps[1], 4) == {0, 2}
    assert rc.bits_to_rows(res.bitmaps[0], 3) == {0, 2}


def test_local_filter_ops(oracle_lib):
    rng = np.random.default_rng(0)
    c32 = rng.integers(-1000, 1000, 777).astype(np.int32)
    c64 = (rng.integers(-1000, 1000, 777) * (1 << 35)).astype(np.int64)
    cases = [(0, "lt", 5, 0), (0, "le", -3, 0), (0, "gt", 100, 0), (0, "ge", 0, 0), (0, "eq", 7, 0),
             (0, "ne", 7, 0), (0, "between", -50, 50), (1, "lt", 0, 0), (1, "between", -(1 << 40), 1 << 40),
             (0, "lt", 1 << 40, 0), (0, "gt", -(1 << 40), 0), (0, "ge", 1 << 40, 0)]
    for case in cases:
        bm, cnt = oracle.local_filter([c32, c64], [case])
        prob = W.Problem(["T"], [{"a": c32, "b": c64}], [], [(0, "ab"[case[0]], *case[1:])])
        expect = rc.local_rows(prob, 0)
        assert np.array_equal(rc.bitmap_to_bool(bm, 777), expect) and cnt == expect.sum()
    bm, cnt = oracle.local_filter([c32, c64], [(0, "gt", -500, 0), (1, "lt", 0, 0)])
    assert cnt == int(((c32 > -500) & (c64 < 0)).sum())
    bm, cnt = oracle.local_filter([c32], [])
    assert cnt == 777 and int(bm[-1]) == (1 << (777 % 64)) - 1


def test_compact(oracle_lib):
    rng = np.random.default_rng(1)
    for n in (0, 1, 63, 64, 65, 1000, 4097):
        mask = rng.random(n) < 0.3
        bm = rc.rows_to_bits(np.nonzero(mask)[0], n)
        idx = oracle.compact(bm, n)
        assert np.array_equal(idx, np.nonzero(mask)[0].astype(np.uint32))


def test_one_hop_survivors_match_cost_model(oracle_lib):
    """Sec. 3.5: after a filter with false-positive rate eps, a table of T
    rows of which T* join passes T* + (T - T*) eps rows. On a star the four
    dimension filters act independently on independent uniform keys, so the
    fact survivors of the forward pass follow the product of the per-filter
    pass rates."""
    prob = W.star(seed=2, n_fact=2_000_000, dims=(200_000, 20_000, 1_000, 25), payload=0)
    res = oracle.transfer(prob, 512, 3, 10, n_passes=1, dump_filters=True)
    n = prob.n_rows(0)
    rate = 1.0
    for d in range(4):
        dim = prob.columns[d + 1]
        keep = rc.local_rows(prob, d + 1)
        share = keep.sum() / len(keep)  # fraction of fact rows whose key joins
        words, nb = res.filters[(0, d)], res.filter_nb[(0, d)]
        absent = dim["pk"][~keep]
        if len(absent):
            _, passed = oracle.bloom_probe(absent.copy(), words, nb, 512, 3)
            eps = passed / len(absent)
        else:
            eps = 0.0
        rate *= share + (1 - share) * eps
    expect = n * rate
    sd = np.sqrt(n * rate * (1 - rate))
    assert abs(res.fwd_counts[0] - expect) < 5 * sd, (res.fwd_counts[0], expect, sd)
