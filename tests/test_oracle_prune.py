"""Pins of the oracle's transfer path pruning (Sec. 3.2, "Transfer Path
Pruning": the paper asks for skipping transfers that cannot make a filter
more selective and leaves the rule open). The rule read here: a non-empty
table whose selection still holds every one of its rows sends no filter,
and the tables it would have sent one to are not probed with it.

* an authored chain worked by hand, where pruning keeps a row that the full
  transfer removes, and the join result is the same;
* pruning changes no join result and keeps every participating row (brute
  force on random graphs); with precise filters the kept rows contain those
  of the full transfer;
* on a star whose foreign keys all reference existing keys, the pruned
  filters remove nothing, so the result is bit for bit the full one;
* an unreduced table passes its state on: a table that receives only
  pruned filters is unreduced in turn and sends none either;
* an empty table's filter (it holds no key) is never pruned;
* on the paper's own Fig. 3 instance (no table has a predicate) nothing is
  transferred at all.
"""
import numpy as np
import pytest

import goldens
import oracle
import refcheck as rc
from paper_2307_15255_amd.workloads import Problem
from test_oracle_transfer import SHAPES, _problems, kept_rows, masks_from


def _rows(res, prob, name, fwd=False):
    t = prob.table(name)
    bm = res.fwd_bitmaps[t] if fwd else res.bitmaps[t]
    return rc.bits_to_rows(bm, prob.n_rows(t))


@pytest.mark.parametrize("kind,bk,bpk", [(oracle.EXACT, 3, 10), (oracle.BLOOM, 8, 64)])
def test_prune_worked_example(oracle_lib, kind, bk, bpk):
    prob, spec = goldens.load("prune_chain.json")
    full = oracle.transfer(prob, 512, bk, bpk, kind=kind)
    pruned = oracle.transfer(prob, 512, bk, bpk, kind=kind, prune=True)
    for res, tag in ((full, "full"), (pruned, "pruned")):
        for name, rows in spec[f"expect_{tag}_forward_rows_1based"].items():
            assert _rows(res, prob, name, fwd=True) == {r - 1 for r in rows}, (tag, name)
        for name, rows in spec[f"expect_{tag}_final_rows_1based"].items():
            assert _rows(res, prob, name) == {r - 1 for r in rows}, (tag, name)
    want = sorted(tuple(r - 1 for r in t) for t in spec["expect_join_tuples_1based"])
    for res in (full, pruned):
        comp, tuples = oracle.join(prob, res.bitmaps, root=0)
        assert [prob.names[t] for t in comp] == ["R", "S", "T"]
        assert sorted(map(tuple, tuples.tolist())) == want


def test_prune_skips_only_unreduced_senders(oracle_lib):
    prob, spec = goldens.load("prune_chain.json")
    res = oracle.transfer(prob, 512, 8, 64, prune=True, dump_filters=True)
    names = {(prob.names[u], prob.names[v]): e for e, (u, _, v, _) in enumerate(prob.edges)}
    for arrow, built in spec["expect_pruned_forward_filters"].items():
        a, b = arrow.split("->")
        e = names.get((a, b), names.get((b, a)))
        assert res.edge_src[(0, e)] == prob.table(a)
        assert (res.filter_nb[(0, e)] > 0) == built, arrow
    # backward pass: S lost a row, so both its filters are built
    for e in range(len(prob.edges)):
        assert res.edge_src[(1, e)] == prob.table("S") and res.filter_nb[(1, e)] > 0


@pytest.mark.parametrize("shape", SHAPES)
def test_prune_sound_and_superset(oracle_lib, shape):
    for prob in _problems(shape, 30, base_seed=11):
        part = rc.participating_rows(prob)
        base = rc.join_multiset(prob)
        full_exact = kept_rows(oracle.transfer(prob, kind=oracle.EXACT), prob)
        for kind in (oracle.BLOOM, oracle.EXACT):
            res = oracle.transfer(prob, 512, 3, 10, kind=kind, prune=True)
            kept = kept_rows(res, prob)
            for t in range(prob.n_tables):
                local = set(np.nonzero(rc.local_rows(prob, t))[0].tolist())
                assert part[t] <= kept[t] <= local, (prob.label, t)
                assert res.counts[t] == len(kept[t])
                if kind == oracle.EXACT:
                    # precise filters only ever shrink with more transfers
                    assert full_exact[t] <= kept[t], (prob.label, t)
            assert rc.join_multiset(prob, masks_from(res, prob)) == base, prob.label


def _fk_star(seed, filtered):
    """A fact table of 3000 rows whose foreign keys all reference existing
    dimension keys (0..n-1 in shuffled order); dimension i has a predicate
    iff filtered[i]."""
    rng = np.random.default_rng(seed)
    sizes = [97, 40, 13, 5][:len(filtered)]
    names, cols, edges, preds = ["F"], [{}], [], []
    n_fact = 3000
    for i, (n, f) in enumerate(zip(sizes, filtered)):
        names.append(f"D{i}")
        cols.append({"pk": rng.permutation(n).astype(np.int32), "attr": rng.integers(0, 100, n).astype(np.int32)})
        cols[0][f"k{i}"] = rng.integers(0, n, n_fact).astype(np.int32)
        edges.append((0, f"k{i}", i + 1, "pk"))
        if f:
            preds.append((i + 1, "attr", "lt", 30, 0))
    return Problem(names, cols, edges, preds, label=f"fk_star{seed}")


@pytest.mark.parametrize("kind", [oracle.BLOOM, oracle.EXACT])
def test_prune_referential_integrity_changes_nothing(oracle_lib, kind):
    for seed in range(6):
        filtered = [seed % 2 == 0, True, seed % 3 == 0, False]
        prob = _fk_star(seed, filtered)
        full = oracle.transfer(prob, 512, 3, 10, kind=kind)
        pruned = oracle.transfer(prob, 512, 3, 10, kind=kind, prune=True, dump_filters=True)
        for t in range(prob.n_tables):
            assert np.array_equal(full.bitmaps[t], pruned.bitmaps[t]), (seed, prob.names[t])
            assert np.array_equal(full.fwd_bitmaps[t], pruned.fwd_bitmaps[t]), (seed, prob.names[t])
        if kind == oracle.BLOOM:
            for e, f in enumerate(filtered):
                # forward pass: dimension -> fact, built only from a filtered dimension
                assert pruned.edge_src[(0, e)] == e + 1
                assert (pruned.filter_nb[(0, e)] > 0) == f, (seed, e)
                # backward pass: the fact table lost rows (a filtered dimension keeps 30 %)
                assert pruned.filter_nb[(1, e)] > 0


def test_prune_propagates_along_a_path(oracle_lib):
    """A -> B -> C, with B receiving only A's filter and no predicate on A or
    B: A is unreduced, so B receives nothing and is unreduced too; only the
    filtered table D sends C a filter in the forward pass."""
    rng = np.random.default_rng(5)
    A = {"id": np.arange(8, dtype=np.int32)}
    B = {"id": np.arange(20, dtype=np.int32), "a": rng.integers(0, 8, 20).astype(np.int32)}
    D = {"id": np.arange(12, dtype=np.int32), "x": rng.integers(0, 10, 12).astype(np.int32)}
    Cc = {"b": rng.integers(0, 20, 60).astype(np.int32), "d": rng.integers(0, 12, 60).astype(np.int32)}
    prob = Problem(["A", "B", "C", "D"], [A, B, Cc, D],
                   [(0, "id", 1, "a"), (1, "id", 2, "b"), (3, "id", 2, "d")], [(3, "x", "lt", 4, 0)])
    res = oracle.transfer(prob, 512, 3, 10, prune=True, dump_filters=True)
    full = oracle.transfer(prob, 512, 3, 10, dump_filters=True)
    assert [res.filter_nb[(0, e)] > 0 for e in range(3)] == [False, False, True]
    assert all(full.filter_nb[(0, e)] > 0 for e in range(3))
    assert res.fwd_counts[prob.table("A")] == 8 and res.fwd_counts[prob.table("B")] == 20
    assert rc.join_multiset(prob, masks_from(res, prob)) == rc.join_multiset(prob)


def test_prune_keeps_an_empty_tables_filter(oracle_lib):
    """An empty table holds all of its (zero) rows, but its filter holds no
    key: it still goes out and empties every table it reaches, as without
    pruning (the join result is empty either way)."""
    prob = Problem(["E", "S", "T"],
                   [{"a": np.zeros(0, np.int32)}, {"a": np.arange(6, dtype=np.int32), "b": np.arange(6, dtype=np.int32)},
                    {"b": np.arange(9, dtype=np.int32)}],
                   [(0, "a", 1, "a"), (1, "b", 2, "b")], [])
    for kind in (oracle.BLOOM, oracle.EXACT):
        res = oracle.transfer(prob, 512, 3, 10, kind=kind, prune=True)
        assert res.counts == [0, 0, 0]


def test_prune_on_fig3_transfers_nothing(oracle_lib):
    """No table of the Fig. 3 instance has a predicate, so no table is ever
    reduced and nothing is sent: every row stays (without pruning the
    transfer removes the rows the paper lists)."""
    prob, _ = goldens.load("fig3_chain.json")
    res = oracle.transfer(prob, 512, 3, 10, kind=oracle.EXACT, prune=True)
    for t in range(prob.n_tables):
        assert res.counts[t] == prob.n_rows(t)


def test_prune_off_is_the_default(oracle_lib):
    for prob in _problems("tree", 10, base_seed=3):
        a = oracle.transfer(prob, 512, 3, 10)
        b = oracle.transfer(prob, 512, 3, 10, prune=False)
        assert all(np.array_equal(x, y) for x, y in zip(a.bitmaps, b.bitmaps))
