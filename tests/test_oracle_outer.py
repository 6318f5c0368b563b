"""Pins of the oracle's outer-join edges (Sec. 3.4: a left outer join lets
filters go only from its left table to its right table, a right outer join
the reverse, a full outer join not at all):

* soundness against the query itself: on random join trees whose edges are
  inner, left, right or full outer joins, the query evaluated bottom-up with
  pandas (tests/refcheck.py) gives the same tuples, null-extended ones
  included, on the tables the transfer phase reduced as on the tables
  reduced by their local predicates only;
* the preserved side of an outer join is never reduced through it: with
  every edge a full outer join each table keeps exactly its local rows, and
  the left table of a single left outer join keeps exactly its local rows;
* the blocked direction builds no filter.
"""
import numpy as np
import pytest

import oracle
import refcheck as rc
from paper_2307_15255_amd import workloads as W


def local_masks(prob):
    return [rc.local_rows(prob, t) for t in range(prob.n_tables)]


def masks_from(res, prob):
    return [rc.bitmap_to_bool(res.bitmaps[t], prob.n_rows(t)) if prob.n_rows(t) else np.zeros(0, bool)
            for t in range(prob.n_tables)]


@pytest.mark.parametrize("shape", ["chain", "star", "tree"])
def test_outer_tree_query_unchanged(oracle_lib, shape):
    for s in range(40):
        prob = W.tiny_random(np.random.default_rng(31_000 + 100 * ["chain", "star", "tree"].index(shape) + s),
                             shape, max_rows=12, domain=4, outer=0.6)
        res = oracle.transfer(prob, 512, 3, 4)
        for root in range(prob.n_tables):
            want = rc.outer_tree_result(prob, local_masks(prob), root)
            got = rc.outer_tree_result(prob, masks_from(res, prob), root)
            assert got == want, (prob.label, s, root, prob.edge_flags)


def test_full_outer_blocks_every_transfer(oracle_lib):
    for s in range(20):
        prob = W.tiny_random(np.random.default_rng(32_000 + s), "tree")
        prob.edge_flags = [3] * len(prob.edges)
        res = oracle.transfer(prob, 512, 3, 10, dump_filters=True)
        for t in range(prob.n_tables):
            assert rc.bits_to_rows(res.bitmaps[t], prob.n_rows(t)) == set(np.nonzero(rc.local_rows(prob, t))[0].tolist())
        assert all(nb == 0 for nb in res.filter_nb.values())


@pytest.mark.parametrize("flag,preserved", [(1, 0), (2, 1)])
def test_preserved_side_keeps_its_rows(oracle_lib, flag, preserved):
    """One edge: the preserved table keeps exactly its local rows; the other
    keeps at least the rows that match one of the preserved table's local
    rows (the filter has no false negatives) and only rows it kept locally;
    the only filter built goes from the preserved table to the other."""
    for s in range(30):
        rng = np.random.default_rng(33_000 + s)
        a = rng.integers(0, 6, int(rng.integers(1, 30))).astype(np.int32)
        b = rng.integers(0, 6, int(rng.integers(1, 30))).astype(np.int32)
        prob = W.Problem(["A", "B"], [{"k": a, "x": rng.integers(0, 100, len(a)).astype(np.int32)},
                                      {"k": b, "x": rng.integers(0, 100, len(b)).astype(np.int32)}],
                         [(0, "k", 1, "k")], [(0, "x", "lt", 50, 0), (1, "x", "lt", 70, 0)], label="one edge",
                         edge_flags=[flag])
        res = oracle.transfer(prob, 512, 3, 10)
        other = 1 - preserved
        local = [set(np.nonzero(rc.local_rows(prob, t))[0].tolist()) for t in range(2)]
        kept = [rc.bits_to_rows(res.bitmaps[t], prob.n_rows(t)) for t in range(2)]
        assert kept[preserved] == local[preserved]
        keys = {int(prob.columns[preserved]["k"][r]) for r in local[preserved]}
        must = {r for r in local[other] if int(prob.columns[other]["k"][r]) in keys}
        assert must <= kept[other] <= local[other]
        built = [p for p, src in res.edge_src.items() if src != 0xFFFFFFFF]
        assert all(res.edge_src[p] == preserved for p in built) and len(built) == 1
