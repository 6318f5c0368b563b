"""Pins of the oracle's join phase (Sec. 3.3: regular joins on the tables the
transfer phase reduced) against what the definition and the paper fix:

* brute force: on tiny tables, every combination of selected rows that
  agrees on every edge, enumerated directly;
* an independent join: pandas merges over all edges (tests/refcheck.py), on
  chains, stars, trees, cycles, parallel edges and forests;
* the paper's soundness property: joining the tables reduced by the
  transfer phase gives the same tuples as joining the tables reduced by
  their local predicates only (a transferred filter drops only rows that
  join with nothing, Sec. 3.1; a Bloom filter has no false negatives,
  Sec. 2.1);
* edge cases: empty tables and bitmaps, a table with no edge, duplicate
  keys on both sides (many-to-many), composite keys.
"""
import itertools

import numpy as np
import pytest

import oracle
import refcheck as rc
from paper_2307_15255_amd import workloads as W

SHAPES = ["chain", "star", "tree", "cycle", "parallel", "forest"]


def local_bitmaps(prob):
    return [rc.rows_to_bits(np.nonzero(rc.local_rows(prob, t))[0], prob.n_rows(t)) for t in range(prob.n_tables)]


def pandas_join(prob, masks, comp):
    """The component's tuples from refcheck.join_tuples, columns in
    ascending table order, sorted."""
    for df in rc.join_tuples(prob, masks):
        if sorted(int(c[1:]) for c in df.columns) == sorted(comp):
            arr = df[[f"r{t}" for t in sorted(comp)]].to_numpy(dtype=np.int64)
            return sorted(map(tuple, arr.tolist()))
    raise AssertionError("component not found")


def brute_force(prob, masks, comp):
    """Every combination of selected rows of the component's tables that
    satisfies every edge between them."""
    comp = sorted(comp)
    rows = [np.nonzero(masks[t])[0].tolist() for t in comp]
    pos = {t: i for i, t in enumerate(comp)}
    out = []
    for combo in itertools.product(*rows):
        ok = True
        for u, uc, v, vc in prob.edges:
            if u in pos and v in pos:
                if int(prob.columns[u][uc][combo[pos[u]]]) != int(prob.columns[v][vc][combo[pos[v]]]):
                    ok = False
                    break
        if ok:
            out.append(tuple(int(x) for x in combo))
    return sorted(out)


def as_tuples(arr):
    return [tuple(int(x) for x in row) for row in arr]


def _problems(shape, n, base_seed=0, **kw):
    for s in range(n):
        rng = np.random.default_rng(base_seed + 7000 + 1000 * SHAPES.index(shape) + s)
        yield W.tiny_random(rng, shape, **kw)


@pytest.mark.parametrize("shape", SHAPES)
def test_join_matches_brute_force(oracle_lib, shape):
    for prob in _problems(shape, 25, max_tables=4, max_rows=7, domain=3):
        masks = [rc.local_rows(prob, t) for t in range(prob.n_tables)]
        bms = local_bitmaps(prob)
        for comp0 in rc._components(prob):
            comp, got = oracle.join(prob, bms, root=comp0[-1])
            assert comp == sorted(comp0)
            assert as_tuples(got) == brute_force(prob, masks, comp), prob.label


@pytest.mark.parametrize("shape", SHAPES)
def test_join_matches_pandas(oracle_lib, shape):
    for prob in _problems(shape, 30):
        masks = [rc.local_rows(prob, t) for t in range(prob.n_tables)]
        bms = local_bitmaps(prob)
        for comp0 in rc._components(prob):
            for root in (comp0[0], max(comp0, key=prob.n_rows)):
                comp, got = oracle.join(prob, bms, root=root)
                assert as_tuples(got) == pandas_join(prob, masks, comp), (prob.label, root)


@pytest.mark.parametrize("shape", SHAPES)
def test_join_after_transfer_equals_join_after_local_filters(oracle_lib, shape):
    """Sec. 3.1 / Sec. 2.1: pre-filtering never removes a joining row, so
    the join phase on the transferred tables has exactly the tuples of the
    join on the locally filtered tables; it also only reads selected rows."""
    for prob in _problems(shape, 25, base_seed=50):
        masks = [rc.local_rows(prob, t) for t in range(prob.n_tables)]
        res = oracle.transfer(prob, 512, 3, 4)
        for comp0 in rc._components(prob):
            comp, got = oracle.join(prob, res.bitmaps, root=comp0[0])
            assert as_tuples(got) == pandas_join(prob, masks, comp), prob.label
            for c, t in enumerate(comp):
                sel = rc.bits_to_rows(res.bitmaps[t], prob.n_rows(t))
                assert set(got[:, c].tolist()) <= sel


def test_join_chain_config(oracle_lib):
    """The 1 000 / 10 000 / 1 000-row chain R - S - T with a 10 % predicate
    on R: pandas and the oracle agree, from every root."""
    prob = W.chain(seed=1)
    masks = [rc.local_rows(prob, t) for t in range(prob.n_tables)]
    bms = local_bitmaps(prob)
    want = pandas_join(prob, masks, [0, 1, 2])
    assert len(want) > 0
    for root in range(3):
        comp, got = oracle.join(prob, bms, root=root)
        assert comp == [0, 1, 2]
        assert as_tuples(got) == want


def _problem(columns, edges, preds=()):
    return W.Problem([f"T{t}" for t in range(len(columns))], columns, list(edges), list(preds), label="hand")


def test_join_edge_cases(oracle_lib):
    i32 = lambda *v: np.array(v, np.int32)
    i64 = lambda *v: np.array(v, np.int64)
    # many-to-many: key 1 twice on each side -> 4 tuples; key 2 once each -> 1
    p = _problem([{"a": i32(1, 1, 2, 3)}, {"a": i64(2, 1, 1, 4)}], [(0, "a", 1, "a")])
    comp, got = oracle.join(p)
    assert comp == [0, 1]
    assert as_tuples(got) == [(0, 1), (0, 2), (1, 1), (1, 2), (2, 0)]
    # int32 -1 equals int64 -1 (keys compare as int64 values)
    p = _problem([{"a": i32(-1, 5)}, {"a": i64(-1, 5 + (1 << 32))}], [(0, "a", 1, "a")])
    assert as_tuples(oracle.join(p)[1]) == [(0, 0)]
    # composite key: both columns must agree
    p = _problem([{"a": i32(1, 1, 2), "b": i32(7, 8, 7)}, {"a": i32(1, 2, 1), "b": i32(8, 7, 7)}],
                 [(0, "a", 1, "a"), (1, "b", 0, "b")])
    assert as_tuples(oracle.join(p)[1]) == [(0, 2), (1, 0), (2, 1)]
    # a bitmap that selects nothing empties the join
    empty = [np.zeros(1, np.uint64), None]
    assert oracle.join(p, empty)[1].shape == (0, 2)
    # a table with no edge: its selected rows, one per tuple
    p = _problem([{"a": i32(3, 4, 5)}, {"a": i32(1)}], [])
    comp, got = oracle.join(p, [rc.rows_to_bits([0, 2], 3), None], root=0)
    assert comp == [0] and as_tuples(got) == [(0,), (2,)]
    # a table with no rows
    p = _problem([{"a": i32()}, {"a": i32(1, 2)}], [(0, "a", 1, "a")])
    assert oracle.join(p, root=1)[1].shape == (0, 2)
    # a triangle: the closing edge filters tuples the tree edges allow
    p = _problem([{"x": i32(1, 1), "z": i32(5, 6)}, {"x": i32(1), "y": i32(2)}, {"y": i32(2, 2), "z": i32(6, 7)}],
                 [(0, "x", 1, "x"), (1, "y", 2, "y"), (2, "z", 0, "z")])
    assert as_tuples(oracle.join(p)[1]) == [(1, 0, 0)]


def test_join_rejects_bad_arguments(oracle_lib):
    p = _problem([{"a": np.array([1], np.int32)}], [(0, "a", 0, "a")])
    with pytest.raises(ValueError):
        oracle.join(p)
    p = _problem([{"a": np.array([1], np.int32)}], [])
    with pytest.raises(ValueError):
        oracle.join(p, root=1)
