"""The oracle's optional row split (an OpenMP split of the transfer's row
scans by whole bitmap words, Bloom filters built in private copies and
OR-ed) gives the one-thread oracle's results bit for bit: every bitmap,
count and filter word, in Bloom and exact mode, on random small graphs of
every shape, the chain, a star and a scaled snowflake."""
import os

import numpy as np
import pytest

import oracle
from paper_2307_15255_amd import workloads as W

SHAPES = ["chain", "star", "tree", "cycle", "parallel", "forest"]


def same(a, b):
    assert a.counts == b.counts
    for x, y in zip(a.bitmaps, b.bitmaps):
        assert np.array_equal(x, y)
    for x, y in zip(a.fwd_bitmaps, b.fwd_bitmaps):
        assert np.array_equal(x, y)
    assert a.filter_nb == b.filter_nb
    assert a.filters.keys() == b.filters.keys()
    for key in a.filters:
        assert np.array_equal(a.filters[key], b.filters[key]), key


@pytest.mark.parametrize("shape", SHAPES)
def test_threads_tiny(oracle_lib, shape):
    for s in range(15):
        prob = W.tiny_random(np.random.default_rng(4000 + 100 * SHAPES.index(shape) + s), shape, max_rows=300)
        for kind in (oracle.BLOOM, oracle.EXACT):
            one = oracle.transfer(prob, 512, 3, 6, kind=kind, dump_filters=True)
            for threads in (2, 3, 8):
                same(one, oracle.transfer(prob, 512, 3, 6, kind=kind, dump_filters=True, threads=threads))


@pytest.mark.parametrize("make", [lambda: W.chain(seed=2),
                                  lambda: W.star(seed=4, n_fact=400_000, dims=(40_000, 4_000, 100, 25), payload=0),
                                  lambda: W.snowflake(seed=3, scale=0.005)])
def test_threads_workloads(oracle_lib, make):
    prob = make()
    one = oracle.transfer(prob, 512, 3, 10, dump_filters=True)
    n = max(2, min(8, len(os.sched_getaffinity(0))))
    same(one, oracle.transfer(prob, 512, 3, 10, dump_filters=True, threads=n))
