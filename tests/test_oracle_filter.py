"""Pins of the oracle's Bloom filter: the filter specification's hash and
layout (retyped with Python integers), no false negatives (Sec. 2.1), and the
false-positive rate against the blocked-Bloom closed form and against the
exact prediction from the filter's own bits."""
import math

import numpy as np
import pytest

import oracle
import refcheck as rc

EDGE_KEYS = [0, 1, -1, 2, -2, 2**31 - 1, -2**31, 2**32 - 1, 2**32, -2**32, 2**63 - 1, -2**63,
             123456789, -987654321, 0x0123456789ABCDEF, -0x0123456789ABCDEF]


def test_hash_matches_python_integers(oracle_lib):
    rng = np.random.default_rng(7)
    keys = EDGE_KEYS + [int(x) for x in rng.integers(-2**63, 2**63 - 1, 200, dtype=np.int64)]
    for key in keys:
        assert oracle.hash_key(key) == rc.spec_hash(key), key


@pytest.mark.parametrize("block_bits", [32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("k", [1, 3, 8, 16])
def test_slots_match_python_integers(oracle_lib, block_bits, k):
    rng = np.random.default_rng(block_bits * 100 + k)
    keys = EDGE_KEYS + [int(x) for x in rng.integers(-2**40, 2**40, 50)]
    for nb in (1, 7, 391, 11719, 2**31 + 3):
        for key in keys:
            blk, pos = oracle.key_slots(key, nb, block_bits, k)
            assert (blk, pos) == rc.spec_slots(key, nb, block_bits, k)
            assert 0 <= blk < nb
            assert len(set(pos)) == k  # odd stride: k distinct bits in a block


def test_filter_blocks(oracle_lib):
    assert oracle.filter_blocks(0, 10, 512) == 1
    assert oracle.filter_blocks(1, 10, 512) == 1
    assert oracle.filter_blocks(51, 10, 512) == 1     # 510 bits
    assert oracle.filter_blocks(52, 10, 512) == 2     # 520 bits
    assert oracle.filter_blocks(20_000, 10, 512) == 391
    assert oracle.filter_blocks(40_000, 10, 512) == 782
    assert oracle.filter_blocks(10_000, 10, 512) == 196
    assert oracle.filter_blocks(25, 10, 512) == 1
    assert oracle.filter_blocks(3, 64, 32) == 6
    for n in (0, 1, 99, 100_000, 2**32 - 1):
        for bpk in (1, 8, 10, 64):
            for B in (32, 512, 1024):
                assert oracle.filter_blocks(n, bpk, B) == max(1, -(-n * bpk // B))


@pytest.mark.parametrize("block_bits,k,bpk", [(512, 3, 10), (32, 1, 1), (64, 3, 8), (1024, 16, 64),
                                              (256, 6, 12), (128, 2, 3)])
def test_no_false_negatives(oracle_lib, block_bits, k, bpk):
    rng = np.random.default_rng(block_bits + k + bpk)
    for dtype in (np.int32, np.int64):
        info = np.iinfo(dtype)
        keys = rng.integers(info.min, info.max, 5000, dtype=dtype)
        keys[:4] = [info.min, info.max, 0, -1]
        words, nb = oracle.bloom_build(keys, None, block_bits, k, bpk)
        assert nb == oracle.filter_blocks(len(keys), bpk, block_bits)
        bm, cnt = oracle.bloom_probe(keys, words, nb, block_bits, k)
        assert cnt == len(keys)
        # build from a selection: every selected key passes
        sel = rng.random(len(keys)) < 0.3
        bits = rc.rows_to_bits(np.nonzero(sel)[0], len(keys))
        words, nb = oracle.bloom_build(keys, bits, block_bits, k, bpk)
        assert nb == oracle.filter_blocks(int(sel.sum()), bpk, block_bits)
        bm, cnt = oracle.bloom_probe(keys[sel].copy(), words, nb, block_bits, k)
        assert cnt == int(sel.sum())


def _measure_fpr(members, absent, block_bits, k, bpk):
    words, nb = oracle.bloom_build(members, None, block_bits, k, bpk)
    _, cnt = oracle.bloom_probe(absent, words, nb, block_bits, k)
    return cnt / len(absent), words, nb


KEY_SETS = {
    # members, absent keys (disjoint from members)
    "random64": lambda rng, n: (rng.integers(0, 2**62, n, dtype=np.int64),
                                rng.integers(2**62, 2**63 - 1, 1_000_000, dtype=np.int64)),
    "dense32": lambda rng, n: (np.arange(n, dtype=np.int32),
                               np.arange(n, n + 1_000_000, dtype=np.int32)),
    "strided32": lambda rng, n: (np.arange(n, dtype=np.int32) * 64,
                                 np.arange(n, n + 1_000_000, dtype=np.int32) * 64 + 1),
    "negative32": lambda rng, n: (-np.arange(1, n + 1, dtype=np.int32),
                                  np.arange(0, 1_000_000, dtype=np.int32)),
    "highword64": lambda rng, n: (np.arange(n, dtype=np.int64) << 32,
                                  (np.arange(n, n + 1_000_000, dtype=np.int64) << 32)),
    "subset_of_ids": lambda rng, n: _subset(rng, n),
}


def _subset(rng, n):
    ids = rng.permutation(20 * n).astype(np.int32)
    return ids[:n].copy(), ids[n:n + 1_000_000].copy() if 19 * n >= 1_000_000 else ids[n:].copy()


RANDOM_SETS = ("random64", "subset_of_ids")


@pytest.mark.parametrize("keyset", list(KEY_SETS))
@pytest.mark.parametrize("block_bits,k,bpk", [(512, 3, 10), (512, 3, 8), (512, 3, 16),
                                              (256, 3, 10), (64, 3, 10), (32, 3, 10),
                                              (1024, 5, 10), (128, 2, 4)])
def test_fpr_near_closed_form(oracle_lib, keyset, block_bits, k, bpk):
    """Measured false-positive rate on 10^6 absent keys against the blocked
    closed form with k distinct bits per key. Random key sets must land
    within 15 %. Structured key sets (dense, strided, negative, high-word
    only) must never be worse than 15 % above it; they may be better, since
    multiplicative hashing spreads arithmetic progressions more evenly over
    blocks than chance does."""
    rng = np.random.default_rng(11)
    members, absent = KEY_SETS[keyset](rng, 100_000)
    fpr, _, _ = _measure_fpr(members, absent, block_bits, k, bpk)
    expect = rc.blocked_fpr_distinct(block_bits, bpk, k)
    if keyset in RANDOM_SETS:
        assert abs(fpr - expect) / expect < 0.15, (fpr, expect)
    else:
        assert 0.5 * expect < fpr < 1.15 * expect, (fpr, expect)


def test_closed_form_reference_values():
    # the blocked form sits slightly above the classic unblocked rate
    assert abs(rc.blocked_fpr(512, 10, 3) - 0.01807) < 2e-4
    assert abs(rc.classic_fpr(10, 3) - 0.01741) < 2e-4
    assert rc.blocked_fpr(512, 10, 3) > rc.classic_fpr(10, 3)
    assert rc.blocked_fpr(32, 10, 3) > rc.blocked_fpr(512, 10, 3)


@pytest.mark.parametrize("block_bits,k,bpk", [(512, 3, 10), (64, 3, 8), (128, 4, 12)])
def test_fpr_matches_filter_bits(oracle_lib, block_bits, k, bpk):
    """Given the filter's bits, an absent key passes with probability equal to
    the share of (block, g1, g2) triples whose k bits are all set; the
    measured rate must lie within 4 binomial standard deviations of it."""
    rng = np.random.default_rng(3)
    members = rng.integers(-2**31, 2**31 - 1, 4000, dtype=np.int64)
    absent = rng.integers(2**40, 2**41, 1_000_000, dtype=np.int64)
    fpr, words, nb = _measure_fpr(members, absent, block_bits, k, bpk)
    pred = rc.per_filter_fpr(words, nb, block_bits, k)
    sigma = math.sqrt(pred * (1 - pred) / len(absent))
    assert abs(fpr - pred) < 4 * sigma + 1e-12, (fpr, pred, sigma)


def test_block_load_is_uniform(oracle_lib):
    """Keys spread over blocks like balls into bins: the number of keys per
    block has the binomial mean and variance (chi-square style bound)."""
    nb = 391
    for keys in (np.arange(20_000, dtype=np.int64), np.arange(20_000, dtype=np.int64) * 1000003,
                 np.random.default_rng(5).integers(-2**63, 2**63 - 1, 20_000, dtype=np.int64)):
        blocks = np.array([oracle.key_slots(int(x), nb, 512, 1)[0] for x in keys[:20_000]])
        cnt = np.bincount(blocks, minlength=nb)
        mean = len(keys) / nb
        chi2 = ((cnt - mean) ** 2 / mean).sum()
        # chi-square with nb-1 dof: mean nb-1, sd sqrt(2(nb-1)); allow 5 sd
        assert chi2 < (nb - 1) + 5 * math.sqrt(2 * (nb - 1)), chi2
