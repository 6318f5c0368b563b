"""The autotuner's host logic: its closed-form false-positive rate agrees
with the test suite's own implementation (k distinct bits per key), every
candidate meets the cap with the fewest bits per key, the choice is the
cheapest setting for the problem's size class, and it is a function of the
problem and the cost table alone (repeated calls agree)."""
import math

import numpy as np
import pytest

import refcheck as rc
from paper_2307_15255_amd import autotune as A
from paper_2307_15255_amd import workloads as W


@pytest.mark.parametrize("B,k,bpk", [(512, 3, 10), (256, 2, 14), (512, 4, 9), (1024, 8, 16), (64, 1, 4)])
def test_fpr_matches_reference(B, k, bpk):
    assert math.isclose(A.blocked_fpr(B, k, bpk), rc.blocked_fpr_distinct(B, bpk, k), rel_tol=1e-6)


@pytest.mark.parametrize("cap", [0.005, 0.02, 0.05])
def test_candidates_meet_cap_with_fewest_bits(cap):
    cands = A.candidates(cap)
    assert cands
    for B, k, bpk in cands:
        assert (B, k) in [(b, h) for b in A.BLOCK_BITS for h in A.HASHES]
        assert A.blocked_fpr(B, k, bpk) <= cap
        if bpk > min(A.BITS_PER_KEY):
            assert A.blocked_fpr(B, k, bpk - 1) > cap


def _table(seed=3):
    ct = A.CostTable(device="test")
    rng = np.random.default_rng(seed)
    for size in A.SIZE_CLASSES:
        for c in A.candidates(0.02):
            ct.probe[(size, *c)] = float(rng.uniform(0.01, 0.1))
            ct.build[(size, *c)] = float(rng.uniform(0.01, 0.1))
    return ct


def test_choice_is_cheapest_for_the_size_class():
    ct = _table()
    cands = A.candidates(0.02)
    small = W.chain(n_r=20_000, n_s=30_000, n_t=20_000)
    got = A.choose(small, ct)
    best = min(cands, key=lambda c: ct.probe[(20_000, *c)] + ct.build[(20_000, *c)])
    assert got == best
    back = A.CostTable.from_json(ct.to_json())
    assert back.probe == ct.probe and back.build == ct.build and back.device == "test"


def test_choice_is_a_function_of_the_problem():
    """Same problems and cost table: the same parameters, call after call,
    whatever the order of the problems."""
    ct = _table(11)
    probs = W.batch(seed=4, n_problems=24, lo=1_000, hi=50_000)
    first, _ = A.tune(probs, ct, n_cu=256)
    for _ in range(3):
        again, _ = A.tune(probs, ct, n_cu=256)
        assert [(p.block_bits, p.k, p.bits_per_key, p.tile_rows) for p in again] == \
            [(p.block_bits, p.k, p.bits_per_key, p.tile_rows) for p in first]
    rev, _ = A.tune(probs[::-1], ct, n_cu=256)
    assert [(p.block_bits, p.k, p.bits_per_key) for p in rev[::-1]] == \
        [(p.block_bits, p.k, p.bits_per_key) for p in first]
    assert all(p.block_bits == 512 and p.k in (2, 3) for p in first)


def test_tile_rows_follow_the_batch_size():
    small = [W.chain(n_r=1_000, n_s=2_000, n_t=1_000)]
    assert A.tile_rows_for(small, 256) == min(A.TILE_ROWS)
    big = W.batch(seed=1, n_problems=8, lo=4_000_000, hi=5_000_000)
    assert A.tile_rows_for(big, 8) == max(A.TILE_ROWS)


def test_tile_choice_saved_for_a_batch_is_reused(tmp_path, monkeypatch):
    """tune_tiles reads its choice from the device's table when the batch's
    digest is there (no measurement), and the digest follows what the batch
    is made of."""
    from paper_2307_15255_amd import pt
    monkeypatch.setattr(A, "COST_DIR", str(tmp_path))
    monkeypatch.setattr(A, "device_name", lambda: "test device 8cu")
    probs = [W.tiny_random(np.random.default_rng(s), "tree") for s in range(6)]
    params = [pt.params(512, 3, 10)] * len(probs)
    digest = A.batch_digest(probs, params)
    with open(A._tiles_path("test device 8cu"), "w") as f:
        f.write('{"%s": {"tile_rows": 65536, "ms": {}}}' % digest)

    class DP:
        def __init__(self, p):
            self.problem = p

    out, rec = A.tune_tiles([DP(p) for p in probs], params)
    assert [p.tile_rows for p in out] == [65536] * len(probs)
    assert rec["measured_ms"] is None and rec["digest"] == digest
    assert [(p.block_bits, p.k, p.bits_per_key) for p in out] == [(512, 3, 10)] * len(probs)
    # another predicate constant or other filter settings: another batch
    changed = [W.Problem(p.names, p.columns, p.edges, [(t, c, op, lo + 1, hi) for t, c, op, lo, hi in p.preds],
                         p.orient, p.label, p.edge_flags) for p in probs]
    if any(p.preds for p in probs):
        assert A.batch_digest(changed, params) != digest
    assert A.batch_digest(probs, [pt.params(512, 2, 14)] * len(probs)) != digest
    assert A.batch_digest(probs[::-1], params) != digest
