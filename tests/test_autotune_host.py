"""The autotuner's host logic: its closed-form false-positive rate agrees
with the test suite's own implementation, every candidate meets the cap with
the fewest bits per key, and the choice is the cheapest measured setting for
the problem's size class."""
import math

import numpy as np
import pytest

import refcheck as rc
from paper_2307_15255_amd import autotune as A
from paper_2307_15255_amd import workloads as W


@pytest.mark.parametrize("B,k,bpk", [(512, 3, 10), (256, 2, 14), (512, 4, 9), (1024, 8, 16), (64, 1, 4)])
def test_fpr_matches_reference(B, k, bpk):
    assert math.isclose(A.blocked_fpr(B, k, bpk), rc.blocked_fpr(B, bpk, k), rel_tol=1e-6)


@pytest.mark.parametrize("cap", [0.005, 0.02, 0.05])
def test_candidates_meet_cap_with_fewest_bits(cap):
    cands = A.candidates(cap)
    assert cands
    for B, k, bpk in cands:
        assert A.blocked_fpr(B, k, bpk) <= cap
        if bpk > min(A.BITS_PER_KEY):
            assert A.blocked_fpr(B, k, bpk - 1) > cap


def test_choice_is_cheapest_for_the_size_class():
    ct = A.CostTable()
    cands = A.candidates(0.02)
    rng = np.random.default_rng(3)
    for size in A.SIZE_CLASSES:
        for c in cands:
            ct.probe[(size, *c)] = float(rng.uniform(0.01, 0.1))
            ct.build[(size, *c)] = float(rng.uniform(0.01, 0.1))
    small = W.chain(n_r=20_000, n_s=30_000, n_t=20_000)
    for prob, size in [(small, 20_000)]:
        got = A.choose(prob, ct)
        best = min(cands, key=lambda c: ct.probe[(size, *c)] + ct.build[(size, *c)])
        assert got == best
    assert A.CostTable.from_json(ct.to_json()).probe == ct.probe
