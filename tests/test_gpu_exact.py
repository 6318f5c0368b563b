"""GPU parity of the transfer phase with exact filters (PT_FLAG_EXACT: the
precise filter of Sec. 3.2, every transfer a semi-join) against the
oracle's exact mode: every table's bitmap and count, bit for bit, on random
graphs of every shape (outer-join edges included), the chain, a star, the
cyclic snowflake at 1 % size, and keys equal to INT64_MIN."""
import numpy as np
import pytest
import torch

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


def check_exact(pt, prob, runs=1):
    dp = pt.DeviceProblem(prob)
    tr = pt.Transfer(dp, pt.params(flags=pt.PT_FLAG_EXACT))
    for _ in range(runs):
        tr.run()
    tr.check_status()
    ref = oracle.transfer(prob, kind=oracle.EXACT)
    counts = tr.counts.cpu().numpy()
    for t in range(prob.n_tables):
        assert_bitmaps_equal(tr.bitmap(t), ref.bitmaps[t], f"{prob.label} table {t}")
        assert counts[t] == ref.counts[t], (prob.label, t)
    return tr, ref


@pytest.mark.parametrize("shape", SHAPES)
def test_tiny_graphs(pt, shape):
    for s in range(20):
        prob = W.tiny_random(np.random.default_rng(97_000 + 1000 * SHAPES.index(shape) + s), shape,
                             outer=0.3 if s % 2 else 0.0)
        say(prob.label, s)
        check_exact(pt, prob, runs=2)


def test_workloads(pt):
    for prob in (W.chain(seed=3), W.star(seed=2, n_fact=2_000_000, dims=(200_000, 20_000, 1_000, 25), payload=0),
                 W.snowflake(seed=4, scale=0.01)):
        say(prob.label)
        tr, ref = check_exact(pt, prob)
        # an exact filter keeps no more rows than a Bloom filter would
        bloom = oracle.transfer(prob, 512, 3, 10)
        assert all(e <= b for e, b in zip(ref.counts, bloom.counts))


def test_int64_min_keys(pt):
    lo = np.iinfo(np.int64).min
    prob = W.Problem(["A", "B", "C"],
                     [{"k": np.array([lo, 1, 2, lo, 7], np.int64)},
                      {"k": np.array([lo, 2, 5], np.int64), "j": np.array([3, 4, 3], np.int32)},
                      {"j": np.array([3, 9, 3, 4], np.int32)}],
                     [(0, "k", 1, "k"), (1, "j", 2, "j")], [], label="int64 min keys")
    tr, ref = check_exact(pt, prob)
    assert ref.counts == [3, 2, 3]  # A: MIN, MIN, 2; B: rows 0 and 1; C: j in {3, 4}


def test_exact_rejected_where_unsupported(pt):
    prob = W.chain(seed=1)
    dp = pt.DeviceProblem(prob)
    p = pt.params(flags=pt.PT_FLAG_EXACT)
    tr = pt.Transfer(dp, p)
    tr.run()
    with pytest.raises(pt.PtError) as ei:
        tr.filter(1, 0)
    assert ei.value.status == pt.PT_EUNSUPPORTED
    with pytest.raises(pt.PtError) as ei:
        pt.Batch([dp], [p])
    assert ei.value.status == pt.PT_EUNSUPPORTED
