"""GPU serving: every query's bitmaps and counts are the same when it runs
alone (plain pt_transfer, one query at a time) and when it is served in a
mix (batched with other queries, batches overlapping on two streams), and
match the oracle on a sample."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_bitmaps_equal, say
from paper_2307_15255_amd import serve as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def resident():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return S.ResidentStar(seed=4, n_fact=2_000_000, dims=(200_000, 20_000, 1_000, 25))


def test_alone_and_in_the_mix_agree(resident):
    rng = np.random.default_rng(21)
    qs = [S.random_query(rng, i) for i in range(48)]
    for q, t in zip(qs, S.poisson_arrivals(rng, len(qs), qps=4000)):
        q.arrival = float(t)
    mixed = S.GpuExecutor(resident, slots=2, keep=True)
    say("serve mix")
    rep = S.serve(qs, mixed, budget_bytes=1 << 30, slots=2, max_batch=16)
    assert len(rep.batches) < len(qs)  # queries were batched
    assert any(len(ids) > 1 for _, ids, _ in rep.batches)
    alone = S.GpuExecutor(resident, keep=True)
    say("serve alone")
    S.one_at_a_time(qs, alone)
    torch.cuda.synchronize()
    for q in qs:
        bm_mix, cnt_mix = mixed.results[q.qid]
        bm_one, cnt_one = alone.results[q.qid]
        assert torch.equal(cnt_mix, cnt_one), q.qid
        for a, b in zip(bm_mix, bm_one):
            assert torch.equal(a, b), q.qid
    for q in qs[:4]:
        prob, _ = resident.problem(q)
        ref = oracle.transfer(prob)
        bm, cnt = mixed.results[q.qid]
        for t in range(prob.n_tables):
            assert_bitmaps_equal(bm[t].cpu().numpy().view(np.uint64), ref.bitmaps[t], f"{prob.label} table {t}")
        assert list(cnt.cpu().numpy()) == list(ref.counts)
