"""Per-launch HIP events: every launch of a transfer records one event pair
in mode 1, probe launches only in mode 2, and a selection of one (name,
table, pass) records that launch alone, once per transfer."""
import numpy as np
import pytest
import torch

from gpu_util import say
from paper_2307_15255_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_15255_amd import pt as ptmod
    return ptmod


def _records(pt, tr, mode, only=None, runs=1):
    if only:
        pt.pt_profile_only(*only)
    pt.pt_profile_enable(mode)
    try:
        for _ in range(runs):
            tr.run()
        torch.cuda.synchronize()
    finally:
        pt.pt_profile_enable(0)
        pt.pt_profile_only(None)
    return pt.pt_profile_read(1 << 12)


def test_profile_modes_and_selection(pt):
    prob = W.star(seed=7, n_fact=300_000, dims=(50_000, 5_000, 500, 25), payload=0)
    tr = pt.Transfer(pt.DeviceProblem(prob), pt.params(512, 3, 10))
    tr.run()
    torch.cuda.synchronize()
    say("profile mode 1")
    every = _records(pt, tr, 1)
    keys = {(r["name"], r["table"], r["pass_"]) for r in every}
    assert any(k[0] == "probe" for k in keys) and any(k[0] != "probe" for k in keys)
    assert all(r["ms"] >= 0 for r in every)
    say("profile mode 2")
    probes = _records(pt, tr, 2)
    assert probes and all("probe" in r["name"] for r in probes)
    fact = prob.table("F")
    key = ("probe", fact, 1)
    assert key in keys
    say("profile selection")
    sel = _records(pt, tr, 1, only=key, runs=3)
    assert len(sel) == 3 * sum(1 for r in every if (r["name"], r["table"], r["pass_"]) == key)
    assert all((r["name"], r["table"], r["pass_"]) == key for r in sel)
    assert np.mean([r["ms"] for r in sel]) > 0
    # cleared: every launch records again
    again = _records(pt, tr, 1)
    assert len(again) == len(every)
