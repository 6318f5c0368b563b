"""The allocation-free compaction (pt_compact_noalloc, static device scratch)
against pt_compact with a caller workspace: the same ascending row ids and
count, bit for bit, on two calls in a row (the second smaller, so stale
partial counts in the shared scratch would show), plus an empty input."""
import numpy as np
import pytest
import torch

from gpu_util import bitmap_tensor, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_15255_amd import pt as ptmod
    return ptmod


def _bits(rng, n, density):
    """A bitmap of n rows (row r = bit r % 64 of word r // 64), tail bits 0."""
    words = (n + 63) // 64
    bits = rng.random(words * 64) < density
    bits[n:] = False
    return np.packbits(bits, bitorder="little").view("<u8").astype(np.uint64)


def _with_workspace(pt, bm, n):
    idx = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    ws = torch.empty(pt.pt_compact_workspace_size(n), dtype=torch.uint8, device="cuda")
    pt.pt_compact(bm, n, idx, cnt, ws)
    return idx, cnt


def _without(pt, bm, n):
    idx = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    pt.pt_compact_noalloc(bm, n, idx, cnt)
    return idx, cnt


def test_noalloc_compaction_matches_the_workspace_one(pt):
    rng = np.random.default_rng(2024)
    for n, density in [(3_000_017, 0.3), (100_003, 0.02), (0, 0.5), (65, 1.0), (4_194_304, 0.001)]:
        say("compact_noalloc", n, density)
        host = _bits(rng, n, density) if n else np.zeros(1, np.uint64)
        bm = bitmap_tensor(host)
        idx_a, cnt_a = _with_workspace(pt, bm, n)
        idx_b, cnt_b = _without(pt, bm, n)
        torch.cuda.synchronize()
        c = int(cnt_a.item())
        assert int(cnt_b.item()) == c
        assert torch.equal(idx_a[:c], idx_b[:c])
        if n:
            expect = np.flatnonzero(np.unpackbits(host.view(np.uint8), bitorder="little")[:n]).astype(np.int32)
            assert c == len(expect)
            assert np.array_equal(idx_b[:c].cpu().numpy(), expect)
