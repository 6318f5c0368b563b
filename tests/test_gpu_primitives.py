"""GPU parity of each C-ABI entry point against the oracle, bit for bit:
local filter, Bloom build (every filter word), Bloom probe (bitmap and
count), compaction. Sizes span several workgroups and ragged tails."""
import numpy as np
import pytest
import torch

import oracle
import refcheck as rc
from gpu_util import assert_bitmaps_equal, bitmap_tensor, dev, host_u64, say

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 63, 64, 65, 1000, 4097, 100_003, 1_000_001]


@pytest.fixture(scope="module")
def pt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_15255_amd import pt as ptmod
    return ptmod


def _keys(rng, n, dtype, domain=None):
    if domain is None:
        info = np.iinfo(dtype)
        return rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
    return rng.integers(-domain, domain, n).astype(dtype)


@pytest.mark.parametrize("n", SIZES)
def test_local_filter(pt, n):
    rng = np.random.default_rng(n)
    c32 = rng.integers(-1000, 1000, n).astype(np.int32)
    c64 = (rng.integers(-1000, 1000, n) * (1 << 35)).astype(np.int64)
    cases = [[], [(0, "lt", 5, 0)], [(1, "between", -(1 << 40), 1 << 40)], [(0, "ne", 7, 0), (1, "ge", 0, 0)],
             [(0, "gt", -900, 0)] * 3 + [(0, "lt", 900, 0)] * 3 + [(1, "le", 1 << 44, 0)] * 4,  # 10 > one launch
             [(0, "eq", 3, 0)], [(0, "lt", 1 << 40, 0)]]
    d32, d64 = dev(c32), dev(c64)
    for preds in cases:
        say("local", n, preds)
        bm = torch.full((max(1, (n + 63) // 64),), -1, dtype=torch.int64, device="cuda")
        cnt = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
        pt.pt_local_filter([d32, d64], preds, n, bm, cnt)
        ref, rcnt = oracle.local_filter([c32, c64], preds)
        assert_bitmaps_equal(host_u64(bm)[:len(ref)], ref, f"local {preds}")
        assert int(cnt.item()) == rcnt


@pytest.mark.parametrize("B,k,bpk", [(512, 3, 10), (32, 1, 1), (64, 3, 8), (128, 2, 4), (256, 5, 12),
                                     (1024, 16, 64), (512, 7, 16), (1024, 3, 10)])
@pytest.mark.parametrize("n", [0, 1, 65, 4097, 200_001])
def test_build_words_match(pt, B, k, bpk, n):
    rng = np.random.default_rng(B * 7 + k + n)
    p = pt.params(B, k, bpk)
    for dtype in (np.int32, np.int64):
        keys = _keys(rng, n, dtype)
        for selected in (None, 0.3, 0.0):
            say("build", B, k, bpk, n, dtype.__name__, selected)
            f = pt.Bloom(n, p)
            f.words.fill_(-1)  # garbage beyond the used blocks must not matter
            if selected is None:
                pt.pt_bloom_build([dev(keys)], [f], n)
                ref, nb = oracle.bloom_build(keys, None, B, k, bpk)
            else:
                mask = rng.random(n) < selected
                bits = rc.rows_to_bits(np.nonzero(mask)[0], n)
                cnt = torch.tensor([int(mask.sum())], dtype=torch.int64, device="cuda")
                pt.pt_bloom_build([dev(keys)], [f], n, bitmap_tensor(bits) if n else None, cnt)
                ref, nb = oracle.bloom_build(keys, bits if n else None, B, k, bpk)
            torch.cuda.synchronize()
            assert int(f.nb.item()) == nb
            assert np.array_equal(f.used_words(), ref)


def test_build_many_filters_one_call(pt):
    """Nine outgoing filters from one scan (more than one launch's worth)."""
    rng = np.random.default_rng(9)
    n = 50_000
    cols = [_keys(rng, n, np.int32 if i % 2 else np.int64, domain=10_000) for i in range(9)]
    mask = rng.random(n) < 0.5
    bits = rc.rows_to_bits(np.nonzero(mask)[0], n)
    cnt = torch.tensor([int(mask.sum())], dtype=torch.int64, device="cuda")
    p = pt.params()
    fs = [pt.Bloom(n, p) for _ in cols]
    pt.pt_bloom_build([dev(c) for c in cols], fs, n, bitmap_tensor(bits), cnt)
    for c, f in zip(cols, fs):
        ref, nb = oracle.bloom_build(c, bits, 512, 3, 10)
        assert int(f.nb.item()) == nb and np.array_equal(f.used_words(), ref)


@pytest.mark.parametrize("B,k", [(512, 3), (32, 1), (64, 4), (256, 3), (1024, 9)])
@pytest.mark.parametrize("n", [0, 1, 63, 65, 4097, 300_007, 2_000_003])
def test_probe_matches(pt, B, k, n):
    """Probing 1 to 6 filters at once (int32 and int64 key columns, a small
    filter staged in LDS and a large one read from global memory, an initial
    bitmap with holes) leaves the oracle's bitmap and count."""
    rng = np.random.default_rng(B + k + n)
    p = pt.params(B, k, 10)
    n_filters = 1 + n % 6
    cols, filters, refs = [], [], []
    for i in range(n_filters):
        dtype = np.int64 if i % 3 == 1 else np.int32
        build_n = [50, 20_000, 3_000_000][i % 3]   # 3M keys -> ~3.7 MB filter, not staged
        members = _keys(rng, build_n, dtype, domain=4_000_000)
        f = pt.Bloom(build_n, p)
        pt.pt_bloom_build([dev(members)], [f], build_n)
        ref_words, nb = oracle.bloom_build(members, None, B, k, 10)
        probe = _keys(rng, n, dtype, domain=4_000_000)
        cols.append(probe)
        filters.append(f)
        refs.append((ref_words, nb))
    start = rng.random(n) < 0.9
    bits = rc.rows_to_bits(np.nonzero(start)[0], n)
    say("probe", B, k, n, n_filters)
    bm = bitmap_tensor(bits) if n else torch.zeros(1, dtype=torch.int64, device="cuda")
    cnt = torch.full((1,), 777, dtype=torch.int64, device="cuda")
    pt.pt_bloom_probe([dev(c) for c in cols], filters, n, bm, cnt)
    ref = bits.copy()
    for c, (w, nb) in zip(cols, refs):
        ref, rcnt = oracle.bloom_probe(c, w, nb, B, k, ref)
    if n == 0:
        rcnt = 0
    assert_bitmaps_equal(host_u64(bm)[:len(ref)], ref, "probe")
    assert int(cnt.item()) == rcnt


@pytest.mark.parametrize("first_pass", [1.0, 0.5, 0.05, 0.0])
def test_probe_first_filter_pass_rates(pt, first_pass):
    """The first filter passing everything, half, few or none of the rows
    (queue overflow, queue, and empty paths of the probe), with int32 and
    int64 columns mixed in one launch."""
    rng = np.random.default_rng(int(first_pass * 100))
    n = 777_777
    p = pt.params()
    domain = 100_000
    cols = [rng.integers(0, domain, n).astype(np.int32), rng.integers(0, domain, n).astype(np.int64),
            rng.integers(0, domain, n).astype(np.int32)]
    members = [np.arange(int(domain * first_pass), dtype=np.int32),
               rng.integers(0, domain, domain // 3).astype(np.int64),
               rng.integers(0, domain, domain // 2).astype(np.int32)]
    filters, refs = [], []
    for m in members:
        f = pt.Bloom(max(1, len(m)), p)
        pt.pt_bloom_build([dev(m)], [f], len(m))
        filters.append(f)
        refs.append(oracle.bloom_build(m, None, 512, 3, 10))
    say("probe first pass", first_pass)
    bm = bitmap_tensor(oracle.all_rows_bitmap(n))
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    pt.pt_bloom_probe([dev(c) for c in cols], filters, n, bm, cnt)
    ref = oracle.all_rows_bitmap(n)
    for c, (w, nb) in zip(cols, refs):
        ref, rcnt = oracle.bloom_probe(c, w, nb, 512, 3, ref)
    assert_bitmaps_equal(host_u64(bm), ref, "probe")
    assert int(cnt.item()) == rcnt


@pytest.mark.parametrize("n", SIZES + [65536 * 3 + 17])
def test_compact(pt, n):
    rng = np.random.default_rng(n + 5)
    for density in (0.0, 0.01, 0.5, 1.0):
        say("compact", n, density)
        mask = rng.random(n) < density
        bits = rc.rows_to_bits(np.nonzero(mask)[0], n)
        idx = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws = torch.empty(pt.pt_compact_workspace_size(n), dtype=torch.uint8, device="cuda")
        bm = bitmap_tensor(bits) if n else torch.zeros(1, dtype=torch.int64, device="cuda")
        pt.pt_compact(bm, n, idx, cnt, ws)
        ref = oracle.compact(bits, n)
        c = int(cnt.item())
        assert c == len(ref)
        assert np.array_equal(idx[:c].cpu().numpy().view(np.uint32), ref)


def test_rejects_bad_arguments_before_launch(pt):
    p = pt.params()
    f = pt.Bloom(10, p)
    keys = dev(np.arange(100, dtype=np.int32))
    with pytest.raises(pt.PtError) as ei:   # capacity for 10 keys, 100 rows
        pt.pt_bloom_build([keys], [f], 100)
    assert ei.value.status == pt.PT_EINVAL
    bm = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(pt.PtError):         # a bitmap without its count
        pt.pt_bloom_build([keys], [pt.Bloom(100, p)], 100, bm, None)


def test_overflow_is_reported(pt):
    """A count above the filter's capacity, or a block count above it, is
    clamped on the device and reported through the status word."""
    n = 5000
    rng = np.random.default_rng(77)
    keys = dev(rng.integers(0, 1 << 30, n).astype(np.int32))
    p = pt.params()
    f = pt.Bloom(n, p)
    bm = torch.full(((n + 63) // 64,), -1, dtype=torch.int64, device="cuda")
    bm[-1] = (1 << (n % 64)) - 1
    cnt = torch.tensor([n], dtype=torch.int64, device="cuda")
    say("overflow: clean build and probe")
    pt.pt_bloom_build([keys], [f], n, bm, cnt)
    pt.pt_check_status(f.status)
    probe_bm = bm.clone()
    pt.pt_bloom_probe([keys], [f], n, probe_bm)
    pt.pt_check_status(f.status)
    assert torch.equal(probe_bm, bm)  # no false negatives
    say("overflow: count above the capacity")
    cnt.fill_(4 * n)
    pt.pt_bloom_build([keys], [f], n, bm, cnt)
    with pytest.raises(pt.PtError) as ei:
        pt.pt_check_status(f.status)
    assert ei.value.status == pt.PT_EOVERFLOW
    assert int(f.nb.item()) == f.cap_words // (p.block_bits // 32)  # clamped to the capacity
    pt.pt_check_status(f.status)  # the read cleared it
    say("overflow: block count above the capacity")
    f.nb.fill_(1 << 40)
    pt.pt_bloom_probe([keys], [f], n, probe_bm)
    with pytest.raises(pt.PtError):
        pt.pt_check_status(f.status)
