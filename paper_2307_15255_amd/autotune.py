"""Autotuner of the filter parameters of a batch (block bits B, hash count
k, bits per key).

The paper leaves the filter's configuration open (Sec. 3.3: the filter size
can be configured). Here each problem gets the (B, k, bits per key) that
minimises its modelled time among the settings whose false-positive rate
(closed form for blocked filters, Putze, Sanders and Singler 2007) is at
most `fpr_cap`. The model's per-row probe and per-key build costs are
measured on this GPU with the library's own kernels (`measure`), once per
device; the choice is then a function of the problem's shape only, so the
same problem always gets the same parameters for a given cost table.
"""
from __future__ import annotations

import json
import math
import time
from dataclasses import dataclass, field

import torch

BLOCK_BITS = (256, 512)
HASHES = (2, 3, 4)
BITS_PER_KEY = tuple(range(6, 17))


def blocked_fpr(block_bits: int, k: int, bits_per_key: float) -> float:
    """False-positive rate of a blocked Bloom filter: the number of keys in
    a block is Poisson with mean B / bits_per_key, and a block holding i
    keys answers yes for an absent key with probability
    (1 - (1 - 1/B)^(k i))^k."""
    lam = block_bits / bits_per_key
    total, i = 0.0, 0
    log_p = -lam  # log Pois(0)
    while True:
        p = math.exp(log_p)
        total += p * (1.0 - (1.0 - 1.0 / block_bits) ** (k * i)) ** k
        i += 1
        log_p += math.log(lam) - math.log(i)
        if i > lam and math.exp(log_p) < 1e-12:
            break
    return total


@dataclass
class CostTable:
    """Measured nanoseconds per probed row and per inserted key, by (B, k)
    and by where the probe's filters live (LDS or global memory)."""
    probe_lds: dict = field(default_factory=dict)
    probe_global: dict = field(default_factory=dict)
    build: dict = field(default_factory=dict)

    def to_json(self) -> str:
        enc = lambda d: {f"{b},{k}": v for (b, k), v in d.items()}
        return json.dumps({"probe_lds": enc(self.probe_lds), "probe_global": enc(self.probe_global),
                           "build": enc(self.build)})

    @staticmethod
    def from_json(text: str) -> "CostTable":
        raw = json.loads(text)
        dec = lambda d: {tuple(int(x) for x in key.split(",")): v for key, v in d.items()}
        return CostTable(dec(raw["probe_lds"]), dec(raw["probe_global"]), dec(raw["build"]))


def _time_ms(fn, reps: int = 5) -> float:
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def measure(n_rows: int = 1 << 24, small_keys: int = 20_000, large_keys: int = 2_000_000,
            device: str = "cuda") -> CostTable:
    """Times pt_bloom_build and pt_bloom_probe for every (B, k): a probe of
    n_rows int32 keys against a filter of small_keys keys (held in LDS) and
    one of large_keys keys (read from L2 / HBM), and a build of large_keys
    keys."""
    from . import pt
    g = torch.Generator(device=device).manual_seed(7)
    probe_keys = torch.randint(0, 1 << 30, (n_rows,), dtype=torch.int32, device=device, generator=g)
    bitmap = torch.empty(pt.bitmap_words(n_rows), dtype=torch.int64, device=device)
    count = torch.zeros(1, dtype=torch.int64, device=device)
    out = CostTable()
    for B in BLOCK_BITS:
        for k in HASHES:
            p = pt.params(B, k, 10)
            for keys_n, table in ((small_keys, out.probe_lds), (large_keys, out.probe_global)):
                keys = probe_keys[:keys_n].contiguous()
                f = pt.Bloom(keys_n, p, device)
                pt.pt_bloom_build([keys], [f], keys_n)

                def probe():
                    bitmap.fill_(-1)
                    pt.pt_bloom_probe([probe_keys], [f], n_rows, bitmap, count)
                fill = _time_ms(lambda: bitmap.fill_(-1))
                table[(B, k)] = max(0.0, _time_ms(probe) - fill) * 1e6 / n_rows
            keys = probe_keys[:large_keys].contiguous()
            f = pt.Bloom(large_keys, p, device)
            out.build[(B, k)] = _time_ms(lambda: pt.pt_bloom_build([keys], [f], large_keys)) * 1e6 / large_keys
    return out


# LDS words a probe may stage its filters in (a little under 160 KB).
LDS_WORDS = 36_000


def choose(problem, costs: CostTable, fpr_cap: float = 0.02):
    """(block_bits, k, bits_per_key) for one problem (`workloads.Problem`):
    the cheapest modelled setting with blocked_fpr <= fpr_cap."""
    n = [problem.n_rows(t) for t in range(problem.n_tables)]
    # Work of the schedule, from the shape only: every edge is probed once
    # per pass at each end's table and built from the other end's rows.
    probe_rows, build_keys, max_filter_keys = 0, 0, 0
    for u, _, v, _ in problem.edges:
        probe_rows += n[u] + n[v]
        build_keys += n[u] + n[v]
        max_filter_keys = max(max_filter_keys, min(n[u], n[v]))
    best = None
    for B in BLOCK_BITS:
        for k in HASHES:
            for bpk in BITS_PER_KEY:
                fpr = blocked_fpr(B, k, bpk)
                if fpr > fpr_cap:
                    continue
                words = max_filter_keys * bpk / 32
                probe = costs.probe_lds if words <= LDS_WORDS else costs.probe_global
                t = probe_rows * probe[(B, k)] + build_keys * costs.build[(B, k)]
                # more bits per key only costs filter memory: prefer fewer on ties
                key = (round(t, 3), bpk, fpr)
                if best is None or key < best[0]:
                    best = (key, (B, k, bpk))
    if best is None:
        raise ValueError(f"no setting reaches a false-positive rate of {fpr_cap}")
    return best[1]


def tune(problems, costs: CostTable | None = None, fpr_cap: float = 0.02):
    """pt_params for every problem (measuring the cost table first when none
    is given) and the table used."""
    from . import pt
    if costs is None:
        t0 = time.time()
        costs = measure()
        costs.seconds = time.time() - t0
    return [pt.params(*choose(p, costs, fpr_cap)) for p in problems], costs
