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


SIZE_CLASSES = (20_000, 400_000, 4_000_000)  # filter keys the costs are measured at


@dataclass
class CostTable:
    """Measured nanoseconds per probed row and per inserted key, by filter
    size class (keys) and setting (B, k, bits per key)."""
    probe: dict = field(default_factory=dict)   # (size, B, k, bpk) -> ns per probed row
    build: dict = field(default_factory=dict)   # (size, B, k, bpk) -> ns per inserted key

    def to_json(self) -> str:
        enc = lambda d: {",".join(map(str, key)): v for key, v in d.items()}
        return json.dumps({"probe": enc(self.probe), "build": enc(self.build)})

    @staticmethod
    def from_json(text: str) -> "CostTable":
        raw = json.loads(text)
        dec = lambda d: {tuple(int(x) for x in key.split(",")): v for key, v in d.items()}
        return CostTable(dec(raw["probe"]), dec(raw["build"]))


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


def candidates(fpr_cap: float) -> list[tuple[int, int, int]]:
    """For every (B, k): the fewest bits per key whose false-positive rate
    is within the cap (more bits only make the filter larger)."""
    out = []
    for B in BLOCK_BITS:
        for k in HASHES:
            for bpk in BITS_PER_KEY:
                if blocked_fpr(B, k, bpk) <= fpr_cap:
                    out.append((B, k, bpk))
                    break
    return out


def measure(fpr_cap: float = 0.02, sizes: tuple[int, ...] = SIZE_CLASSES, n_rows: int = 1 << 24,
            device: str = "cuda") -> CostTable:
    """Times pt_bloom_probe (n_rows int32 keys) and pt_bloom_build for every
    candidate setting with filters of each size class: the filter's size
    decides whether it is read from LDS, L2 or beyond, so each size is
    measured."""
    from . import pt
    g = torch.Generator(device=device).manual_seed(7)
    probe_keys = torch.randint(0, 1 << 30, (n_rows,), dtype=torch.int32, device=device, generator=g)
    bitmap = torch.empty(pt.bitmap_words(n_rows), dtype=torch.int64, device=device)
    count = torch.zeros(1, dtype=torch.int64, device=device)
    out = CostTable()
    fill = _time_ms(lambda: bitmap.fill_(-1))
    for size in sizes:
        keys = probe_keys[:size].contiguous()
        for B, k, bpk in candidates(fpr_cap):
            f = pt.Bloom(size, pt.params(B, k, bpk), device)
            pt.pt_bloom_build([keys], [f], size)

            def probe():
                bitmap.fill_(-1)
                pt.pt_bloom_probe([probe_keys], [f], n_rows, bitmap, count)
            out.probe[(size, B, k, bpk)] = max(0.0, _time_ms(probe) - fill) * 1e6 / n_rows
            out.build[(size, B, k, bpk)] = _time_ms(lambda: pt.pt_bloom_build([keys], [f], size)) * 1e6 / size
    return out


def modelled_ms(problem, costs: CostTable, setting: tuple[int, int, int]) -> float:
    """Modelled time of `problem` with `setting`, from the costs at the
    size class nearest (in log scale) to the problem's median table. Every
    edge is probed once per pass at each end's table and built from the
    other end's rows."""
    n = sorted(problem.n_rows(t) for t in range(problem.n_tables))
    median = max(1, n[len(n) // 2])
    sizes = sorted({key[0] for key in costs.probe})
    if not sizes:
        raise ValueError("empty cost table")
    size = min(sizes, key=lambda c: abs(math.log(c) - math.log(median)))
    rows = [problem.n_rows(t) for t in range(problem.n_tables)]
    work = sum(rows[u] + rows[v] for u, _, v, _ in problem.edges)
    key = (size, *setting)
    return work * (costs.probe[key] + costs.build[key]) * 1e-6


def choose(problem, costs: CostTable, fpr_cap: float = 0.02):
    """(block_bits, k, bits_per_key) for one problem (`workloads.Problem`):
    the measured setting (all within fpr_cap) with the lowest modelled time,
    using the costs measured at the size class nearest (in log scale) to the
    problem's median table. Model: every edge is probed once per pass at
    each end's table and built from the other end's rows."""
    n = sorted(problem.n_rows(t) for t in range(problem.n_tables))
    median = max(1, n[len(n) // 2])
    sizes = sorted({key[0] for key in costs.probe})
    if not sizes:
        raise ValueError("empty cost table")
    size = min(sizes, key=lambda c: abs(math.log(c) - math.log(median)))
    rows = [problem.n_rows(t) for t in range(problem.n_tables)]
    work = sum(rows[u] + rows[v] for u, _, v, _ in problem.edges)
    best = None
    for key in sorted(k for k in costs.probe if k[0] == size):
        t = work * (costs.probe[key] + costs.build[key])
        if best is None or t < best[0]:
            best = (t, key[1:])
    return best[1]


def tune(problems, costs: CostTable | None = None, fpr_cap: float = 0.02):
    """pt_params for every problem and the cost table used (measured first
    when none is given)."""
    from . import pt
    if costs is None:
        costs = measure(fpr_cap=fpr_cap)
    picks = [choose(p, costs, fpr_cap) for p in problems]
    # Settings that differ in B or k run in separate launches of a batch: a
    # problem takes the most common setting when it costs at most 3 % more.
    if picks:
        common = max(set(picks), key=picks.count)
        picks = [common if modelled_ms(p, costs, common) <= 1.03 * modelled_ms(p, costs, c) else c
                 for p, c in zip(problems, picks)]
    return [pt.params(*c) for c in picks], costs
