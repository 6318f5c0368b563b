"""Autotuner of the filter parameters of a batch (block bits B, hash count
k, bits per key) and of its work-item size (rows per item).

The paper leaves the filter's configuration open (Sec. 3.5: the filter size
can be configured, trading its false-positive rate against its cost). Each
problem gets the (B, k, bits per key) that minimises its modelled time among
the settings whose false-positive rate (closed form for blocked filters
with k distinct bits per key, after Putze, Sanders and Singler 2007) is at
most `fpr_cap`. The model's per-row probe and per-key build costs are
measured on this GPU with the library's own kernels (`measure`), once per
device, and kept in a JSON cost table keyed by the device's name; with a
given cost table the choice is a function of the problem alone. The
candidates are the settings the batch kernel is specialised for (512-bit
blocks, k = 2 or 3), so a tuned batch never runs the generic kernel.

The rows per work item (`tile_rows`) are picked by `tune_tiles`: the batch
itself is timed with every candidate and the fastest is kept in a second
table keyed by the device and a digest of the batch (its tables, edges,
predicates and filter settings), so a batch seen before gets the same
choice without a measurement. Without a GPU measurement `tile_rows_for`
gives a rule of thumb from the batch's shape.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
from dataclasses import dataclass, field

import torch

BLOCK_BITS = (512,)
HASHES = (2, 3)
BITS_PER_KEY = tuple(range(6, 25))
SIZE_CLASSES = (20_000, 400_000, 4_000_000)  # filter keys the costs are measured at
TILE_ROWS = (32_768, 65_536, 131_072, 262_144)

_HERE = os.path.dirname(os.path.abspath(__file__))
# Saved cost tables, one per device (PT_TUNING_DIR overrides the folder).
COST_DIR = os.environ.get("PT_TUNING_DIR", os.path.join(_HERE, "tuning"))


def blocked_fpr(block_bits: int, k: int, bits_per_key: float) -> float:
    """False-positive rate of a blocked Bloom filter whose keys each set k
    distinct bits of one B-bit block: the number of keys in a block is
    Poisson with mean B / bits_per_key; after i keys a given bit is set with
    probability 1 - (1 - k/B)^i, and an absent key passes when its k bits
    are set."""
    lam = block_bits / bits_per_key
    total, i = 0.0, 0
    log_p = -lam  # log Pois(0)
    while True:
        p = math.exp(log_p)
        total += p * (1.0 - (1.0 - k / block_bits) ** i) ** k
        i += 1
        log_p += math.log(lam) - math.log(i)
        if i > lam and math.exp(log_p) < 1e-12:
            break
    return total


@dataclass
class CostTable:
    """Measured nanoseconds per probed row and per inserted key, by filter
    size class (keys) and setting (B, k, bits per key)."""
    probe: dict = field(default_factory=dict)   # (size, B, k, bpk) -> ns per probed row
    build: dict = field(default_factory=dict)   # (size, B, k, bpk) -> ns per inserted key
    device: str = ""

    def to_json(self) -> str:
        enc = lambda d: {",".join(map(str, key)): v for key, v in sorted(d.items())}
        return json.dumps({"device": self.device, "probe": enc(self.probe), "build": enc(self.build)}, indent=1)

    @staticmethod
    def from_json(text: str) -> "CostTable":
        raw = json.loads(text)
        dec = lambda d: {tuple(int(x) for x in key.split(",")): v for key, v in d.items()}
        return CostTable(dec(raw["probe"]), dec(raw["build"]), raw.get("device", ""))


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
    out = CostTable(device=device_name())
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


def device_name() -> str:
    """The key of a device's cost table: its architecture and CU count (the
    marketing name is not reported the same way on every host)."""
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(props, 'gcnArchName', props.name)} {props.multi_processor_count}cu"


def _cost_path(name: str) -> str:
    safe = "".join(c if c.isalnum() else "_" for c in name)
    return os.path.join(COST_DIR, f"costs_{safe}.json")


def load_or_measure(fpr_cap: float = 0.02) -> CostTable:
    """The cost table of this device: read from tuning/ when one was saved
    for it, else measured once and saved there."""
    path = _cost_path(device_name())
    if os.path.exists(path):
        with open(path) as f:
            return CostTable.from_json(f.read())
    costs = measure(fpr_cap=fpr_cap)
    os.makedirs(COST_DIR, exist_ok=True)
    with open(path + ".tmp", "w") as f:
        f.write(costs.to_json())
    os.replace(path + ".tmp", path)
    return costs


def modelled_ns(problem, costs: CostTable, setting: tuple[int, int, int]) -> float:
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
    if key not in costs.probe:
        return math.inf
    return work * (costs.probe[key] + costs.build[key])


def choose(problem, costs: CostTable, fpr_cap: float = 0.02) -> tuple[int, int, int]:
    """(block_bits, k, bits_per_key) for one problem (`workloads.Problem`):
    among the candidates within fpr_cap, the one with the lowest modelled
    time (ties broken by the setting's order)."""
    return min(candidates(fpr_cap), key=lambda c: (modelled_ns(problem, costs, c), c))


def tile_rows_for(problems, n_cu: int = 256) -> int:
    """Rows per work item: the largest candidate that still gives every CU
    four items of the batch's probe work (a function of the batch alone)."""
    rows = sum(p.n_rows(t) for p in problems for t in range(p.n_tables))
    for tr in sorted(TILE_ROWS, reverse=True):
        if rows / tr >= 4 * n_cu:
            return tr
    return min(TILE_ROWS)


def tune(problems, costs: CostTable | None = None, fpr_cap: float = 0.02, n_cu: int | None = None):
    """pt_params for every problem and the cost table used (the device's
    saved table, or measured and saved when there is none)."""
    from . import pt
    if costs is None:
        costs = load_or_measure(fpr_cap)
    if n_cu is None:
        n_cu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    picks = [choose(p, costs, fpr_cap) for p in problems]
    # A batch runs one kernel: the specialised one when every problem shares
    # (B, k). A problem takes the most common (B, k) when its fewest bits
    # per key for that pair cost at most 3 % more.
    if picks:
        common_bk = max(sorted({c[:2] for c in picks}), key=lambda bk: sum(c[:2] == bk for c in picks))
        alt = {c[:2]: c for c in candidates(fpr_cap)}[common_bk]
        picks = [alt if modelled_ns(p, costs, alt) <= 1.03 * modelled_ns(p, costs, c) else c
                 for p, c in zip(problems, picks)]
    tile = tile_rows_for(problems, n_cu)
    return [pt.params(*c, tile_rows=tile) for c in picks], costs


def batch_digest(problems, params) -> str:
    """A digest of a batch: every problem's table sizes, edges, edge kinds,
    predicates and filter settings."""
    h = hashlib.sha256()
    for prob, p in zip(problems, params):
        rows = [prob.n_rows(t) for t in range(prob.n_tables)]
        h.update(repr((rows, prob.edges, prob.edge_flags, prob.orient, prob.preds,
                       (p.block_bits, p.k, p.bits_per_key, p.flags))).encode())
    return h.hexdigest()[:32]


def _tiles_path(name: str) -> str:
    safe = "".join(c if c.isalnum() else "_" for c in name)
    return os.path.join(COST_DIR, f"tiles_{safe}.json")


def tune_tiles(dps, params, reps: int = 5) -> tuple[list, dict]:
    """The batch's parameters with the fastest rows per work item. A choice
    saved for this device and batch digest is reused; otherwise the batch
    runs with every candidate in TILE_ROWS (two warm-up runs, then the
    median of `reps`) and the fastest is saved. The bits do not depend on
    this choice. Returns the parameters and a record of the choice."""
    from . import pt
    digest = batch_digest([dp.problem for dp in dps], params)
    path = _tiles_path(device_name())
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    times = None
    if digest in table:
        best = int(table[digest]["tile_rows"])
    else:
        times = {}
        for tr in TILE_ROWS:
            ps = [pt.params(p.block_bits, p.k, p.bits_per_key, p.flags, hash_version=p.hash_version,
                            lds_budget=p.lds_budget, tile_rows=tr, probe_order=p.probe_order) for p in params]
            bt = pt.Batch(dps, ps)
            for _ in range(2):
                bt.run()
            runs = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                bt.run()
                b.record()
                b.synchronize()
                runs.append(a.elapsed_time(b))
            bt.close()
            del bt
            times[tr] = sorted(runs)[len(runs) // 2]
        best = min(TILE_ROWS, key=lambda tr: (times[tr], tr))
        table[digest] = {"tile_rows": best, "ms": {str(k): round(v, 4) for k, v in times.items()}}
        os.makedirs(COST_DIR, exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    out = [pt.params(p.block_bits, p.k, p.bits_per_key, p.flags, hash_version=p.hash_version,
                     lds_budget=p.lds_budget, tile_rows=best, probe_order=p.probe_order) for p in params]
    return out, {"tile_rows": best, "digest": digest, "measured_ms": times}
