"""Seeded synthetic inputs for the predicate-transfer phase.

This module only describes problems and draws random inputs. It holds none of
the method's arithmetic (no hashing, no filtering, no orientation), so both
the GPU path and the CPU oracle can take their inputs from it.

A problem is a join graph (Sec. 3.1: vertices are tables, edges are
equi-joins) with local predicates on base tables (Sec. 3.4). The workloads
stand in for the paper's TPC-H measurements (Sec. 4.1) with synthetic chain,
star and snowflake schemas; no TPC-H data is used or recreated.

Random streams: numpy ``Generator(PCG64)`` seeded from ``SeedSequence(seed)``,
one spawned child stream per table so tables are independent of each other.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

OPS = ("lt", "le", "gt", "ge", "eq", "ne", "between")


@dataclass
class Problem:
    """Tables (ordered name -> column dict), undirected join edges
    ``(u, u_col, v, v_col)``, predicates ``(table, col, op, lo, hi)`` (a
    conjunction per table, values compared as int64) and an optional explicit
    orientation (+1: u -> v, -1: v -> u per edge)."""

    names: list[str]
    columns: list[dict[str, np.ndarray]]
    edges: list[tuple[int, str, int, str]]
    preds: list[tuple[int, str, str, int, int]] = field(default_factory=list)
    orient: list[int] | None = None
    label: str = ""
    # per edge: 0 inner join, 1 u LEFT JOIN v, 2 u RIGHT JOIN v, 3 full outer
    edge_flags: list[int] | None = None

    @property
    def n_tables(self) -> int:
        return len(self.names)

    def n_rows(self, t: int) -> int:
        cols = self.columns[t]
        return len(next(iter(cols.values()))) if cols else 0

    def col_index(self, t: int, name: str) -> int:
        return list(self.columns[t].keys()).index(name)

    def table(self, name: str) -> int:
        return self.names.index(name)

    def validate(self) -> None:
        for t, cols in enumerate(self.columns):
            lens = {len(a) for a in cols.values()}
            if len(lens) > 1:
                raise ValueError(f"table {self.names[t]}: columns of unequal length")
            for a in cols.values():
                if a.dtype not in (np.int32, np.int64):
                    raise ValueError("columns must be int32 or int64")
        for u, uc, v, vc in self.edges:
            assert u != v and uc in self.columns[u] and vc in self.columns[v]
        for t, c, op, lo, hi in self.preds:
            assert c in self.columns[t] and op in OPS


def _streams(seed: int, n: int) -> list[np.random.Generator]:
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


def _uniform_i32(rng: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    return rng.integers(lo, hi, size=n, dtype=np.int32)


# --------------------------------------------------------------------- chain

def chain(seed: int = 1, n_r: int = 1000, n_s: int = 10_000, n_t: int = 1000, domain: int = 2000,
          keep: float = 0.10) -> Problem:
    """Three-table chain R(a, p) - S(a, b) - T(b).

    a and b are int32 uniform on [0, domain); p is int32 uniform on
    [0, 10^6) and the predicate ``p < keep * 10^6`` keeps about `keep` of R.
    """
    g = _streams(seed, 3)
    R = {"a": _uniform_i32(g[0], 0, domain, n_r), "p": _uniform_i32(g[0], 0, 1_000_000, n_r)}
    S = {"a": _uniform_i32(g[1], 0, domain, n_s), "b": _uniform_i32(g[1], 0, domain, n_s)}
    T = {"b": _uniform_i32(g[2], 0, domain, n_t)}
    return Problem(["R", "S", "T"], [R, S, T], [(0, "a", 1, "a"), (1, "b", 2, "b")],
                   [(0, "p", "lt", int(keep * 1_000_000), 0)],
                   label=f"chain R{n_r}-S{n_s}-T{n_t} int32 keys U[0,{domain}) keep {keep:g}")


# ---------------------------------------------------------------------- star

STAR_DIMS = (2_000_000, 200_000, 10_000, 25)


def star(seed: int = 1, n_fact: int = 100_000_000, dims: tuple[int, ...] = STAR_DIMS,
         keeps: tuple[float | None, ...] = (0.01, 0.20, None, None), payload: int = 2,
         key64: tuple[bool, ...] = ()) -> Problem:
    """Star schema: a fact table with one int32 foreign key per dimension,
    uniform over that dimension's keys, plus `payload` int32 columns.

    Dimension d has a primary key 0..n_d-1 stored in shuffled order and an
    int32 attribute uniform on [0, 10^6); ``keeps[d]`` (if set) adds the range
    predicate ``attr < keeps[d] * 10^6``. ``key64[d]`` stores that edge's two
    key columns as int64 instead.
    """
    nd = len(dims)
    g = _streams(seed, nd + 1)
    fact: dict[str, np.ndarray] = {}
    for d, n in enumerate(dims):
        wide = d < len(key64) and key64[d]
        fk = g[0].integers(0, n, size=n_fact, dtype=np.int64 if wide else np.int32)
        fact[f"k{d}"] = fk
    for j in range(payload):
        fact[f"p{j}"] = _uniform_i32(g[0], 0, 1 << 30, n_fact)
    names, columns, edges, preds = ["F"], [fact], [], []
    for d, n in enumerate(dims):
        wide = d < len(key64) and key64[d]
        pk = g[d + 1].permutation(n).astype(np.int64 if wide else np.int32)
        attr = _uniform_i32(g[d + 1], 0, 1_000_000, n)
        names.append(f"D{d}")
        columns.append({"pk": pk, "attr": attr})
        edges.append((0, f"k{d}", d + 1, "pk"))
        if d < len(keeps) and keeps[d] is not None:
            preds.append((d + 1, "attr", "lt", int(round(keeps[d] * 1_000_000)), 0))
    return Problem(names, columns, edges, preds,
                   label=f"star fact {n_fact} rows, dims {list(dims)}, keeps {list(keeps)}")


# ----------------------------------------------------------------- snowflake

SNOWFLAKE_ROWS = {"F": 200_000_000, "D1": 50_000_000, "D2": 10_000_000, "D3": 2_000_000,
                  "D4": 500_000, "D5": 100_000, "D6": 10_000, "D7": 1_000}
# (table, fk column) -> referenced dimension; D2.k3 -> D3 closes the cycle F - D2 - D3
SNOWFLAKE_FKS = [("F", "k1", "D1"), ("F", "k2", "D2"), ("F", "k3", "D3"), ("D2", "k3", "D3"),
                 ("D1", "k4", "D4"), ("D2", "k5", "D5"), ("D3", "k6", "D6"), ("D5", "k7", "D7")]
SNOWFLAKE_KEEPS = {"D3": 0.005, "D5": 0.05, "D7": 0.10, "D6": 0.30}
_SCRAMBLE = 0xD6E8FEB86659FD93  # odd: multiplication by it is a bijection of uint64


def scrambled_ids(ids: np.ndarray) -> np.ndarray:
    """Dense ids mapped to int64 keys with non-zero high words (a fixed
    bijection of the 64-bit integers), so that equal ids give equal keys."""
    with np.errstate(over="ignore"):
        return (ids.astype(np.uint64) * np.uint64(_SCRAMBLE) + np.uint64(0x9E37)).view(np.int64)


def snowflake(seed: int = 1, scale: float = 1.0, zipf_s: float = 1.1) -> Problem:
    """Cyclic snowflake of eight tables: fact F with foreign keys into D1, D2,
    D3; D2 also references D3 (a three-table cycle F - D2 - D3); D1 -> D4,
    D2 -> D5, D3 -> D6, D5 -> D7. Every key is int64. A dimension's primary
    key is its scrambled dense id; a foreign key is the scrambled id of a
    Zipf(zipf_s)-distributed rank, mapped to ids by a seeded permutation.
    Range predicates keep 0.5 % of D3, 5 % of D5, 10 % of D7, 30 % of D6.
    `scale` shrinks every table (at least 1 000 rows, 100 for the smallest)."""
    names = list(SNOWFLAKE_ROWS)
    rows = {t: max(min(n, 100) if n <= 1000 else 1000, int(round(n * scale))) for t, n in SNOWFLAKE_ROWS.items()}
    g = dict(zip(names, _streams(seed, len(names))))
    columns: dict[str, dict[str, np.ndarray]] = {t: {} for t in names}
    rank_to_id = {}
    for t in names:
        if t != "F":
            n = rows[t]
            columns[t]["pk"] = scrambled_ids(g[t].permutation(n))
            columns[t]["attr"] = _uniform_i32(g[t], 0, 1_000_000, n)
            rank_to_id[t] = g[t].permutation(n)
    for t, c, ref in SNOWFLAKE_FKS:
        ranks = zipf_ranks(g[t], rows[ref], zipf_s, rows[t])
        columns[t][c] = scrambled_ids(rank_to_id[ref][ranks])
    edges = [(names.index(t), c, names.index(ref), "pk") for t, c, ref in SNOWFLAKE_FKS]
    preds = [(names.index(t), "attr", "lt", int(round(keep * 1_000_000)), 0)
             for t, keep in SNOWFLAKE_KEEPS.items()]
    return Problem(names, [columns[t] for t in names], edges, preds,
                   label=f"snowflake scale {scale:g} (F {rows['F']} rows), int64 Zipf({zipf_s}) keys")


# ------------------------------------------------------------ tiny / random

def tiny_random(rng: np.random.Generator, shape: str = "tree", max_tables: int = 6,
                max_rows: int = 40, domain: int = 8, pred_prob: float = 0.5,
                allow_empty: bool = True, outer: float = 0.0) -> Problem:
    """A small random join problem for brute-force checks.

    shape: "chain", "star", "tree" (random tree), "cycle" (a tree plus one
    extra edge closing a cycle), "parallel" (a tree plus one edge that
    duplicates a pair on other columns), "forest" (two components and
    possibly an isolated table). outer > 0 makes each edge an outer join
    (left, right or full, uniformly) with that probability.
    """
    n_t = int(rng.integers(2, max_tables + 1))
    if shape == "cycle":
        n_t = max(n_t, 3)
    pairs: list[tuple[int, int]] = []
    if shape == "chain":
        pairs = [(i, i + 1) for i in range(n_t - 1)]
    elif shape == "star":
        pairs = [(0, i) for i in range(1, n_t)]
    elif shape in ("tree", "cycle", "parallel"):
        pairs = [(int(rng.integers(0, i)), i) for i in range(1, n_t)]
        if shape == "cycle":
            # close a cycle: join two tables that are not adjacent in the tree
            cands = [(a, b) for a in range(n_t) for b in range(a + 1, n_t)
                     if (a, b) not in pairs and (b, a) not in pairs]
            a, b = cands[int(rng.integers(0, len(cands)))]
            pairs.append((a, b))
        if shape == "parallel":
            a, b = pairs[int(rng.integers(0, len(pairs)))]
            pairs.append((a, b))
    elif shape == "forest":
        n_t = max(n_t, 4)
        cut = int(rng.integers(2, n_t))
        pairs = [(int(rng.integers(0, i)), i) for i in range(1, cut)]
        pairs += [(int(rng.integers(cut, i)), i) for i in range(cut + 1, n_t)]
    else:
        raise ValueError(shape)
    lo_rows = 0 if allow_empty else 1
    rows = [int(rng.integers(lo_rows, max_rows + 1)) for _ in range(n_t)]
    columns: list[dict[str, np.ndarray]] = [dict() for _ in range(n_t)]
    edges = []
    for j, (a, b) in enumerate(pairs):
        ca, cb = f"j{j}", f"j{j}"
        # one edge in six carries keys with a non-zero high word (both sides
        # int64); otherwise each side is int32 or int64 on its own, so an
        # edge may join an int32 column with an int64 column
        wide = rng.random() < 1 / 6
        for t, c in ((a, ca), (b, cb)):
            vals = rng.integers(-domain // 2, domain - domain // 2, size=rows[t]).astype(np.int64)
            if wide:
                columns[t][c] = vals * (1 << 33) + 5
            else:
                columns[t][c] = vals.astype(np.int64 if rng.random() < 0.3 else np.int32)
        if rng.random() < 0.5:
            edges.append((a, ca, b, cb))
        else:
            edges.append((b, cb, a, ca))
    preds = []
    for t in range(n_t):
        columns[t]["x"] = rng.integers(0, 100, size=rows[t]).astype(np.int32)
        if rng.random() < pred_prob:
            op = OPS[int(rng.integers(0, len(OPS)))]
            lo = int(rng.integers(0, 100))
            hi = int(rng.integers(lo, 101))
            preds.append((t, "x", op, lo, hi))
    flags = None
    if outer > 0:
        # each edge an outer join with probability `outer`: left, right or full
        flags = [int(rng.integers(1, 4)) if rng.random() < outer else 0 for _ in edges]
    return Problem([f"T{t}" for t in range(n_t)], columns, edges, preds, label=f"tiny-{shape}", edge_flags=flags)


_ZIPF_CHUNK = 1 << 22


def _zipf_chunk(seed_seq: np.random.SeedSequence, n: int, s: float, size: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed_seq))

    def h(x):
        return np.power(x, -s)

    def H(x):
        return (np.power(x, 1.0 - s) - 1.0) / (1.0 - s)

    def H_inv(y):
        return np.power(1.0 + y * (1.0 - s), 1.0 / (1.0 - s))

    h_x1 = H(1.5) - 1.0
    h_n = H(n + 0.5)
    s_const = 2.0 - H_inv(H(2.5) - h(2.0))
    out = np.empty(size, np.int64)
    filled = 0
    while filled < size:
        m = int((size - filled) * 1.05) + 1024
        u = h_n + rng.random(m) * (h_x1 - h_n)
        x = H_inv(u)
        kk = np.clip(np.floor(x + 0.5), 1, n)
        acc = (kk - x <= s_const) | (u >= H(kk + 0.5) - h(kk))
        good = kk[acc].astype(np.int64) - 1
        take = min(len(good), size - filled)
        out[filled:filled + take] = good[:take]
        filled += take
    return out


def zipf_ranks(rng: np.random.Generator, n: int, s: float, size: int) -> np.ndarray:
    """Zipf(s) ranks in [0, n): rank r is drawn with probability proportional
    to (r+1)^-s. Rejection-inversion sampling (Hormann and Derflinger 1996)
    with the hat function h(x) = x^-s over [0.5, n + 0.5]. Fixed chunks of
    2^22 draws, each from its own seeded stream, run on a thread pool, so the
    result depends on `rng` alone and not on the number of threads."""
    if abs(s - 1.0) < 1e-12 or s <= 0:
        raise ValueError("need s > 0, s != 1")
    n_chunks = (size + _ZIPF_CHUNK - 1) // _ZIPF_CHUNK
    seqs = np.random.SeedSequence(int(rng.integers(0, 2**63 - 1))).spawn(max(1, n_chunks))
    sizes = [min(_ZIPF_CHUNK, size - i * _ZIPF_CHUNK) for i in range(n_chunks)]
    if n_chunks <= 1:
        return _zipf_chunk(seqs[0], n, s, size)
    import concurrent.futures as cf
    workers = min(16, os.cpu_count() or 1, n_chunks)
    with cf.ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda i: _zipf_chunk(seqs[i], n, s, sizes[i]), range(n_chunks)))
    return np.concatenate(parts)


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


# ------------------------------------------------------------------- batches

def batch(seed: int = 1, n_problems: int = 256, lo: int = 10_000, hi: int = 5_000_000) -> list[Problem]:
    """Independent transfer problems of uneven sizes: alternately a chain
    R - S - T (key domain twice the smaller end table, R keeps U[1 %, 50 %])
    and a star with 2 to 4 dimensions (two of them with a predicate keeping
    U[1 %, 50 %]). Every table has a row count log-uniform on [lo, hi];
    keys are int32 uniform."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    out = []
    for i in range(n_problems):
        sub = int(rng.integers(1, 1 << 31))
        if i % 2 == 0:
            n_r, n_s, n_t = (log_uniform_int(rng, lo, hi) for _ in range(3))
            keep = float(rng.uniform(0.01, 0.50))
            out.append(chain(sub, n_r, n_s, n_t, domain=2 * min(n_r, n_t), keep=keep))
        else:
            nd = int(rng.integers(2, 5))
            n_fact = log_uniform_int(rng, lo, hi)
            dims = tuple(log_uniform_int(rng, lo, hi) for _ in range(nd))
            keeps = (float(rng.uniform(0.01, 0.50)), float(rng.uniform(0.01, 0.50))) + (None,) * (nd - 2)
            out.append(star(sub, n_fact, dims, keeps, payload=0))
    return out
