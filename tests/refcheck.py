"""Independent checkers that pin the oracle to what the paper and the
mathematics fix. Nothing here calls the oracle or the GPU library.

* brute-force join and participating rows (the exact result a pre-filter may
  never cut into: Sec. 3.1, a transferred filter only removes rows that join
  with nothing);
* the Yannakakis full reducer on acyclic join graphs (Sec. 2.2);
* the closed-form false-positive rate of a blocked Bloom filter (Putze,
  Sanders, Singler 2007) and the exact per-filter prediction given a
  filter's bits;
* the filter specification's hash, retyped with Python integers.
"""
from __future__ import annotations

import math
from collections import defaultdict, deque

import numpy as np
import pandas as pd

MASK64 = (1 << 64) - 1
MULT = 0x9E3779B97F4A7C15


# ------------------------------------------------------------------ bitmaps

def bits_to_rows(bitmap: np.ndarray, n_rows: int) -> set[int]:
    rows = set()
    for r in range(n_rows):
        if (int(bitmap[r // 64]) >> (r % 64)) & 1:
            rows.add(r)
    return rows


def rows_to_bits(rows, n_rows: int) -> np.ndarray:
    bm = np.zeros((n_rows + 63) // 64, np.uint64)
    for r in rows:
        bm[r // 64] |= np.uint64(1 << (r % 64))
    return bm


def bitmap_to_bool(bitmap: np.ndarray, n_rows: int) -> np.ndarray:
    b = np.unpackbits(np.ascontiguousarray(bitmap).view(np.uint8), bitorder="little")
    return b[:n_rows].astype(bool)


# -------------------------------------------------------------- predicates

def local_rows(problem, t: int) -> np.ndarray:
    """Boolean mask of the rows of table t that satisfy its predicates."""
    n = problem.n_rows(t)
    keep = np.ones(n, bool)
    for tt, c, op, lo, hi in problem.preds:
        if tt != t:
            continue
        v = problem.columns[t][c].astype(np.int64)
        keep &= {"lt": v < lo, "le": v <= lo, "gt": v > lo, "ge": v >= lo, "eq": v == lo,
                 "ne": v != lo, "between": (v >= lo) & (v <= hi)}[op]
    return keep


# ---------------------------------------------------------- brute-force join

def _components(problem) -> list[list[int]]:
    adj = defaultdict(set)
    for u, _, v, _ in problem.edges:
        adj[u].add(v)
        adj[v].add(u)
    seen, comps = set(), []
    for s in range(problem.n_tables):
        if s in seen:
            continue
        comp, q = [], deque([s])
        seen.add(s)
        while q:
            x = q.popleft()
            comp.append(x)
            for y in sorted(adj[x]):
                if y not in seen:
                    seen.add(y)
                    q.append(y)
        comps.append(comp)
    return comps


def join_tuples(problem, masks: list[np.ndarray] | None = None) -> list[pd.DataFrame]:
    """Per connected component, every combination of row ids (one column
    ``r<t>`` per table) that satisfies all join edges of the component.
    `masks` restricts each table to some rows (default: its local
    predicates)."""
    if masks is None:
        masks = [local_rows(problem, t) for t in range(problem.n_tables)]
    out = []
    for comp in _components(problem):
        placed: list[int] = []
        df = None
        for t in comp:
            rows = np.nonzero(masks[t])[0]
            tdf = pd.DataFrame({f"r{t}": rows})
            for name, col in problem.columns[t].items():
                tdf[f"t{t}.{name}"] = col.astype(np.int64)[rows]
            if df is None:
                df = tdf
            else:
                lk, rk = [], []
                for u, uc, v, vc in problem.edges:
                    if u == t and v in placed:
                        lk.append(f"t{v}.{vc}")
                        rk.append(f"t{u}.{uc}")
                    elif v == t and u in placed:
                        lk.append(f"t{u}.{uc}")
                        rk.append(f"t{v}.{vc}")
                if lk:
                    df = df.merge(tdf, left_on=lk, right_on=rk, how="inner")
                else:
                    df = df.merge(tdf, how="cross")
            placed.append(t)
        out.append(df[[f"r{t}" for t in comp]])
    return out


def participating_rows(problem) -> list[set[int]]:
    """Rows of each table that appear in at least one tuple of the full
    join (after local predicates). If any component joins to nothing, the
    whole (cross-product) join is empty and no row participates."""
    comps = join_tuples(problem)
    rows: list[set[int]] = [set() for _ in range(problem.n_tables)]
    if any(len(df) == 0 for df in comps):
        return rows
    for df in comps:
        for c in df.columns:
            rows[int(c[1:])] = set(df[c].tolist())
    return rows


def join_size(problem, masks: list[np.ndarray] | None = None) -> int:
    size = 1
    for df in join_tuples(problem, masks):
        size *= len(df)
    return size


def join_multiset(problem, masks: list[np.ndarray] | None = None):
    """The join result as a sorted list of row-id tuples (all components)."""
    comps = join_tuples(problem, masks)
    if any(len(df) == 0 for df in comps):
        return []
    full = comps[0]
    for df in comps[1:]:
        full = full.merge(df, how="cross")
    cols = sorted(full.columns, key=lambda c: int(c[1:]))
    return sorted(map(tuple, full[cols].itertuples(index=False, name=None)))


# ----------------------------------------------------- Yannakakis reducer

def is_forest(problem) -> bool:
    parent = list(range(problem.n_tables))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, _, v, _ in problem.edges:
        a, b = find(u), find(v)
        if a == b:
            return False
        parent[a] = b
    return True


def yannakakis_full_reduction(problem, root: int = 0) -> list[set[int]]:
    """Semi-join phase of Yannakakis (Sec. 2.2) on each tree of a forest join
    graph: bottom-up semi-joins of every parent with its children, then
    top-down semi-joins of every child with its parent. Exact key sets."""
    assert is_forest(problem)
    n = problem.n_tables
    masks = [local_rows(problem, t) for t in range(n)]
    adj = defaultdict(list)
    for u, uc, v, vc in problem.edges:
        adj[u].append((v, uc, vc))
        adj[v].append((u, vc, uc))

    def keys(t, col):
        return problem.columns[t][col].astype(np.int64)

    def semijoin(t, tcol, s, scol):
        allowed = set(keys(s, scol)[masks[s]].tolist())
        masks[t] &= np.isin(keys(t, tcol), list(allowed))

    seen = set()
    roots = [root] + [t for t in range(n) if t != root]
    for r in roots:
        if r in seen:
            continue
        order, parent_of = [], {r: None}
        q = deque([r])
        seen.add(r)
        while q:
            x = q.popleft()
            order.append(x)
            for y, xc, yc in adj[x]:
                if y not in seen:
                    seen.add(y)
                    parent_of[y] = (x, yc, xc)
                    q.append(y)
        for x in reversed(order):           # bottom-up
            if parent_of[x] is not None:
                p, xc, pc = parent_of[x]
                semijoin(p, pc, x, xc)
        for x in order:                     # top-down
            if parent_of[x] is not None:
                p, xc, pc = parent_of[x]
                semijoin(x, xc, p, pc)
    rows = [set(np.nonzero(m)[0].tolist()) for m in masks]
    if any(len(r) == 0 for r in rows):
        # a component reduced to nothing empties the cross-product join
        pass
    return rows


def in_tree_orientation(problem, root: int) -> list[int]:
    """Orientation override that points every edge of a forest towards the
    root of its tree (child -> parent): one sink per tree, out-degree <= 1."""
    adj = defaultdict(list)
    for e, (u, _, v, _) in enumerate(problem.edges):
        adj[u].append((v, e))
        adj[v].append((u, e))
    orient = [0] * len(problem.edges)
    seen = set()
    for r in [root] + list(range(problem.n_tables)):
        if r in seen:
            continue
        seen.add(r)
        q = deque([r])
        while q:
            x = q.popleft()
            for y, e in adj[x]:
                if y in seen:
                    continue
                seen.add(y)
                u = problem.edges[e][0]
                orient[e] = +1 if u == y else -1   # y (child) -> x (parent)
                q.append(y)
    return orient


# ------------------------------------------------------------ filter maths

def blocked_fpr(block_bits: int, bits_per_key: int, k: int, terms: int = 400) -> float:
    """Putze, Sanders, Singler (2007): a blocked Bloom filter's false-positive
    rate is the plain Bloom rate inside one block, averaged over the Poisson
    number of keys per block (mean B / bits_per_key)."""
    lam = block_bits / bits_per_key
    total, logp = 0.0, -lam
    for i in range(terms):
        if i > 0:
            logp += math.log(lam) - math.log(i)
        inner = (1.0 - (1.0 - 1.0 / block_bits) ** (k * i)) ** k
        total += math.exp(logp) * inner
    return total


def blocked_fpr_distinct(block_bits: int, bits_per_key: int, k: int, terms: int = 400) -> float:
    """The same average when every key sets k distinct bits of its block (as
    double hashing with an odd stride does): after i keys a bit is set with
    probability 1 - (1 - k/B)^i."""
    lam = block_bits / bits_per_key
    total, logp = 0.0, -lam
    for i in range(terms):
        if i > 0:
            logp += math.log(lam) - math.log(i)
        total += math.exp(logp) * (1.0 - (1.0 - k / block_bits) ** i) ** k
    return total


def classic_fpr(bits_per_key: int, k: int) -> float:
    return (1.0 - math.exp(-k / bits_per_key)) ** k


def per_filter_fpr(words: np.ndarray, nb: int, block_bits: int, k: int) -> float:
    """Probability that a key outside the filter passes, given the filter's
    bits, when its block and its double-hashing pair (g1, g2 odd) are uniform:
    the average over blocks and over all (g1, g2) of 'all k bits set'."""
    w = np.ascontiguousarray(words, np.uint32).reshape(nb, block_bits // 32)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little").reshape(nb, block_bits).astype(bool)
    g1 = np.arange(block_bits)[:, None, None]
    g2 = (2 * np.arange(block_bits // 2) + 1)[None, :, None]
    i = np.arange(k)[None, None, :]
    pos = (g1 + i * g2) % block_bits
    total = 0.0
    for b in range(nb):
        total += bits[b][pos].all(axis=2).mean()
    return total / nb


# ------------------------------------------------------ spec hash, retyped

def spec_hash(key: int) -> tuple[int, int]:
    x = key & MASK64
    p = (x * MULT) & MASK64
    hi, lo = p >> 32, p & 0xFFFFFFFF
    t = lo ^ hi
    t ^= t >> 16
    return hi, (t * 0x85EBCA6B) & 0xFFFFFFFF


def spec_slots(key: int, nb: int, block_bits: int, k: int) -> tuple[int, list[int]]:
    h1, h2 = spec_hash(key)
    b = block_bits.bit_length() - 1
    blk = (h1 * nb) >> 32
    g1 = h2 >> (32 - b)
    g2 = ((h2 >> (32 - 2 * b)) & (block_bits - 1)) | 1
    return blk, [(g1 + i * g2) % block_bits for i in range(k)]


# ------------------------------------------------------- outer-join trees

_HOW = {0: "inner", 3: "outer"}


def outer_tree_result(problem, masks: list[np.ndarray], root: int) -> list[tuple]:
    """The query of a join tree with inner and outer edges (Sec. 3.4),
    evaluated bottom-up from `root`: each table joins the result of every
    child subtree with its edge's join type (u LEFT JOIN v keeps every row of
    u, RIGHT every row of v, FULL both). Rows are restricted to `masks`.
    Returns the sorted row-id tuples (one column per table, ascending table
    order; -1 where a row is null-extended). Null join keys never match."""
    adj = defaultdict(list)
    for e, (u, uc, v, vc) in enumerate(problem.edges):
        adj[u].append((e, v))
        adj[v].append((e, u))
    flags = problem.edge_flags or [0] * len(problem.edges)
    sentinel = [-(1 << 52)]  # below every key of the tests, exact in float64

    def frame(t):
        rows = np.nonzero(masks[t])[0]
        df = pd.DataFrame({f"r{t}": rows.astype(np.float64)})
        for name, col in problem.columns[t].items():
            df[f"t{t}.{name}"] = col.astype(np.int64)[rows].astype(np.float64)
        return df

    def fill_null_keys(df, col):
        # a null key must match nothing: give each null its own value
        df = df.copy()
        miss = df[col].isna().to_numpy()
        n = int(miss.sum())
        df.loc[miss, col] = np.arange(sentinel[0], sentinel[0] + n, dtype=np.float64)
        sentinel[0] += n
        return df

    def build(t, parent_edge):
        df = frame(t)
        for e, c in adj[t]:
            if e == parent_edge:
                continue
            sub = build(c, e)
            u, uc, v, vc = problem.edges[e]
            mine, theirs = (uc, vc) if u == t else (vc, uc)
            f = flags[e]
            if f in (1, 2):  # the preserved side: u for LEFT, v for RIGHT
                preserved = u if f == 1 else v
                how = "left" if preserved == t else "right"
            else:
                how = _HOW[f]
            lk, rk = f"t{t}.{mine}", f"t{c}.{theirs}"
            df = fill_null_keys(df, lk)
            sub = fill_null_keys(sub, rk)
            df = df.merge(sub, left_on=lk, right_on=rk, how=how)
        return df

    df = build(root, -1)
    cols = sorted([c for c in df.columns if c.startswith("r")], key=lambda c: int(c[1:]))
    out = df[cols].fillna(-1).astype(np.int64)
    return sorted(map(tuple, out.itertuples(index=False, name=None)))
