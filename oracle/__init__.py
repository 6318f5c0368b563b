"""CPU oracle for the predicate-transfer phase (ctypes wrapper of pt_oracle.c).

TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. Nothing in the GPU product path imports
this package, and this package imports nothing from the GPU product path: the
only module both sides share is the seeded input generator
(`paper_2307_15255_amd.workloads`), which holds none of the method's
arithmetic.

Every routine follows Yang, Zhao, Yu, Koutris, "Predicate Transfer", CIDR
2024, Sec. 3.2 (filter transformation, predicate transfer graph, transfer
schedule, filter type); the filter specification is restated in
`pt_oracle.h`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpt_oracle.so")

BLOOM = 0
EXACT = 1

OPS = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5, "between": 6}


class _Column(C.Structure):
    _fields_ = [("data", C.c_void_p), ("is64", C.c_uint32), ("pad", C.c_uint32)]


class _Table(C.Structure):
    _fields_ = [("n_rows", C.c_uint64), ("n_cols", C.c_uint32), ("pad", C.c_uint32),
                ("cols", C.POINTER(_Column))]


class _Edge(C.Structure):
    _fields_ = [("u", C.c_uint32), ("u_col", C.c_uint32), ("v", C.c_uint32), ("v_col", C.c_uint32),
                ("flags", C.c_uint32)]


class _Pred(C.Structure):
    _fields_ = [("table", C.c_uint32), ("col", C.c_uint32), ("op", C.c_uint32), ("pad", C.c_uint32),
                ("lo", C.c_int64), ("hi", C.c_int64)]


class _Problem(C.Structure):
    _fields_ = [("n_tables", C.c_uint32), ("n_edges", C.c_uint32),
                ("tables", C.POINTER(_Table)), ("edges", C.POINTER(_Edge)),
                ("orient", C.POINTER(C.c_int8)), ("preds", C.POINTER(_Pred)),
                ("n_preds", C.c_uint32), ("pad", C.c_uint32)]


class _Params(C.Structure):
    _fields_ = [("block_bits", C.c_uint32), ("k", C.c_uint32), ("bits_per_key", C.c_uint32),
                ("kind", C.c_uint32), ("n_passes", C.c_uint32), ("variant", C.c_uint32),
                ("threads", C.c_uint32), ("prune", C.c_uint32)]


class _Dump(C.Structure):
    _fields_ = [("filter_words", C.POINTER(C.POINTER(C.c_uint32))),
                ("filter_cap", C.POINTER(C.c_uint64)),
                ("filter_nb", C.POINTER(C.c_uint64)),
                ("fwd_bitmaps", C.POINTER(C.POINTER(C.c_uint64))),
                ("fwd_counts", C.POINTER(C.c_uint64)),
                ("edge_src", C.POINTER(C.c_uint32))]


_SAN_PATH = os.path.join(_HERE, "libpt_oracle_san.so")


def build_sanitized() -> str:
    """The oracle under AddressSanitizer and UBSan (any finding aborts), for
    the CPU test that runs the pins against it under gcc's runtime."""
    tmp = _SAN_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", tmp, _SRC])
    os.replace(tmp, _SAN_PATH)
    return _SAN_PATH


def build(force: bool = True) -> str:
    """Compile pt_oracle.c with gcc into oracle/libpt_oracle.so (plain -O2,
    no SIMD intrinsics; OpenMP only for the optional row split of the
    transfer's scans, off unless threads > 1 is asked for)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-fopenmp",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def build_variant(source_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (used by the tests that
    plant mistakes in the oracle to show that the pins catch them)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-I", _HERE,
                           "-o", out_path, src])
    return out_path


def use_library(path: str) -> None:
    """Load the oracle from another shared object (a planted-mistake build)."""
    global _lib
    _lib = None
    lib(path)


def lib(path: str | None = None) -> C.CDLL:
    global _lib
    if _lib is None:
        if path is None:
            path = _LIB_PATH
            if not os.path.exists(path):
                build()
        L = C.CDLL(path)
        u32p, u64p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
        L.ptor_hash.argtypes = [C.c_int64, u32p, u32p]
        L.ptor_filter_blocks.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.ptor_filter_blocks.restype = C.c_uint64
        L.ptor_key_slots.argtypes = [C.c_int64, C.c_uint64, C.c_uint32, C.c_uint32, u64p, u32p]
        L.ptor_bloom_insert.argtypes = [u32p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64]
        L.ptor_bloom_contains.argtypes = [u32p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64]
        L.ptor_local_filter.argtypes = [C.POINTER(_Table), C.POINTER(_Pred), C.c_uint32, u64p, u64p]
        L.ptor_bloom_build.argtypes = [C.POINTER(_Column), C.c_uint64, u64p, C.c_uint32, C.c_uint32,
                                       C.c_uint32, u32p, C.c_uint64, u64p]
        L.ptor_bloom_probe.argtypes = [C.POINTER(_Column), C.c_uint64, u32p, C.c_uint64, C.c_uint32,
                                       C.c_uint32, u64p, u64p]
        L.ptor_compact.argtypes = [u64p, C.c_uint64, u32p, u64p]
        L.ptor_transfer.argtypes = [C.POINTER(_Problem), C.POINTER(_Params),
                                    C.POINTER(C.POINTER(C.c_uint64)), u64p, C.POINTER(_Dump)]
        L.ptor_join.argtypes = [C.POINTER(_Problem), C.c_uint32, C.POINTER(u64p), u32p, u32p, u32p,
                                C.c_uint64, u64p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _column(a: np.ndarray) -> _Column:
    if a.dtype not in (np.int32, np.int64) or not a.flags.c_contiguous:
        raise ValueError("columns must be contiguous int32 or int64 arrays")
    return _Column(a.ctypes.data, 1 if a.dtype == np.int64 else 0, 0)


def bitmap_words(n_rows: int) -> int:
    return (n_rows + 63) // 64


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


# ---------------------------------------------------------------- primitives

def hash_key(key: int) -> tuple[int, int]:
    h1, h2 = C.c_uint32(), C.c_uint32()
    lib().ptor_hash(int(key), C.byref(h1), C.byref(h2))
    return h1.value, h2.value


def filter_blocks(n_keys: int, bits_per_key: int, block_bits: int) -> int:
    return int(lib().ptor_filter_blocks(n_keys, bits_per_key, block_bits))


def key_slots(key: int, nb: int, block_bits: int, k: int) -> tuple[int, list[int]]:
    blk = C.c_uint64()
    pos = (C.c_uint32 * 16)()
    lib().ptor_key_slots(int(key), nb, block_bits, k, C.byref(blk), pos)
    return blk.value, [pos[i] for i in range(k)]


def local_filter(cols: list[np.ndarray], preds: list[tuple]) -> tuple[np.ndarray, int]:
    """preds: (col_index, op, lo, hi). Returns (bitmap, count)."""
    n = len(cols[0]) if cols else 0
    ccols = (_Column * max(1, len(cols)))(*[_column(c) for c in cols])
    t = _Table(n, len(cols), 0, ccols)
    cp = (_Pred * max(1, len(preds)))(*[_Pred(0, c, OPS[op], 0, lo, hi) for c, op, lo, hi in preds])
    bm = np.zeros(max(1, bitmap_words(n)), np.uint64)
    cnt = C.c_uint64()
    _check(lib().ptor_local_filter(C.byref(t), cp, len(preds), _ptr(bm, C.c_uint64), C.byref(cnt)),
           "local_filter")
    return bm[:bitmap_words(n)], cnt.value


def bloom_build(keys: np.ndarray, bitmap: np.ndarray | None, block_bits: int, k: int,
                bits_per_key: int) -> tuple[np.ndarray, int]:
    n = len(keys)
    cap_keys = n if bitmap is None else int(n)
    cap = filter_blocks(cap_keys, bits_per_key, block_bits) * (block_bits // 32)
    words = np.zeros(cap, np.uint32)
    nb = C.c_uint64()
    col = _column(keys)
    bm = None if bitmap is None else _ptr(np.ascontiguousarray(bitmap, np.uint64), C.c_uint64)
    _check(lib().ptor_bloom_build(C.byref(col), n, bm, block_bits, k, bits_per_key,
                                  _ptr(words, C.c_uint32), cap, C.byref(nb)), "bloom_build")
    return words[:nb.value * (block_bits // 32)].copy(), nb.value


def bloom_probe(keys: np.ndarray, words: np.ndarray, nb: int, block_bits: int, k: int,
                bitmap: np.ndarray | None = None) -> tuple[np.ndarray, int]:
    n = len(keys)
    if bitmap is None:
        bitmap = all_rows_bitmap(n)
    bm = np.array(bitmap, np.uint64, copy=True)
    words = np.ascontiguousarray(words, np.uint32)
    cnt = C.c_uint64()
    col = _column(keys)
    _check(lib().ptor_bloom_probe(C.byref(col), n, _ptr(words, C.c_uint32), nb, block_bits, k,
                                  _ptr(bm, C.c_uint64), C.byref(cnt)), "bloom_probe")
    return bm, cnt.value


def bloom_contains(words: np.ndarray, nb: int, block_bits: int, k: int, key: int) -> bool:
    words = np.ascontiguousarray(words, np.uint32)
    return bool(lib().ptor_bloom_contains(_ptr(words, C.c_uint32), nb, block_bits, k, int(key)))


def compact(bitmap: np.ndarray, n_rows: int) -> np.ndarray:
    idx = np.zeros(max(1, n_rows), np.uint32)
    cnt = C.c_uint64()
    bm = np.ascontiguousarray(bitmap, np.uint64)
    if bm.size == 0:
        bm = np.zeros(1, np.uint64)
    _check(lib().ptor_compact(_ptr(bm, C.c_uint64), n_rows, _ptr(idx, C.c_uint32), C.byref(cnt)),
           "compact")
    return idx[:cnt.value].copy()


def all_rows_bitmap(n: int) -> np.ndarray:
    bm = np.full(bitmap_words(n), np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64)
    if n % 64:
        bm[-1] = np.uint64((1 << (n % 64)) - 1)
    return bm


# ---------------------------------------------------------------- transfer

class TransferResult:
    """Per-table bitmaps and counts, plus the filters of every (pass, edge)."""

    def __init__(self):
        self.bitmaps: list[np.ndarray] = []
        self.counts: list[int] = []
        self.fwd_bitmaps: list[np.ndarray] = []
        self.fwd_counts: list[int] = []
        self.filters: dict[tuple[int, int], np.ndarray] = {}
        self.filter_nb: dict[tuple[int, int], int] = {}
        self.edge_src: dict[tuple[int, int], int] = {}


def _problem(problem, keep: list) -> _Problem:
    """The C view of a `workloads.Problem` (arrays kept alive in `keep`)."""
    n_t, n_e = problem.n_tables, len(problem.edges)
    tables = (_Table * max(1, n_t))()
    for t in range(n_t):
        cols = [np.ascontiguousarray(a) for a in problem.columns[t].values()]
        keep.append(cols)
        cc = (_Column * max(1, len(cols)))(*[_column(a) for a in cols])
        keep.append(cc)
        tables[t] = _Table(problem.n_rows(t), len(cols), 0, cc)
    flags = problem.edge_flags if problem.edge_flags is not None else [0] * n_e
    edges = (_Edge * max(1, n_e))(*[
        _Edge(u, problem.col_index(u, uc), v, problem.col_index(v, vc), f)
        for (u, uc, v, vc), f in zip(problem.edges, flags)])
    preds = (_Pred * max(1, len(problem.preds)))(*[
        _Pred(t, problem.col_index(t, c), OPS[op], 0, lo, hi) for t, c, op, lo, hi in problem.preds])
    orient = None
    if problem.orient is not None:
        orient_arr = np.array(problem.orient, np.int8)
        keep.append(orient_arr)
        orient = _ptr(orient_arr, C.c_int8)
    keep += [tables, edges, preds]
    return _Problem(n_t, n_e, tables, edges, orient, preds, len(problem.preds), 0)


def transfer(problem, block_bits: int = 512, k: int = 3, bits_per_key: int = 10,
             kind: int = BLOOM, n_passes: int = 2, variant: int = 0,
             dump_filters: bool = False, threads: int = 1, prune: bool = False) -> TransferResult:
    """Run the transfer phase on a `workloads.Problem` (threads > 1: the row
    scans split over that many threads, with the same results; prune: a
    table that still holds every row sends no filter, Sec. 3.2 "Transfer
    Path Pruning")."""
    L = lib()
    n_t, n_e = problem.n_tables, len(problem.edges)
    keep: list = []
    prob = _problem(problem, keep)
    par = _Params(block_bits, k, bits_per_key, kind, n_passes, variant, threads, int(prune))

    res = TransferResult()
    res.bitmaps = [np.zeros(max(1, bitmap_words(problem.n_rows(t))), np.uint64) for t in range(n_t)]
    bm_ptrs = (C.POINTER(C.c_uint64) * max(1, n_t))(*[_ptr(b, C.c_uint64) for b in res.bitmaps])
    counts = np.zeros(max(1, n_t), np.uint64)

    fwd = [np.zeros(max(1, bitmap_words(problem.n_rows(t))), np.uint64) for t in range(n_t)]
    fwd_ptrs = (C.POINTER(C.c_uint64) * max(1, n_t))(*[_ptr(b, C.c_uint64) for b in fwd])
    fwd_counts = np.zeros(max(1, n_t), np.uint64)
    n_slots = max(1, 2 * n_e)
    nb = np.zeros(n_slots, np.uint64)
    src = np.full(n_slots, 0xFFFFFFFF, np.uint32)
    words = []
    caps = np.zeros(n_slots, np.uint64)
    wptrs = (C.POINTER(C.c_uint32) * n_slots)()
    if dump_filters and kind == BLOOM:
        for p in range(2):
            for e, (u, _, v, _) in enumerate(problem.edges):
                cap_rows = max(problem.n_rows(u), problem.n_rows(v))
                cap = filter_blocks(cap_rows, bits_per_key, block_bits) * (block_bits // 32)
                w = np.zeros(cap, np.uint32)
                words.append(w)
                caps[p * n_e + e] = cap
                wptrs[p * n_e + e] = _ptr(w, C.c_uint32)
    dump = _Dump(wptrs if words else None, _ptr(caps, C.c_uint64), _ptr(nb, C.c_uint64),
                 fwd_ptrs, _ptr(fwd_counts, C.c_uint64), _ptr(src, C.c_uint32))
    _check(L.ptor_transfer(C.byref(prob), C.byref(par), bm_ptrs, _ptr(counts, C.c_uint64),
                           C.byref(dump)), "transfer")
    for t in range(n_t):
        nw = bitmap_words(problem.n_rows(t))
        res.bitmaps[t] = res.bitmaps[t][:nw]
        res.fwd_bitmaps.append(fwd[t][:nw])
    res.counts = [int(c) for c in counts[:n_t]]
    res.fwd_counts = [int(c) for c in fwd_counts[:n_t]]
    for p in range(n_passes):
        for e in range(n_e):
            s = p * n_e + e
            res.filter_nb[(p, e)] = int(nb[s])
            res.edge_src[(p, e)] = int(src[s])
            if words:
                res.filters[(p, e)] = words[s][:int(nb[s]) * (block_bits // 32)].copy()
    return res


def join(problem, bitmaps: list | None = None, root: int = 0) -> tuple[list[int], np.ndarray]:
    """Join phase (Sec. 3.3) on the tables reduced to `bitmaps` (None: every
    row; a None entry: every row of that table): the tables of root's
    connected component in ascending order, and every tuple of their row ids
    that satisfies all the component's edges, one tuple per row, sorted."""
    L = lib()
    keep: list = []
    prob = _problem(problem, keep)
    n_t = problem.n_tables
    bm = (C.POINTER(C.c_uint64) * max(1, n_t))()
    if bitmaps is not None:
        for t, b in enumerate(bitmaps):
            if b is not None:
                b = np.ascontiguousarray(b, dtype=np.uint64)
                keep.append(b)
                bm[t] = _ptr(b, C.c_uint64)
    comp = np.zeros(max(1, n_t), np.uint32)
    n_comp, n_out = C.c_uint32(), C.c_uint64()
    cap = 1 << 12
    while True:
        out = np.zeros(cap * max(1, n_t), np.uint32)
        _check(L.ptor_join(C.byref(prob), root, bm, _ptr(comp, C.c_uint32), C.byref(n_comp),
                           _ptr(out, C.c_uint32), cap, C.byref(n_out)), "join")
        if n_out.value <= cap:
            break
        cap = n_out.value
    w = n_comp.value
    return [int(t) for t in comp[:w]], out[:n_out.value * w].reshape(n_out.value, w).copy()
