"""Python binding of libpt_hip.so (include/pt.h).

Argument marshalling only: every step of the transfer phase runs in the HIP
kernels behind the C ABI. torch provides device memory (tensors) and streams.
The functions keep the C names; the classes at the end assemble the arguments
of a whole join problem.

Importing this module loads the library, building it first when it is
missing or was built from other sources (``build.ensure_built``); a build or
load failure raises. There is no fallback: every call runs on the GPU.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpt_hip.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_EUNSUPPORTED, PT_EOVERFLOW = 0, 1, 2, 3, 4, 5
PT_STATUS_FILTER_OVERFLOW, PT_STATUS_ENTRIES_OVERFLOW, PT_STATUS_WAIT_TIMEOUT, PT_STATUS_JOIN_OVERFLOW = 1, 2, 4, 8
PT_PROBE_SELECTIVE, PT_PROBE_GIVEN = 0, 1
PT_I32, PT_I64 = 0, 1
OPS = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "eq": 4, "ne": 5, "between": 6}


class PtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pt status {status}: {msg}")
        self.status = status


class pt_column(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_uint32), ("reserved", C.c_uint32)]


class pt_table(C.Structure):
    _fields_ = [("n_rows", C.c_uint64), ("n_cols", C.c_uint32), ("reserved", C.c_uint32),
                ("cols", C.POINTER(pt_column))]


class pt_edge(C.Structure):
    _fields_ = [("u", C.c_uint32), ("u_col", C.c_uint32), ("v", C.c_uint32), ("v_col", C.c_uint32),
                ("flags", C.c_uint32)]


class pt_graph(C.Structure):
    _fields_ = [("n_tables", C.c_uint32), ("n_edges", C.c_uint32), ("edges", C.POINTER(pt_edge)),
                ("orient", C.POINTER(C.c_int8))]


class pt_pred(C.Structure):
    _fields_ = [("table", C.c_uint32), ("col", C.c_uint32), ("op", C.c_uint32),
                ("reserved", C.c_uint32), ("lo", C.c_int64), ("hi", C.c_int64)]


class pt_params(C.Structure):
    _fields_ = [("block_bits", C.c_uint32), ("k", C.c_uint32), ("bits_per_key", C.c_uint32),
                ("flags", C.c_uint32), ("hash_version", C.c_uint32), ("lds_budget", C.c_uint32),
                ("tile_rows", C.c_uint32), ("probe_order", C.c_uint32)]


class pt_bloom(C.Structure):
    _fields_ = [("words", C.c_void_p), ("cap_words", C.c_uint64), ("d_nb", C.c_void_p),
                ("d_status", C.c_void_p), ("params", pt_params)]


class pt_problem(C.Structure):
    _fields_ = [("graph", C.POINTER(pt_graph)), ("tables", C.POINTER(pt_table)), ("preds", C.POINTER(pt_pred)),
                ("n_preds", C.c_uint32), ("reserved", C.c_uint32), ("params", pt_params),
                ("d_bitmaps", C.POINTER(C.c_void_p)), ("d_counts", C.c_void_p)]


class pt_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("table", C.c_uint32), ("pass_", C.c_uint32),
                ("rows", C.c_uint64), ("bytes", C.c_uint64), ("ms", C.c_float),
                ("reserved", C.c_uint32)]


def _load() -> C.CDLL:
    global LIB_PATH
    if os.environ.get("PT_LIB_PATH"):
        # another build of the library (the sanitizer build the CPU tests use)
        LIB_PATH = os.environ["PT_LIB_PATH"]
    else:
        from . import build
        build.ensure_built()
    L = C.CDLL(LIB_PATH)
    vp, u32, u64, st = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    sizep = C.POINTER(C.c_size_t)
    sigs = {
        "pt_version": ([], C.c_char_p),
        "pt_last_error": ([], C.c_char_p),
        "pt_check_status": ([vp, vp], st),
        "pt_local_filter": ([C.POINTER(pt_table), C.POINTER(pt_pred), u32, vp, vp, vp], st),
        "pt_bloom_capacity": ([u64, C.POINTER(pt_params), C.POINTER(u64)], st),
        "pt_bloom_build": ([u32, C.POINTER(pt_column), C.POINTER(pt_bloom), u64, vp, vp, vp], st),
        "pt_bloom_probe": ([u32, C.POINTER(pt_column), C.POINTER(pt_bloom), u64, vp, vp, vp], st),
        "pt_compact_workspace_size": ([u64, sizep], st),
        "pt_compact": ([vp, u64, vp, vp, vp, C.c_size_t, vp], st),
        "pt_compact_noalloc": ([vp, u64, vp, vp, vp], st),
        "pt_transfer_workspace_size": ([C.POINTER(pt_graph), C.POINTER(pt_table),
                                        C.POINTER(pt_params), sizep], st),
        "pt_transfer": ([C.POINTER(pt_graph), C.POINTER(pt_table), C.POINTER(pt_pred), u32,
                         C.POINTER(pt_params), vp, C.c_size_t, C.POINTER(vp), vp, vp], st),
        "pt_transfer_filter": ([C.POINTER(pt_graph), C.POINTER(pt_table), C.POINTER(pt_params), vp,
                                u32, u32, C.POINTER(pt_bloom), C.POINTER(u32)], st),
        "pt_batch_workspace_size": ([u32, C.POINTER(pt_problem), sizep], st),
        "pt_batch_prepare": ([u32, C.POINTER(pt_problem), vp, C.c_size_t, C.POINTER(vp)], st),
        "pt_batch_prepare_async": ([u32, C.POINTER(pt_problem), vp, C.c_size_t, vp, C.POINTER(vp)], st),
        "pt_batch_run": ([vp, vp, u32], st),
        "pt_batch_info": ([vp, C.POINTER(u32), C.POINTER(u64)], st),
        "pt_batch_timeline": ([vp, C.POINTER(u64), u32, C.POINTER(u32), C.POINTER(u32)], st),
        "pt_batch_free": ([vp], None),
        "pt_transfer_batch": ([u32, C.POINTER(pt_problem), vp, C.c_size_t, vp], st),
        "pt_join_workspace_size": ([C.POINTER(pt_graph), C.POINTER(pt_table), u32, u64, sizep], st),
        "pt_join": ([C.POINTER(pt_graph), C.POINTER(pt_table), u32, C.POINTER(vp), C.POINTER(vp), u64, vp, vp,
                     C.c_size_t, vp], st),
        "pt_profile_enable": ([C.c_int], st),
        "pt_profile_only": ([C.c_char_p, u32, u32], st),
        "pt_profile_read": ([C.POINTER(pt_kernel_time), u32, C.POINTER(u32)], st),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib = _load()
EXPORTS = ("pt_version", "pt_last_error", "pt_check_status", "pt_local_filter", "pt_bloom_capacity", "pt_bloom_build",
           "pt_bloom_probe", "pt_compact_workspace_size", "pt_compact", "pt_compact_noalloc", "pt_transfer_workspace_size",
           "pt_transfer", "pt_transfer_filter", "pt_batch_workspace_size", "pt_batch_prepare",
           "pt_batch_prepare_async", "pt_batch_run",
           "pt_batch_info", "pt_batch_timeline", "pt_batch_free", "pt_transfer_batch", "pt_join_workspace_size",
           "pt_join", "pt_profile_enable", "pt_profile_only", "pt_profile_read")
PT_BATCH_EAGER = 1


def lib() -> C.CDLL:
    return _lib


def _check(status: int) -> None:
    if status != PT_OK:
        raise PtError(status, _lib.pt_last_error().decode())


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def column(t: torch.Tensor) -> pt_column:
    if t.dtype not in (torch.int32, torch.int64) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("a column is a contiguous int32 or int64 CUDA tensor")
    return pt_column(t.data_ptr() if t.numel() else 0, PT_I64 if t.dtype == torch.int64 else PT_I32, 0)


PT_FLAG_NO_APPEND = 1
PT_EDGE_INNER, PT_EDGE_LEFT_OUTER, PT_EDGE_RIGHT_OUTER, PT_EDGE_FULL_OUTER = 0, 1, 2, 3
PT_FLAG_SHARED_SCAN = 2
PT_FLAG_EXACT = 4
PT_FLAG_PRUNE = 8


def params(block_bits: int = 512, k: int = 3, bits_per_key: int = 10, flags: int = 0, *, hash_version: int = 1,
           lds_budget: int = 0, tile_rows: int = 0, probe_order: int = PT_PROBE_SELECTIVE) -> pt_params:
    """Filter parameters: the first three fix the filter bits; lds_budget,
    tile_rows and probe_order only change the launch layout."""
    return pt_params(block_bits, k, bits_per_key, flags, hash_version, lds_budget, tile_rows, probe_order)


def pt_check_status(d_status, stream=None) -> None:
    """Waits for the stream, reads and clears a device status word (a
    workspace tensor, a Bloom's status tensor or a raw device address) and
    raises PtError(PT_EOVERFLOW) when a kernel reported an overflow."""
    addr = d_status.data_ptr() if isinstance(d_status, torch.Tensor) else int(d_status)
    _check(_lib.pt_check_status(C.c_void_p(addr), _stream(stream)))


def bitmap_words(n_rows: int) -> int:
    return (n_rows + 63) // 64


def pt_version() -> str:
    return _lib.pt_version().decode()


# ------------------------------------------------------------- primitives

def pt_local_filter(cols: list[torch.Tensor], preds: list[tuple], n_rows: int,
                    bitmap: torch.Tensor, count: torch.Tensor | None = None, stream=None) -> None:
    """preds: (col_index, op, lo, hi); bitmap: int64 tensor of
    ceil(n_rows/64) words (written); count: one int64 (written)."""
    cc = (pt_column * max(1, len(cols)))(*[column(c) for c in cols])
    tb = pt_table(n_rows, len(cols), 0, cc)
    pp = (pt_pred * max(1, len(preds)))(*[pt_pred(0, c, OPS[op], 0, lo, hi) for c, op, lo, hi in preds])
    _check(_lib.pt_local_filter(C.byref(tb), pp, len(preds), _ptr(bitmap), _ptr(count), _stream(stream)))


def pt_bloom_capacity(max_keys: int, p: pt_params) -> int:
    out = C.c_uint64()
    _check(_lib.pt_bloom_capacity(max_keys, C.byref(p), C.byref(out)))
    return out.value


class Bloom:
    """A filter in device memory: `words` (int32 tensor of cap_words) and
    `nb` (one int64: blocks in use)."""

    def __init__(self, max_keys: int, p: pt_params, device="cuda"):
        self.params = p
        self.cap_words = pt_bloom_capacity(max_keys, p)
        self.words = torch.zeros(self.cap_words, dtype=torch.int32, device=device)
        self.nb = torch.zeros(1, dtype=torch.int64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def c(self) -> pt_bloom:
        return pt_bloom(self.words.data_ptr(), self.cap_words, self.nb.data_ptr(), self.status.data_ptr(),
                        self.params)

    def used_words(self) -> np.ndarray:
        nb = int(self.nb.item())
        return self.words[:nb * (self.params.block_bits // 32)].cpu().numpy().view(np.uint32)


def pt_bloom_build(keys: list[torch.Tensor], filters: list[Bloom], n_rows: int,
                   bitmap: torch.Tensor | None = None, count: torch.Tensor | None = None,
                   stream=None) -> None:
    kc = (pt_column * max(1, len(keys)))(*[column(k) for k in keys])
    fc = (pt_bloom * max(1, len(filters)))(*[f.c() for f in filters])
    _check(_lib.pt_bloom_build(len(keys), kc, fc, n_rows, _ptr(bitmap), _ptr(count), _stream(stream)))


def pt_bloom_probe(keys: list[torch.Tensor], filters: list[Bloom], n_rows: int, bitmap: torch.Tensor,
                   count: torch.Tensor | None = None, stream=None) -> None:
    kc = (pt_column * max(1, len(keys)))(*[column(k) for k in keys])
    fc = (pt_bloom * max(1, len(filters)))(*[f.c() for f in filters])
    _check(_lib.pt_bloom_probe(len(keys), kc, fc, n_rows, _ptr(bitmap), _ptr(count), _stream(stream)))


def pt_compact_workspace_size(n_rows: int) -> int:
    out = C.c_size_t()
    _check(_lib.pt_compact_workspace_size(n_rows, C.byref(out)))
    return out.value


def pt_compact(bitmap: torch.Tensor, n_rows: int, idx: torch.Tensor, count: torch.Tensor,
               ws: torch.Tensor, stream=None) -> None:
    _check(_lib.pt_compact(_ptr(bitmap), n_rows, _ptr(idx), _ptr(count), _ptr(ws), ws.numel(),
                           _stream(stream)))


def pt_compact_noalloc(bitmap: torch.Tensor, n_rows: int, idx: torch.Tensor, count: torch.Tensor,
                       stream=None) -> None:
    """pt_compact without a workspace (static device scratch; n_rows <= 2^31)."""
    _check(_lib.pt_compact_noalloc(_ptr(bitmap), n_rows, _ptr(idx), _ptr(count), _stream(stream)))


def pt_profile_enable(on: bool | int) -> None:
    """on: False/0 off, True/1 every launch, 2 probe launches only."""
    _check(_lib.pt_profile_enable(int(on)))


def pt_profile_only(name: str | None, table: int = 0, pass_: int = 0) -> None:
    """Record events only around launches of this (name, table, pass);
    None records every launch the mode selects again."""
    _check(_lib.pt_profile_only(name.encode() if name else None, table, pass_))


def pt_profile_read(max_records: int = 4096) -> list[dict]:
    buf = (pt_kernel_time * max_records)()
    n = C.c_uint32()
    _check(_lib.pt_profile_read(buf, max_records, C.byref(n)))
    return [dict(name=buf[i].name.decode(), table=buf[i].table, pass_=buf[i].pass_, rows=buf[i].rows,
                 bytes=buf[i].bytes, ms=buf[i].ms) for i in range(n.value)]


# ------------------------------------------------------------ transfer

class DeviceProblem:
    """A join problem (`workloads.Problem`) with its columns in device memory
    and the C descriptors of its graph, tables and predicates."""

    def __init__(self, problem, device="cuda", columns=None):
        self.problem = problem
        self.n_tables = problem.n_tables
        self.n_rows = [problem.n_rows(t) for t in range(problem.n_tables)]
        if columns is None:
            columns = [{c: torch.from_numpy(np.ascontiguousarray(a)).to(device) for c, a in cols.items()}
                       for cols in problem.columns]
        self.columns = columns
        self._ccols = []
        self.tables = (pt_table * max(1, self.n_tables))()
        for t in range(self.n_tables):
            cc = (pt_column * max(1, len(columns[t])))(*[column(a) for a in columns[t].values()])
            self._ccols.append(cc)
            self.tables[t] = pt_table(self.n_rows[t], len(columns[t]), 0, cc)
        flags = problem.edge_flags if problem.edge_flags is not None else [0] * len(problem.edges)
        self.edges = (pt_edge * max(1, len(problem.edges)))(*[
            pt_edge(u, problem.col_index(u, uc), v, problem.col_index(v, vc), f)
            for (u, uc, v, vc), f in zip(problem.edges, flags)])
        self._orient = None
        orient_ptr = None
        if problem.orient is not None:
            self._orient = (C.c_int8 * len(problem.orient))(*problem.orient)
            orient_ptr = C.cast(self._orient, C.POINTER(C.c_int8))
        self.graph = pt_graph(self.n_tables, len(problem.edges), self.edges, orient_ptr)
        self.preds = (pt_pred * max(1, len(problem.preds)))(*[
            pt_pred(t, problem.col_index(t, c), OPS[op], 0, lo, hi) for t, c, op, lo, hi in problem.preds])
        self.n_preds = len(problem.preds)


def pt_transfer_workspace_size(dp: DeviceProblem, p: pt_params) -> int:
    out = C.c_size_t()
    _check(_lib.pt_transfer_workspace_size(C.byref(dp.graph), dp.tables, C.byref(p), C.byref(out)))
    return out.value


def pt_transfer(dp: DeviceProblem, p: pt_params, ws: torch.Tensor, bitmaps: list[torch.Tensor],
                counts: torch.Tensor | None = None, stream=None) -> None:
    bm = (C.c_void_p * max(1, dp.n_tables))(*[b.data_ptr() if b.numel() else 0 for b in bitmaps])
    _check(_lib.pt_transfer(C.byref(dp.graph), dp.tables, dp.preds, dp.n_preds, C.byref(p), _ptr(ws),
                            ws.numel(), bm, _ptr(counts), _stream(stream)))


def pt_transfer_filter(dp: DeviceProblem, p: pt_params, ws: torch.Tensor, pass_: int, edge: int):
    out = pt_bloom()
    builder = C.c_uint32()
    _check(_lib.pt_transfer_filter(C.byref(dp.graph), dp.tables, C.byref(p), _ptr(ws), pass_, edge,
                                   C.byref(out), C.byref(builder)))
    return out, builder.value


class Transfer:
    """Holds the workspace, bitmaps and counts of one problem and runs the
    transfer phase on it (all allocation happens here, once)."""

    def __init__(self, dp: DeviceProblem, p: pt_params | None = None, device="cuda",
                 ws: torch.Tensor | None = None):
        self.dp = dp
        self.params = p if p is not None else params()
        self.ws_bytes = pt_transfer_workspace_size(dp, self.params)
        if ws is not None:
            if ws.numel() < self.ws_bytes:
                raise ValueError(f"workspace of {ws.numel()} bytes, {self.ws_bytes} needed")
            self.ws = ws
        else:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.bitmaps = [torch.empty(bitmap_words(n), dtype=torch.int64, device=device) for n in dp.n_rows]
        self.counts = torch.zeros(dp.n_tables, dtype=torch.int64, device=device)

    def run(self, stream=None) -> None:
        pt_transfer(self.dp, self.params, self.ws, self.bitmaps, self.counts, stream)

    def check_status(self, stream=None) -> None:
        """Raises PtError(PT_EOVERFLOW) if the latest run's kernels reported
        an overflow (waits for the stream)."""
        pt_check_status(self.ws, stream)

    def bitmap(self, t: int) -> np.ndarray:
        return self.bitmaps[t].cpu().numpy().view(np.uint64)

    def filter(self, pass_: int, edge: int) -> tuple[np.ndarray, int, int]:
        """(used words, nb, builder) of the filter `edge` carried in pass 1
        (forward) or 2 (backward)."""
        b, builder = pt_transfer_filter(self.dp, self.params, self.ws, pass_, edge)
        off = b.words - self.ws.data_ptr()
        nb_off = b.d_nb - self.ws.data_ptr()
        nb = int(self.ws[nb_off:nb_off + 8].cpu().numpy().view(np.uint64)[0])
        n = nb * (self.params.block_bits // 32)
        words = self.ws[off:off + 4 * n].cpu().numpy().view(np.uint32)
        return words, nb, builder


def pt_join_workspace_size(dp: DeviceProblem, root: int, out_cap: int) -> int:
    out = C.c_size_t()
    _check(_lib.pt_join_workspace_size(C.byref(dp.graph), dp.tables, root, out_cap, C.byref(out)))
    return out.value


def pt_join(dp: DeviceProblem, root: int, bitmaps: list | None, out: list, out_cap: int, n_out: torch.Tensor,
            ws: torch.Tensor, stream=None) -> None:
    """bitmaps: None, or per table a bitmap tensor (None: every row); out:
    per table a uint32 tensor of out_cap ids (None outside root's
    component)."""
    n = max(1, dp.n_tables)
    bm = None
    if bitmaps is not None:
        bm = (C.c_void_p * n)(*[b.data_ptr() if b is not None and b.numel() else None for b in bitmaps])
    op = (C.c_void_p * n)(*[o.data_ptr() if o is not None else None for o in out])
    _check(_lib.pt_join(C.byref(dp.graph), dp.tables, root, bm, op, out_cap, _ptr(n_out), _ptr(ws), ws.numel(),
                        _stream(stream)))


def component_of(problem, root: int) -> list[int]:
    """Tables connected to root through join edges, ascending."""
    seen, todo = {root}, [root]
    while todo:
        t = todo.pop()
        for u, _, v, _ in problem.edges:
            for a, b in ((u, v), (v, u)):
                if a == t and b not in seen:
                    seen.add(b)
                    todo.append(b)
    return sorted(seen)


class Join:
    """Workspace and outputs of the join phase (pt_join) on one problem: row
    ids of every tuple, one uint32 column per table of root's component."""

    def __init__(self, dp: DeviceProblem, root: int | None = None, out_cap: int = 1 << 20, device="cuda"):
        self.dp = dp
        if root is None:  # start from the largest table: the added tables are the build sides
            root = max(range(dp.n_tables), key=lambda t: (dp.n_rows[t], -t))
        self.root = root
        self.comp = component_of(dp.problem, root)
        self.out_cap = out_cap
        self.ws = torch.empty(pt_join_workspace_size(dp, root, out_cap), dtype=torch.uint8, device=device)
        self.out = [torch.empty(max(1, out_cap), dtype=torch.int32, device=device) if t in self.comp else None
                    for t in range(dp.n_tables)]
        self.n_out = torch.zeros(1, dtype=torch.int64, device=device)

    def run(self, bitmaps: list | None = None, stream=None) -> None:
        pt_join(self.dp, self.root, bitmaps, self.out, self.out_cap, self.n_out, self.ws, stream)

    def check_status(self, stream=None) -> None:
        pt_check_status(self.ws, stream)

    def tuples(self) -> np.ndarray:
        """The tuples of the last run (columns: self.comp), sorted."""
        n = int(self.n_out.item())
        n = min(n, self.out_cap)
        cols = [self.out[t][:n].cpu().numpy().view(np.uint32) for t in self.comp]
        arr = np.stack(cols, axis=1) if cols else np.zeros((n, 0), np.uint32)
        return arr[np.lexsort(arr.T[::-1])] if n else arr


def pt_batch_workspace_size(dps: list[DeviceProblem], ps: list[pt_params]) -> int:
    probs = (pt_problem * max(1, len(dps)))()
    for i, dp in enumerate(dps):
        probs[i] = pt_problem(C.pointer(dp.graph), dp.tables, dp.preds, dp.n_preds, 0, ps[i], None, None)
    size = C.c_size_t()
    _check(_lib.pt_batch_workspace_size(len(dps), probs, C.byref(size)))
    return size.value


class Batch:
    """Many problems run together (pt_batch_*): one persistent kernel launch
    for all of them, captured once into a HIP graph. Holds the workspace,
    every problem's bitmaps and counts."""

    def __init__(self, dps: list[DeviceProblem], ps: list[pt_params] | None = None, device="cuda",
                 stream=None, ws: torch.Tensor | None = None):
        """stream: prepare asynchronously on this stream (runs must follow on
        it); ws: a uint8 device buffer to use as the workspace (at least
        pt_batch_workspace_size bytes, 256-byte aligned) instead of a new one."""
        self.dps = dps
        self.params = ps if ps is not None else [params() for _ in dps]
        self.bitmaps = [[torch.empty(bitmap_words(n), dtype=torch.int64, device=device) for n in dp.n_rows]
                        for dp in dps]
        self.counts = [torch.zeros(dp.n_tables, dtype=torch.int64, device=device) for dp in dps]
        self._bm = [(C.c_void_p * max(1, dp.n_tables))(*[b.data_ptr() if b.numel() else 0 for b in bms])
                    for dp, bms in zip(dps, self.bitmaps)]
        self._probs = (pt_problem * max(1, len(dps)))()
        for i, dp in enumerate(dps):
            self._probs[i] = pt_problem(C.pointer(dp.graph), dp.tables, dp.preds, dp.n_preds, 0, self.params[i],
                                        self._bm[i], self.counts[i].data_ptr())
        size = C.c_size_t()
        _check(_lib.pt_batch_workspace_size(len(dps), self._probs, C.byref(size)))
        if ws is not None:
            if ws.numel() < size.value:
                raise ValueError(f"workspace of {ws.numel()} bytes, {size.value} needed")
            self.ws = ws
        else:
            self.ws = torch.empty(size.value, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        if stream is None:
            _check(_lib.pt_batch_prepare(len(dps), self._probs, _ptr(self.ws), self.ws.numel(), C.byref(h)))
        else:
            _check(_lib.pt_batch_prepare_async(len(dps), self._probs, _ptr(self.ws), self.ws.numel(),
                                               _stream(stream), C.byref(h)))
        self._h = h

    def run(self, stream=None, eager: bool = False) -> None:
        _check(_lib.pt_batch_run(self._h, _stream(stream), PT_BATCH_EAGER if eager else 0))

    def check_status(self, stream=None) -> None:
        pt_check_status(self.ws, stream)

    def info(self) -> tuple[int, int]:
        """(kernel launches per run, rows probed per run)."""
        n, rows = C.c_uint32(), C.c_uint64()
        _check(_lib.pt_batch_info(self._h, C.byref(n), C.byref(rows)))
        return n.value, rows.value

    def timeline(self) -> tuple[np.ndarray, int]:
        """Per item (start, end, kind, phase) of the last run, and the wall
        clock's ticks per millisecond (batches prepared with
        PT_BATCH_TIMELINE=1 in the environment)."""
        n_items, _ = self.info()
        buf = (C.c_uint64 * (4 * 1_000_000))()
        n, rate = C.c_uint32(), C.c_uint32()
        _check(_lib.pt_batch_timeline(self._h, buf, 1_000_000, C.byref(n), C.byref(rate)))
        return np.frombuffer(buf, dtype=np.uint64, count=4 * n.value).reshape(n.value, 4).copy(), rate.value

    def bitmap(self, i: int, t: int) -> np.ndarray:
        return self.bitmaps[i][t].cpu().numpy().view(np.uint64)

    def close(self) -> None:
        if self._h:
            _lib.pt_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
