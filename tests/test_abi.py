"""The C ABI library loads and exports every symbol include/pt.h declares;
host-side argument checks and sizing run without a GPU (no kernel is
launched by anything in this file)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ptlib():
    from paper_2307_15255_amd import pt
    return pt


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pt_local_filter", "pt_bloom_build", "pt_bloom_probe", "pt_compact",
                     "pt_transfer"):
        assert required in names


def test_library_exports_every_declared_symbol(ptlib):
    lib = C.CDLL(ptlib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(ptlib.EXPORTS)


def test_version(ptlib):
    assert "gfx950" in ptlib.pt_version()


def test_capacity_and_workspace_sizes(ptlib):
    import oracle
    p = ptlib.params(512, 3, 10)
    for n in (0, 1, 51, 52, 20_000, 100_000_000):
        assert ptlib.pt_bloom_capacity(n, p) == oracle.filter_blocks(n, 10, 512) * 16
    assert ptlib.pt_compact_workspace_size(0) == 8
    assert ptlib.pt_compact_workspace_size(65536 * 3 + 1) == 5 * 8


def test_parameter_validation(ptlib):
    bad = [ptlib.pt_params(48, 3, 10, 0), ptlib.pt_params(2048, 3, 10, 0), ptlib.pt_params(512, 0, 10, 0),
           ptlib.pt_params(512, 17, 10, 0), ptlib.pt_params(512, 3, 0, 0), ptlib.pt_params(512, 3, 65, 0),
           ptlib.pt_params(512, 3, 10, 16), ptlib.pt_params(512, 3, 10, 0x80000001)]
    for p in bad:
        with pytest.raises(ptlib.PtError) as ei:
            ptlib.pt_bloom_capacity(10, p)
        assert ei.value.status == ptlib.PT_EINVAL


class _HostProblem:
    """C descriptors for a graph whose columns point at host memory: enough
    for the planner (workspace size), which never touches column data."""

    def __init__(self, ptlib, rows, edges, orient=None):
        self.keep = []
        self.tables = (ptlib.pt_table * len(rows))()
        for t, n in enumerate(rows):
            a = np.zeros(max(n, 1), np.int32)
            self.keep.append(a)
            cc = (ptlib.pt_column * 2)(ptlib.pt_column(a.ctypes.data, 0, 0), ptlib.pt_column(a.ctypes.data, 0, 0))
            self.keep.append(cc)
            self.tables[t] = ptlib.pt_table(n, 2, 0, cc)
        self.edges = (ptlib.pt_edge * max(1, len(edges)))(*[ptlib.pt_edge(*e) for e in edges])
        o = None
        if orient is not None:
            self.o = (C.c_int8 * len(orient))(*orient)
            o = C.cast(self.o, C.POINTER(C.c_int8))
        self.graph = ptlib.pt_graph(len(rows), len(edges), self.edges, o)

    def ws(self, ptlib, p):
        out = C.c_size_t()
        st = ptlib.lib().pt_transfer_workspace_size(C.byref(self.graph), self.tables, C.byref(p), C.byref(out))
        return st, out.value


def test_planner_validation(ptlib):
    p = ptlib.params()
    ok = _HostProblem(ptlib, [10, 100, 1000], [(0, 0, 1, 0), (1, 1, 2, 0)])
    st, size = ok.ws(ptlib, p)
    assert st == ptlib.PT_OK and size > 0
    # every filter at its largest size: forward builders R (10 rows) and S (100); backward S and T
    cap = lambda n: ptlib.pt_bloom_capacity(n, p) * 4
    assert size >= cap(10) + cap(100) + cap(100) + cap(1000)
    for rows, edges, orient in [
        ([10, 100], [(0, 0, 0, 1)], None),          # self-join edge
        ([10, 100], [(0, 0, 2, 0)], None),          # table out of range
        ([10, 100], [(0, 5, 1, 0)], None),          # column out of range
        ([10, 100, 5], [(0, 0, 1, 0), (1, 0, 2, 0), (2, 0, 0, 0)], [1, 1, 1]),  # directed cycle
        ([10, 100], [(0, 0, 1, 0)], [0]),           # orientation not +-1
        ([2**32, 5], [(0, 0, 1, 0)], None),         # too many rows
    ]:
        st, _ = _HostProblem(ptlib, rows, edges, orient).ws(ptlib, p)
        assert st == ptlib.PT_EINVAL, (rows, edges, orient)
    # a cycle in the join graph itself is fine: the size rule orients it acyclically
    st, _ = _HostProblem(ptlib, [10, 100, 5], [(0, 0, 1, 0), (1, 0, 2, 0), (2, 0, 0, 0)]).ws(ptlib, p)
    assert st == ptlib.PT_OK


def test_layout_parameters_validation(ptlib):
    """hash_version, tile_rows and probe_order are checked on the host; only
    the filter specification of version 1 is implemented."""
    ok = [ptlib.params(512, 3, 10, hash_version=0), ptlib.params(512, 3, 10, hash_version=1),
          ptlib.params(512, 3, 10, tile_rows=4096), ptlib.params(512, 3, 10, tile_rows=1 << 24),
          ptlib.params(512, 3, 10, probe_order=ptlib.PT_PROBE_GIVEN), ptlib.params(512, 3, 10, lds_budget=1)]
    for p in ok:
        assert ptlib.pt_bloom_capacity(10, p) == 16
    for p, status in [(ptlib.params(512, 3, 10, hash_version=2), ptlib.PT_EUNSUPPORTED),
                      (ptlib.params(512, 3, 10, tile_rows=100), ptlib.PT_EINVAL),
                      (ptlib.params(512, 3, 10, tile_rows=(1 << 24) + 4096), ptlib.PT_EINVAL),
                      (ptlib.params(512, 3, 10, probe_order=2), ptlib.PT_EINVAL)]:
        with pytest.raises(ptlib.PtError) as ei:
            ptlib.pt_bloom_capacity(10, p)
        assert ei.value.status == status


def test_edge_flags(ptlib):
    """Join types 0-3 (inner, left, right, full outer) are planned; other
    values are rejected."""
    p = ptlib.params()
    for flags in (ptlib.PT_EDGE_INNER, ptlib.PT_EDGE_LEFT_OUTER, ptlib.PT_EDGE_RIGHT_OUTER, ptlib.PT_EDGE_FULL_OUTER):
        assert _HostProblem(ptlib, [10, 100], [(0, 0, 1, 0, flags)]).ws(ptlib, p)[0] == ptlib.PT_OK
    assert _HostProblem(ptlib, [10, 100], [(0, 0, 1, 0, 4)]).ws(ptlib, p)[0] == ptlib.PT_EUNSUPPORTED
    assert "flags" in ptlib.lib().pt_last_error().decode()


def test_check_status_rejects_null(ptlib):
    assert ptlib.lib().pt_check_status(None, None) == ptlib.PT_EINVAL


def test_compact_noalloc_rejects_inputs_beyond_its_scratch(ptlib):
    """Host-side checks of the allocation-free compaction: nothing is queued."""
    lib = ptlib.lib()
    assert lib.pt_compact_noalloc(None, (1 << 31) + 1, None, None, None) == ptlib.PT_EINVAL
    assert "2^31" in lib.pt_last_error().decode()
    assert lib.pt_compact_noalloc(None, 10, None, None, None) == ptlib.PT_EINVAL  # NULL count


def _join_ws(ptlib, prob, root, cap):
    out = C.c_size_t()
    st = ptlib.lib().pt_join_workspace_size(C.byref(prob.graph), prob.tables, root, cap, C.byref(out))
    return st, out.value


def test_join_planner_validation(ptlib):
    """pt_join's host checks and workspace sizing (no kernel runs)."""
    chain = _HostProblem(ptlib, [10, 100, 1000], [(0, 0, 1, 0), (1, 1, 2, 0)])
    st, size = _join_ws(ptlib, chain, 2, 4096)
    assert st == ptlib.PT_OK
    # ids of three tables, hash tables of the two added ones (at least twice
    # their rows in 8-byte keys), two buffers of two-column intermediate tuples
    assert size >= 4 * 1110 + 12 * (2 * 10 + 2 * 100) + 2 * 2 * 4096 * 4
    assert _join_ws(ptlib, chain, 2, 8192)[1] > size  # intermediates grow with out_cap
    two = _HostProblem(ptlib, [10, 100], [(0, 0, 1, 0)])
    assert _join_ws(ptlib, two, 1, 1 << 30)[1] < 1 << 20  # a two-table join has no intermediates
    lone = _HostProblem(ptlib, [10, 100, 7], [(0, 0, 1, 0)])
    assert _join_ws(ptlib, lone, 2, 100)[0] == ptlib.PT_OK  # a table with no edge joins alone
    assert _join_ws(ptlib, chain, 3, 100)[0] == ptlib.PT_EINVAL  # root out of range
    assert _join_ws(ptlib, _HostProblem(ptlib, [10, 100], [(0, 0, 0, 1)]), 0, 100)[0] == ptlib.PT_EINVAL
    assert _join_ws(ptlib, _HostProblem(ptlib, [10, 100], [(0, 0, 1, 5)]), 0, 100)[0] == ptlib.PT_EINVAL
    assert _join_ws(ptlib, _HostProblem(ptlib, [10, 100], [(0, 0, 1, 0, 1)]), 0, 100)[0] == ptlib.PT_EUNSUPPORTED
    assert _join_ws(ptlib, chain, 0, (1 << 36) + 1)[0] == ptlib.PT_EINVAL
    # more than 32 tables in one component
    big = _HostProblem(ptlib, [5] * 33, [(i, 0, i + 1, 0) for i in range(32)])
    assert _join_ws(ptlib, big, 0, 100)[0] == ptlib.PT_EUNSUPPORTED
    # ten edges from one table to the tables before it
    par = _HostProblem(ptlib, [5, 5], [(0, 0, 1, 0)] * 10)
    assert _join_ws(ptlib, par, 0, 100)[0] == ptlib.PT_EUNSUPPORTED
    assert _join_ws(ptlib, _HostProblem(ptlib, [5, 5], [(0, 0, 1, 0)] * 9), 0, 100)[0] == ptlib.PT_OK


def test_join_rejects_bad_buffers(ptlib):
    lib = ptlib.lib()
    chain = _HostProblem(ptlib, [10, 100, 1000], [(0, 0, 1, 0), (1, 1, 2, 0)])
    st, size = _join_ws(ptlib, chain, 2, 16)
    n_out = C.c_uint64()
    outs = (C.c_void_p * 3)(1 << 12, 1 << 12, 1 << 12)
    # NULL workspace, misaligned workspace, short workspace, NULL count, NULL output column
    assert lib.pt_join(C.byref(chain.graph), chain.tables, 2, None, outs, 16, C.byref(n_out), None, size,
                       None) == ptlib.PT_EINVAL
    assert lib.pt_join(C.byref(chain.graph), chain.tables, 2, None, outs, 16, C.byref(n_out), 4096 + 8, size,
                       None) == ptlib.PT_EINVAL
    assert lib.pt_join(C.byref(chain.graph), chain.tables, 2, None, outs, 16, C.byref(n_out), 4096, size - 1,
                       None) == ptlib.PT_ENOMEM
    assert lib.pt_join(C.byref(chain.graph), chain.tables, 2, None, outs, 16, None, 4096, size,
                       None) == ptlib.PT_EINVAL
    outs[1] = None
    assert lib.pt_join(C.byref(chain.graph), chain.tables, 2, None, outs, 16, C.byref(n_out), 4096, size,
                       None) == ptlib.PT_EINVAL
    assert "d_out[1]" in lib.pt_last_error().decode()


def test_exact_flag_planning(ptlib):
    """PT_FLAG_EXACT: the transfer plans key sets (at least 16 bytes per
    builder row); a batch rejects it."""
    chain = _HostProblem(ptlib, [10, 100, 1000], [(0, 0, 1, 0), (1, 1, 2, 0)])
    st, size = chain.ws(ptlib, ptlib.params(flags=ptlib.PT_FLAG_EXACT))
    assert st == ptlib.PT_OK
    # forward builders R (10 rows) and S (100), backward S and T (1 000)
    assert size >= 16 * (10 + 100 + 100 + 1000)
    probs = (ptlib.pt_problem * 1)()
    probs[0] = ptlib.pt_problem(C.pointer(chain.graph), chain.tables, None, 0, 0,
                                ptlib.params(flags=ptlib.PT_FLAG_EXACT), None, None)
    out = C.c_size_t()
    assert ptlib.lib().pt_batch_workspace_size(1, probs, C.byref(out)) == ptlib.PT_EUNSUPPORTED


def test_profile_switches(ptlib):
    """Profiling switches are host state: a mode outside 0..2 is rejected,
    a selection set and cleared, and nothing is recorded without a launch."""
    with pytest.raises(ptlib.PtError) as ei:
        ptlib.pt_profile_enable(3)
    assert ei.value.status == ptlib.PT_EINVAL
    ptlib.pt_profile_only("probe", 2, 1)
    ptlib.pt_profile_only(None)
    assert ptlib.pt_profile_read(16) == []
