"""Plant plausible mistakes in a copy of the oracle (a dropped term, a wrong
sign, index or operand) and check that each one fails at least one pin. The
unmodified oracle must pass the same pins."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(oracle.__file__), "pt_oracle.c")

MUTANTS = {
    "xorshift_direction": ("t = t ^ (t >> 16);", "t = t ^ (t << 16);"),
    "dropped_high_word_fold": ("uint32_t t = lo ^ hi;", "uint32_t t = lo;"),
    "size_floor_not_ceil": ("(bits + block_bits - 1) / block_bits", "bits / block_bits"),
    "block_not_scaled": ("((uint64_t)h1 * nb) >> 32", "((uint64_t)h1 * nb) >> 33"),
    "stride_not_odd": ("& (block_bits - 1)) | 1u;", "& (block_bits - 1));"),
    "dropped_probe_index": ("pos[i] = (g1 + i * g2)", "pos[i] = (g1 + g2)"),
    "word_index_unscaled": ("uint64_t w = blk * words_per_block + pos[i] / 32;\n    words[w]",
                            "uint64_t w = blk + pos[i] / 32;\n    words[w]"),
    "orientation_reversed": ("u_first = (nu < nv) || (nu == nv && u < v);",
                             "u_first = (nu > nv) || (nu == nv && u < v);"),
    "tie_break_reversed": ("u_first = (nu < nv) || (nu == nv && u < v);",
                           "u_first = (nu < nv) || (nu == nv && u > v);"),
    "backward_not_reversed": ("rc = run_pass(p, pa, 1, dst, src, rev_order",
                              "rc = run_pass(p, pa, 1, src, dst, order"),
    "probe_never_clears": ("column_value(col, r))) bit_clear(bm, r);", "column_value(col, r))) (void)0;"),
    "threads_merge_overwrites": ("f->words[i] |= mine[i];", "f->words[i] = mine[i];"),
    "threads_split_drops_tail": ("const uint64_t end = (uint64_t)w * 64 + 64;", "const uint64_t end = (uint64_t)w * 64 + 63;"),
    "between_exclusive": ("p->lo <= v && v <= p->hi", "p->lo <= v && v < p->hi"),
    "lt_as_le": ("case PTOR_LT: return v < p->lo;", "case PTOR_LT: return v <= p->lo;"),
    "zero_extend_int32": ("return (int64_t)((const int32_t *)c->data)[r];",
                          "return (int64_t)((const uint32_t *)c->data)[r];"),
    "build_before_probe": None,  # handled below: outgoing filters built before incoming probes
    "no_backward_pass": ("if (pa->n_passes == 2) {", "if (pa->n_passes == 3) {"),
    "local_preds_ignored": ("if (pr->table == t && !predicate_holds", "if (pr->table == t + 1 && !predicate_holds"),
    "outer_left_reversed": ("case PTOR_LEFT_OUTER: return from == ed->u && to == ed->v;",
                            "case PTOR_LEFT_OUTER: return from == ed->v && to == ed->u;"),
    "outer_full_not_blocked": ("return from == ed->v && to == ed->u;\n    default: return 0;",
                               "return from == ed->v && to == ed->u;\n    default: return 1;"),
    "join_skips_closing_edge": ("if ((uint32_t)slot[b_t] >= i) continue;",
                                "if ((uint32_t)slot[b_t] >= i || b_t != u) continue;"),
    "join_upper_bound": ("if (index[mid].key < key) lo = mid + 1;", "if (index[mid].key <= key) lo = mid + 1;"),
    "join_ignores_bitmap": ("if (!row_selected(bitmaps, v, r)) continue;", "(void)0;"),
    "prune_ignores_reduction": ("pa->prune && t->n_rows > 0 && bitmap_popcount(bitmaps[v], t->n_rows) == t->n_rows",
                                "pa->prune"),
    "prune_empty_tables": ("pa->prune && t->n_rows > 0 && bitmap_popcount", "pa->prune && bitmap_popcount"),
    "prune_absent_blocks_keys": ("if (f->absent) return 1;", "if (f->absent) return 0;"),
    "join_columns_in_bfs_order": ("sorted[j * w + q] = cur[j * w + slot[comp[q]]];",
                                  "sorted[j * w + q] = cur[j * w + q];"),
}


def _mutate(text: str, name: str) -> str:
    if name == "build_before_probe":
        a = text.index("    for (uint32_t j = 0; j < m; j++) {\n      uint32_t e = reverse_probe")
        b = text.index("    /* Transfer path pruning: a non-empty table")
        c = text.index("  return PTOR_OK;\n}\n\nstatic int problem_valid")
        probe, build = text[a:b], text[b:c - len("  }\n")]
        return text[:a] + build + probe + text[c - len("  }\n"):]
    old, new = MUTANTS[name]
    assert text.count(old) >= 1, name
    return text.replace(old, new, 1)


def _run(path):
    return subprocess.run([sys.executable, os.path.join(HERE, "mutant_pins.py"), path],
                          capture_output=True, text=True, timeout=600)


def test_unmodified_oracle_passes_fast_pins(tmp_path):
    with open(SRC) as f:
        text = f.read()
    so = oracle.build_variant(text, str(tmp_path / "plain.so"))
    r = _run(so)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    with open(SRC) as f:
        text = f.read()
    so = oracle.build_variant(_mutate(text, name), str(tmp_path / f"{name}.so"))
    r = _run(so)
    assert r.returncode != 0, f"mistake {name} passed every pin"
