"""Run a fast subset of the oracle pins against an oracle build given on the
command line; exit 0 if every pin holds, 1 if one fails. The planted-mistake
test starts this in a subprocess for each mutated oracle."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import test_oracle_filter as F  # noqa: E402
import test_oracle_join as J  # noqa: E402
import test_oracle_outer as OU  # noqa: E402
import test_oracle_prune as PR  # noqa: E402
import test_oracle_threads as TH  # noqa: E402
import test_oracle_transfer as T  # noqa: E402


def checks():
    yield lambda: F.test_hash_matches_python_integers(None)
    yield lambda: F.test_slots_match_python_integers(None, 512, 3)
    yield lambda: F.test_filter_blocks(None)
    yield lambda: F.test_no_false_negatives(None, 512, 3, 10)
    yield lambda: F.test_fpr_matches_filter_bits(None, 512, 3, 10)
    for shape in ("chain", "cycle", "parallel"):
        yield lambda shape=shape: T.test_sound_and_superset(None, shape)
    yield lambda: T.test_exact_in_tree_is_yannakakis_full_reduction(None, "tree")
    yield lambda: T.test_fig3_worked_example(None, oracle.EXACT, 3, 10)
    yield lambda: T.test_fig2_filter_transformation(None)
    yield lambda: T.test_orientation_rule(None)
    yield lambda: T.test_edge_cases(None)
    yield lambda: T.test_local_filter_ops(None)
    yield lambda: T.test_compact(None)
    yield lambda: T.test_bloom_join_is_one_hop_transfer(None)
    for shape in ("tree", "cycle"):
        yield lambda shape=shape: J.test_join_matches_brute_force(None, shape)
    yield lambda: J.test_join_edge_cases(None)
    yield lambda: TH.test_threads_tiny(None, "tree")
    yield lambda: OU.test_outer_tree_query_unchanged(None, "tree")
    yield lambda: PR.test_prune_worked_example(None, oracle.EXACT, 3, 10)
    yield lambda: PR.test_prune_keeps_an_empty_tables_filter(None)
    yield lambda: OU.test_full_outer_blocks_every_transfer(None)
    yield lambda: OU.test_preserved_side_keeps_its_rows(None, 1, 0)


def main():
    oracle.use_library(sys.argv[1])
    for i, check in enumerate(checks()):
        try:
            check()
        except Exception as e:  # any failing pin (or error) means the mistake was caught
            print(f"pin {i} failed: {type(e).__name__}")
            return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
