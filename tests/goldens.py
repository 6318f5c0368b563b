"""Loaders for the authored worked-example fixtures under tests/golden/."""
from __future__ import annotations

import json
import os

import numpy as np

from paper_2307_15255_amd.workloads import Problem

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> tuple[Problem, dict]:
    with open(os.path.join(GOLDEN, name)) as f:
        spec = json.load(f)
    names = list(spec["tables"].keys())
    columns = [{c: np.array(v, np.int32) for c, v in spec["tables"][t].items()} for t in names]
    edges = [(names.index(u), uc, names.index(v), vc) for u, uc, v, vc in spec["edges"]]
    preds = []
    for t, c, op, lo, hi in spec.get("preds", []):
        preds.append((names.index(t), c, op, lo, hi))
    prob = Problem(names, columns, edges, preds, orient=spec.get("orient"), label=name)
    return prob, spec
