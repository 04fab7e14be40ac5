"""Per-size-class options of the block solves, from a table measured on the GPU.

A plan's block-solve work is set by the width of its widest band and by how
many work units (boxes x 8-column chunks of the LOBPCG block) it spreads over
the 256 CUs.  The size class buckets both:

    widest Ahat band (tiles): <= 20, <= 24, <= 31, <= 41, <= 65
    work units:               < 64, < 256, < 1024, >= 1024

For each class the table (tuning.json, written by autotune.py from timed runs
of the local stage) holds the fastest measured choice of

    split  MSGFEM_OPT_SPLIT  nested dissection of the box matrices (0 / 1)
    solve  MSGFEM_OPT_SOLVE  block-solve family (1 vector, 2 matrix cores x 8
                             columns, 3 matrix cores x 16 columns)
    graph  MSGFEM_OPT_GRAPH  LOBPCG iterations replayed from HIP graphs (0 / 1)

A class missing from the table keeps the library defaults.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
BT_EDGES = (20, 24, 31, 41, 65)
UNIT_EDGES = (64, 256, 1024)
KEYS = ("split", "solve", "graph")


def size_class(max_bt_ahat: int, n_box: int, k: int) -> str:
    units = n_box * ((k + 7) // 8)
    b = next((e for e in BT_EDGES if max_bt_ahat <= e), BT_EDGES[-1])
    u = next((e for e in UNIT_EDGES if units < e), None)
    return f"bt<={b},units<{u}" if u is not None else f"bt<={b},units>={UNIT_EDGES[-1]}"


_cache: Dict[str, dict] = {}


def load(path: str = TABLE) -> dict:
    """The table ({} when there is none)."""
    if path not in _cache:
        try:
            with open(path) as f:
                _cache[path] = json.load(f)
        except FileNotFoundError:
            _cache[path] = {}
    return _cache[path]


def options_for(cls: str, path: str = TABLE) -> Optional[dict]:
    """{"split", "solve", "graph"} for a size class, or None."""
    entry = load(path).get("classes", {}).get(cls)
    if not entry:
        return None
    return {key: int(entry[key]) for key in KEYS if key in entry}
