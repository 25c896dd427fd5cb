"""Panel-height table of the batched form: loaded from ``tune_table.json`` (written by
``autotune.py`` on the GPU) into the library's table once per process."""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tune_table.json")

_loaded = False


def load_table(path: str = TABLE) -> dict | None:
    """Apply the recorded variants with tsqr_tune_set; returns the table, or None if absent."""
    global _loaded
    if not os.path.exists(path):
        _loaded = True
        return None
    import torch
    from .tsqr import tune_set
    with open(path) as f:
        table = json.load(f)
    for e in table.get("entries", []):
        dt = torch.float32 if e["dtype"] == "f32" else torch.float64
        tune_set(dt, int(e["n"]), int(e["variant"]))
    _loaded = True
    return table


def ensure_loaded() -> None:
    if not _loaded:
        load_table()
