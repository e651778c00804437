"""Evidence kept when a run reports corrupted state.

bml_stats returns BML_ECORRUPT when a per-step car count differs from the
lattice's initial one: cars were created or lost, which the automaton never
does (every car either stays or moves into an EMPTY cell).  Callers that hit
it (the autotuner, the benchmark) write what they know before stopping: the
message (it names the first bad step and both counts), the lattice's shape,
layout, tuning and step count, and its cells as they are now.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import _lib as L


def dump_dir() -> str:
    """Where evidence goes: $BML_DUMP_DIR, else ./bml_dumps."""
    return os.environ.get("BML_DUMP_DIR") or os.path.join(os.getcwd(), "bml_dumps")


def dump_corruption(err: L.BmlError, lattice, where: str, extra: dict | None = None) -> str:
    """Write <dump_dir>/<where>-<time>.json (and .npy with the cells when they
    can still be read back); returns the JSON path."""
    d = dump_dir()
    os.makedirs(d, exist_ok=True)
    stem = os.path.join(d, f"{where}-{time.strftime('%Y%m%d-%H%M%S')}-{os.getpid()}")
    rec = {"where": where, "code": err.code, "message": err.message, **(extra or {})}
    try:
        rec.update({"rows": lattice.rows, "cols": lattice.cols, "layout": lattice.layout,
                    "steps_done": lattice.steps_done, "tuning": list(lattice.tuning()),
                    "initial_counts": list(lattice.initial_counts())})
        np.save(stem + ".npy", lattice.cells())
        rec["cells"] = stem + ".npy"
    except Exception as e:      # the device may be unusable by now
        rec["cells_error"] = repr(e)
    with open(stem + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    return stem + ".json"
