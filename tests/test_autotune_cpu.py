"""Host-side checks of the autotuner's bit-exactness gate (no GPU): a
candidate whose car counts are not conserved stops the tuning with its
evidence written to disk, and a candidate that differs from the reference
stops it too -- neither is skipped as a mere rejected candidate."""
import json
import os

import numpy as np
import pytest

from paper_1804_07981_amd import _lib as L
from paper_1804_07981_amd import autotune


class FakeLattice:
    """Stands in for Lattice: fixed cells and counts, or BML_ECORRUPT."""
    corrupt = False
    cells_value = 0

    def __init__(self, n, rho, seed, layout=0, stats_cap=0, stream=None):
        self.rows = self.cols = n
        self.layout = layout
        self.steps_done = 0
        self._tuning = (0, 8, 4)

    def set_tuning(self, tr, tp, w):
        self._tuning = (tr, tp, w)

    def tuning(self):
        return self._tuning

    def initial_counts(self):
        return (10, 10)

    def cells(self):
        return np.full((self.rows, self.cols), self.cells_value, np.uint8)

    def stats(self, first, count):
        if self.corrupt:
            raise L.BmlError(L.BML_ECORRUPT, "step 462: car counts (2, 5) differ from the "
                             "initial (10, 10)")
        rec = np.zeros(count, dtype=L.STEP_STATS_DTYPE)
        rec["n_lr"] = 10
        rec["n_tb"] = 10
        return rec

    def close(self):
        pass


def fake_step(lats, steps):
    for lat in lats:
        lat.steps_done += steps


def test_tune_group_raises_on_corrupted_counts(tmp_path, monkeypatch):
    monkeypatch.setenv("BML_DUMP_DIR", str(tmp_path))
    monkeypatch.setattr(FakeLattice, "corrupt", True)
    with pytest.raises(L.BmlError) as err:
        autotune.tune_group([(32, 0.3, 1), (32, 0.4, 2)], 0, "fake", strip_rows=(16,),
                            t_phases=(14,), waves=(2,), steps=8, log=lambda m: None,
                            make_lattice=FakeLattice, step=fake_step)
    assert err.value.code == L.BML_ECORRUPT
    dumps = sorted(f for f in os.listdir(tmp_path) if f.endswith(".json"))
    assert len(dumps) == 1
    rec = json.load(open(tmp_path / dumps[0]))
    assert "step 462" in rec["message"] and rec["candidate"] == [16, 14, 2]
    assert rec["lattice_index"] == 0 and rec["initial_counts"] == [10, 10]
    cells = np.load(rec["cells"])
    assert cells.shape == (32, 32)


def test_tune_group_raises_on_a_candidate_that_differs(tmp_path, monkeypatch):
    monkeypatch.setenv("BML_DUMP_DIR", str(tmp_path))
    ref_counts = np.zeros((8, 4), np.uint32)
    ref_counts[:, 0] = ref_counts[:, 2] = 10
    reference = [(np.zeros((32, 32), np.uint8), ref_counts)]
    monkeypatch.setattr(FakeLattice, "cells_value", 1)     # one cell value off everywhere
    with pytest.raises(autotune.TuningMismatch):
        autotune.tune_group([(32, 0.3, 1)], 0, "fake", strip_rows=(16,), t_phases=(14,),
                            waves=(2,), steps=8, log=lambda m: None, reference=reference,
                            make_lattice=FakeLattice, step=fake_step)
    assert not os.listdir(tmp_path)
