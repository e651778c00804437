"""``Batch``: many BML lattices advanced together on the GPU (torch-allocated
arena, trace and stream around a libbml batch handle)."""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as B


class Batch:
    """Lattices b = 0..count-1 of side n[b], density rho[b], SplitMix64 stream
    seed[b].  `trace()` gives, per lattice and global step, the number of LR
    and TB cars that moved."""

    def __init__(self, n, rho, seed, *, layout: int = B.BML_LAYOUT_BITPLANE,
                 trace_steps: int = 4096, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None):
        self.n = [int(x) for x in n]
        self.count = len(self.n)
        self.layout = int(layout)
        self.device = torch.device(device)
        self.trace_steps = int(trace_steps)
        self.stream = stream or torch.cuda.Stream(self.device)
        self.arena_bytes = B.bml_batch_arena_bytes(self.n, self.layout)
        self._arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=self.device)
        self._trace = torch.zeros(self.count * self.trace_steps * 2, dtype=torch.int32,
                                  device=self.device)
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            self.handle = B.bml_batch_init(self.n, rho, seed, self.layout, self._arena,
                                           self.arena_bytes, self._trace, self.trace_steps,
                                           self.stream)

    def set_tuning(self, strip_rows: int = 0, t_phases: int = 0, waves_per_block: int = 0):
        B.bml_batch_set_tuning(self.handle, strip_rows, t_phases, waves_per_block)

    def set_resident(self, max_n: int, split_steps: int = 0):
        """Register-resident runs when every lattice has N <= max_n (at most
        1024; 0 = always the streaming kernel); lattices taller than 512 rows
        are cut into slabs with split_steps halo rows (0 = 64), and launches
        then run at most that many steps."""
        B.bml_batch_set_resident(self.handle, max_n, split_steps)

    @property
    def resident(self) -> bool:
        return B.bml_batch_get_resident(self.handle) == 1

    def set_active(self, active=None):
        B.bml_batch_set_active(self.handle, active)

    def run(self, n_steps: int):
        B.bml_batch_run(self.handle, n_steps)

    def capture(self, n_steps: int):
        B.bml_batch_capture(self.handle, n_steps)

    def replay(self):
        B.bml_batch_replay(self.handle)

    def synchronize(self):
        self.stream.synchronize()

    @property
    def steps_done(self) -> int:
        return B.bml_batch_step_count(self.handle)

    def lattice_steps(self, idx: int) -> int:
        return B.bml_batch_lattice_steps(self.handle, idx)

    def initial_counts(self, idx: int) -> tuple[int, int]:
        return B.bml_batch_initial_counts(self.handle, idx)

    def cells(self, idx: int) -> np.ndarray:
        return B.bml_batch_get_cells(self.handle, idx, self.n[idx])

    def check(self) -> None:
        B.bml_batch_check(self.handle)

    def trace(self) -> np.ndarray:
        """(count, trace_steps, 2) uint32: LR moved, TB moved per step."""
        self.synchronize()
        return self._trace.cpu().numpy().view(np.uint32).reshape(
            self.count, self.trace_steps, 2)

    def trace_tensor(self) -> torch.Tensor:
        return self._trace.view(self.count, self.trace_steps, 2)

    def close(self):
        if getattr(self, "handle", None):
            B.bml_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
