"""``Lattice``: one BML lattice on the GPU -- torch-allocated state buffers,
stats ring and stream around a libbml handle."""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as B


class Lattice:
    """A periodic BML lattice resident in device memory: n x n, or n rows of
    `cols` cells.

    Cells start from SplitMix64 stream `seed` at density `rho` (LR and TB
    each with probability rho/2), or with LR / TB probabilities `rho_lr` /
    `rho_tb` when given (the asymmetric draw), or from `cells` (rows x cols
    bytes 0/1/2).
    """

    def __init__(self, n: int, rho: float = 0.3, seed: int = 0, *,
                 layout: int = B.BML_LAYOUT_U8, cells: np.ndarray | None = None,
                 stats_cap: int = 4096, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None, cols: int | None = None,
                 rho_lr: float | None = None, rho_tb: float | None = None):
        self.n = self.rows = int(n)
        self.cols = self.rows if cols is None else int(cols)
        self.layout = int(layout)
        self.device = torch.device(device)
        square = self.cols == self.rows and rho_lr is None and rho_tb is None
        nbytes = (B.bml_state_bytes(self.rows, self.layout) if square else
                  B.bml_state_bytes_rect(self.rows, self.cols, self.layout))
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._bufs = [torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                      for _ in range(2)]
        self.stats_cap = int(stats_cap)
        self._stats = torch.zeros(self.stats_cap * 4, dtype=torch.int32, device=self.device)
        # the ring's zero fill runs on the current stream; the library works
        # on self.stream, so the fill must be done before the first step
        torch.cuda.current_stream(self.device).synchronize()
        with torch.cuda.device(self.device):
            if square:
                self.handle = B.bml_init(self.rows, self.layout, seed, rho, cells,
                                         self._bufs[0], self._bufs[1], self._stats,
                                         self.stats_cap, self.stream)
            else:
                lr = rho / 2 if rho_lr is None else rho_lr
                tb = rho / 2 if rho_tb is None else rho_tb
                self.handle = B.bml_init_rect(self.rows, self.cols, self.layout, seed, lr, tb,
                                              cells, self._bufs[0], self._bufs[1], self._stats,
                                              self.stats_cap, self.stream)

    # -- ABI passthroughs -------------------------------------------------
    def step(self, n_steps: int = 1) -> None:
        B.bml_step(self.handle, n_steps)

    def stats(self, first_step: int | None = None, count: int | None = None,
              check: bool = True) -> np.ndarray:
        done = self.steps_done
        if count is None:
            count = min(done, self.stats_cap) if first_step is None else done - first_step
        if first_step is None:
            first_step = done - count
        return B.bml_stats(self.handle, first_step, count, check=check)

    def cells(self) -> np.ndarray:
        return B.bml_get_cells(self.handle, self.rows, self.cols)

    def set_tuning(self, tile_rows: int = -1, t_phases: int = 0,
                   waves_per_block: int = 0) -> None:
        B.bml_set_tuning(self.handle, tile_rows, t_phases, waves_per_block)

    def set_resident(self, steps: int) -> None:
        """0: the streaming step kernel; K (even, 2..32): the register-resident
        tile kernel, K steps per launch (Sec. 2's model on the torus or the
        Klein bottle, or Model III on the torus; rows a multiple of 32,
        columns a multiple of 256)."""
        B.bml_set_resident(self.handle, steps)

    @property
    def resident(self) -> int:
        return B.bml_get_resident(self.handle)

    def set_topology(self, topology: int) -> None:
        """BML_TOPO_TORUS (default) or BML_TOPO_KLEIN for the steps that follow."""
        B.bml_set_topology(self.handle, topology)

    def set_model(self, model: int, coin_seed: int = 0) -> None:
        """1: the model of Sec. 2 (default); 2: Model II with conflict coins
        from stream `coin_seed`; 3: Model III (a contested cell takes both
        cars, cell value 3)."""
        B.bml_set_model(self.handle, model, coin_seed)

    @property
    def model(self) -> int:
        return B.bml_get_model(self.handle)

    @property
    def topology(self) -> int:
        return B.bml_get_topology(self.handle)

    def tuning(self) -> tuple[int, int, int]:
        return B.bml_get_tuning(self.handle)

    def initial_counts(self) -> tuple[int, int]:
        return B.bml_initial_counts(self.handle)

    @property
    def steps_done(self) -> int:
        return B.bml_step_count(self.handle)

    def state_tensor(self) -> torch.Tensor:
        """The device buffer currently holding the state (uint8 view)."""
        ptr = B.bml_current_state(self.handle)
        return self._bufs[0] if ptr == self._bufs[0].data_ptr() else self._bufs[1]

    def close(self) -> None:
        if getattr(self, "handle", None):
            B.bml_free(self.handle)
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


def step_group(lattices, n_steps: int) -> None:
    """Advance lattices of one size, layout and tuning that share a stream
    by n_steps each, in joint launches (bml_step_group)."""
    B.bml_step_group([lat.handle for lat in lattices], n_steps)
