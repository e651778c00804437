"""Python binding of libbml, the MI355X (gfx950) Biham-Middleton-Levine
step library (M. Marzolla, "Parallel Implementations of Cellular Automata for
Traffic Models", arXiv:1804.07981).

Only argument marshalling lives here: every function of ``include/bml.h`` is
exposed under the same name and every step of the automaton runs in the HIP
kernels of ``libbml.so``.  PyTorch provides device memory and streams; the
``Lattice`` class bundles those buffers with a handle.  There is no CPU
fallback: if the library or a GPU is missing, calls raise.
"""
from __future__ import annotations

from ._lib import (BML_EBADARG, BML_ECORRUPT, BML_EDEVICE, BML_EINVAL,
                   BML_ERANGE, BML_ESTATE, BML_LAYOUT_BITPLANE, BML_LAYOUT_U8,
                   BML_OK, STEP_STATS_DTYPE, BmlError, bml_current_state,
                   bml_free, bml_get_cells, bml_get_tuning, bml_init,
                   bml_initial_counts, bml_last_error, bml_pack, bml_set_tuning,
                   bml_state_bytes, bml_stats, bml_step, bml_step_count,
                   bml_unpack, exported_symbols, lib, library_path)
from .lattice import Lattice

__all__ = [
    "BML_OK", "BML_EINVAL", "BML_EDEVICE", "BML_ERANGE", "BML_ESTATE",
    "BML_ECORRUPT", "BML_EBADARG", "BML_LAYOUT_U8", "BML_LAYOUT_BITPLANE",
    "STEP_STATS_DTYPE", "BmlError", "Lattice", "lib", "library_path",
    "exported_symbols", "bml_state_bytes", "bml_init", "bml_step", "bml_stats",
    "bml_get_cells", "bml_initial_counts", "bml_set_tuning", "bml_get_tuning",
    "bml_step_count", "bml_current_state", "bml_free", "bml_last_error",
    "bml_pack", "bml_unpack",
]
