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
                   bml_state_bytes, bml_state_bytes_rect, bml_init_rect, bml_stats,
                   bml_set_topology, bml_get_topology, BML_TOPO_TORUS, BML_TOPO_KLEIN,
                   bml_set_resident, bml_get_resident,
                   bml_set_model, bml_get_model, bml_step, bml_step_count, bml_step_group, bml_copy,
                   bml_step_group_static,
                   bml_unpack, exported_symbols, lib, library_path,
                   bml_batch_arena_bytes, bml_batch_init, bml_batch_set_tuning,
                   bml_batch_set_active, bml_batch_set_resident, bml_batch_get_resident,
                   bml_batch_run, bml_batch_capture,
                   bml_batch_replay, bml_batch_step_count, bml_batch_lattice_steps,
                   bml_batch_initial_counts, bml_batch_get_cells, bml_batch_check,
                   bml_batch_free, bml_features, bml_trace_frozen, bml_trace_mobility,
                   bml_feature_stats, bml_standardize, bml_mlp_scratch_bytes,
                   bml_mlp_grad, bml_mlp_train_step, bml_mlp_forward, bml_mlp_infer_bf16,
                   BML_MLP_INPUTS, BML_MLP_HIDDEN, BML_MLP_PARAMS, BML_MLP_MAX_BATCH)
from .batch import Batch
from .lattice import Lattice, step_group

__all__ = [
    "BML_OK", "BML_EINVAL", "BML_EDEVICE", "BML_ERANGE", "BML_ESTATE",
    "BML_ECORRUPT", "BML_EBADARG", "BML_LAYOUT_U8", "BML_LAYOUT_BITPLANE",
    "STEP_STATS_DTYPE", "BmlError", "Lattice", "lib", "library_path",
    "exported_symbols", "bml_state_bytes", "bml_init", "bml_step", "bml_stats",
    "bml_step_group", "step_group", "bml_step_group_static", "bml_copy", "bml_state_bytes_rect", "bml_init_rect",
    "bml_set_topology", "bml_get_topology", "BML_TOPO_TORUS", "BML_TOPO_KLEIN",
    "bml_set_resident", "bml_get_resident",
    "bml_set_model", "bml_get_model",
    "bml_get_cells", "bml_initial_counts", "bml_set_tuning", "bml_get_tuning",
    "bml_step_count", "bml_current_state", "bml_free", "bml_last_error",
    "bml_pack", "bml_unpack", "Batch", "bml_batch_arena_bytes", "bml_batch_init",
    "bml_batch_set_tuning", "bml_batch_set_active", "bml_batch_set_resident",
    "bml_batch_get_resident", "bml_batch_run", "bml_batch_capture",
    "bml_batch_replay", "bml_batch_step_count", "bml_batch_lattice_steps",
    "bml_batch_initial_counts", "bml_batch_get_cells", "bml_batch_check", "bml_batch_free",
    "bml_features", "bml_trace_frozen", "bml_trace_mobility", "bml_feature_stats",
    "bml_standardize", "bml_mlp_scratch_bytes", "bml_mlp_grad", "bml_mlp_train_step",
    "bml_mlp_forward", "bml_mlp_infer_bf16", "BML_MLP_INPUTS", "BML_MLP_HIDDEN",
    "BML_MLP_PARAMS", "BML_MLP_MAX_BATCH",
]
