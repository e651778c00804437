"""ctypes declarations of the C ABI in include/bml.h (same names).

torch is imported before libbml.so is opened so that the library binds to
the HIP runtime torch already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the process's HIP runtime first)

BML_OK = 0
BML_EINVAL = -1
BML_EDEVICE = -2
BML_ERANGE = -3
BML_ESTATE = -4
BML_ECORRUPT = -5
BML_EBADARG = BML_EINVAL
BML_LAYOUT_U8 = 0
BML_LAYOUT_BITPLANE = 1
BML_TOPO_TORUS = 0
BML_TOPO_KLEIN = 1

# bml_step_stats as a numpy record: n_lr, moved_lr, n_tb, moved_tb.
STEP_STATS_DTYPE = np.dtype([("n_lr", "<u4"), ("moved_lr", "<u4"),
                             ("n_tb", "<u4"), ("moved_tb", "<u4")])

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libbml.so")


class BmlError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"libbml error {code}: {message}")
        self.code = code
        self.message = message


_lib = None

_i32, _i64, _u64, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
_vp, _sz = ctypes.c_void_p, ctypes.c_size_t

_SIGNATURES = {
    "bml_state_bytes": ([_i32, _i32, ctypes.POINTER(_sz)], ctypes.c_int),
    "bml_init": ([ctypes.POINTER(_vp), _i32, _i32, _u64, _dbl, _vp, _vp, _vp, _vp,
                  _i64, _vp], ctypes.c_int),
    "bml_state_bytes_rect": ([_i32, _i32, _i32, ctypes.POINTER(_sz)], ctypes.c_int),
    "bml_init_rect": ([ctypes.POINTER(_vp), _i32, _i32, _i32, _u64, _dbl, _dbl, _vp, _vp, _vp,
                       _vp, _i64, _vp], ctypes.c_int),
    "bml_step": ([_vp, _i64], ctypes.c_int),
    "bml_step_group": ([ctypes.POINTER(_vp), _i32, _i64], ctypes.c_int),
    "bml_step_group_static": ([_i32, _i32, _i32, _i32, ctypes.POINTER(_vp),
                               ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i64, _i64, _i64,
                               _i32, _vp, ctypes.POINTER(_i32)], ctypes.c_int),
    "bml_copy": ([_vp, _vp, _sz, _vp], ctypes.c_int),
    "bml_stats": ([_vp, _i64, _i64, _vp], ctypes.c_int),
    "bml_get_cells": ([_vp, _vp], ctypes.c_int),
    "bml_initial_counts": ([_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)], ctypes.c_int),
    "bml_set_tuning": ([_vp, _i32, _i32, _i32], ctypes.c_int),
    "bml_set_topology": ([_vp, _i32], ctypes.c_int),
    "bml_set_resident": ([_vp, _i32], ctypes.c_int),
    "bml_get_resident": ([_vp], ctypes.c_int),
    "bml_set_model": ([_vp, _i32, _u64], ctypes.c_int),
    "bml_get_topology": ([_vp], ctypes.c_int),
    "bml_get_model": ([_vp], ctypes.c_int),
    "bml_get_tuning": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                        ctypes.POINTER(_i32)], ctypes.c_int),
    "bml_step_count": ([_vp], _i64),
    "bml_current_state": ([_vp], _vp),
    "bml_free": ([_vp], None),
    "bml_last_error": ([], ctypes.c_char_p),
    "bml_pack": ([_i32, _vp, _vp, _vp], ctypes.c_int),
    "bml_unpack": ([_i32, _vp, _vp, _vp], ctypes.c_int),
    "bml_batch_arena_bytes": ([_i32, _vp, _i32, ctypes.POINTER(_sz)], ctypes.c_int),
    "bml_batch_init": ([ctypes.POINTER(_vp), _i32, _vp, _vp, _vp, _i32, _vp, _sz, _vp, _i64,
                        _vp], ctypes.c_int),
    "bml_batch_set_tuning": ([_vp, _i32, _i32, _i32], ctypes.c_int),
    "bml_batch_set_resident": ([_vp, _i32, _i32], ctypes.c_int),
    "bml_batch_get_resident": ([_vp], ctypes.c_int),
    "bml_batch_set_active": ([_vp, _vp], ctypes.c_int),
    "bml_batch_run": ([_vp, _i64], ctypes.c_int),
    "bml_batch_capture": ([_vp, _i64], ctypes.c_int),
    "bml_batch_replay": ([_vp], ctypes.c_int),
    "bml_batch_step_count": ([_vp], _i64),
    "bml_batch_lattice_steps": ([_vp, _i32, ctypes.POINTER(_i64)], ctypes.c_int),
    "bml_batch_initial_counts": ([_vp, _i32, ctypes.POINTER(_u64), ctypes.POINTER(_u64)],
                                 ctypes.c_int),
    "bml_batch_get_cells": ([_vp, _i32, _vp], ctypes.c_int),
    "bml_batch_check": ([_vp], ctypes.c_int),
    "bml_batch_free": ([_vp], None),
    "bml_features": ([_vp, _i64, _i32, _vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "bml_trace_frozen": ([_vp, _i64, _i32, _i64, _i64, _vp, _vp], ctypes.c_int),
    "bml_trace_mobility": ([_vp, _i64, _i32, _vp, _i64, _i64, _vp, _vp], ctypes.c_int),
    "bml_feature_stats": ([_vp, _i32, _vp, _vp, _vp], ctypes.c_int),
    "bml_standardize": ([_vp, _i32, _vp, _vp, _vp], ctypes.c_int),
    "bml_mlp_scratch_bytes": ([], _sz),
    "bml_mlp_grad": ([_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp], ctypes.c_int),
    "bml_mlp_train_step": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _i32, ctypes.c_float,
                            ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp, _vp, _vp],
                           ctypes.c_int),
    "bml_mlp_forward": ([_vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "bml_mlp_infer_bf16": ([_vp, _vp, _i32, _vp, _vp], ctypes.c_int),
}


def lib() -> ctypes.CDLL:
    """The loaded libbml.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise BmlError(BML_EDEVICE, f"{path} is missing: run "
                           "`python -m paper_1804_07981_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(path)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return sorted(_SIGNATURES)


def _check(rc: int) -> int:
    if rc < 0:
        raise BmlError(rc, bml_last_error())
    return rc


def _ptr(x) -> int | None:
    """Device or host address of a torch tensor / numpy array / int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def bml_last_error() -> str:
    msg = lib().bml_last_error()
    return msg.decode() if msg else ""


def bml_state_bytes(n: int, layout: int) -> int:
    out = _sz()
    _check(lib().bml_state_bytes(n, layout, ctypes.byref(out)))
    return int(out.value)


def bml_init(n: int, layout: int, seed: int, rho: float, cells_host, d_state_a,
             d_state_b, d_stats, stats_cap: int, stream) -> int:
    """Returns the opaque handle (an int)."""
    h = _vp()
    cells = None
    if cells_host is not None:
        cells = np.ascontiguousarray(cells_host, dtype=np.uint8)
        if cells.size != n * n:
            raise BmlError(BML_EINVAL, f"cells_host must hold {n}*{n} bytes")
    _check(lib().bml_init(ctypes.byref(h), n, layout, seed & (2**64 - 1), float(rho),
                          _ptr(cells), _ptr(d_state_a), _ptr(d_state_b), _ptr(d_stats),
                          stats_cap, _stream_ptr(stream)))
    return int(h.value)


def bml_state_bytes_rect(rows: int, cols: int, layout: int) -> int:
    out = _sz()
    _check(lib().bml_state_bytes_rect(rows, cols, layout, ctypes.byref(out)))
    return int(out.value)


def bml_init_rect(rows: int, cols: int, layout: int, seed: int, rho_lr: float, rho_tb: float,
                  cells_host, d_state_a, d_state_b, d_stats, stats_cap: int, stream) -> int:
    """Rectangular / asymmetric lattice; returns the opaque handle."""
    h = _vp()
    cells = None
    if cells_host is not None:
        cells = np.ascontiguousarray(cells_host, dtype=np.uint8)
        if cells.size != rows * cols:
            raise BmlError(BML_EINVAL, f"cells_host must hold {rows}*{cols} bytes")
    _check(lib().bml_init_rect(ctypes.byref(h), rows, cols, layout, seed & (2**64 - 1),
                               float(rho_lr), float(rho_tb), _ptr(cells), _ptr(d_state_a),
                               _ptr(d_state_b), _ptr(d_stats), stats_cap, _stream_ptr(stream)))
    return int(h.value)


def bml_set_topology(handle: int, topology: int) -> None:
    _check(lib().bml_set_topology(handle, topology))


def bml_set_resident(handle: int, steps: int) -> None:
    _check(lib().bml_set_resident(handle, steps))


def bml_get_resident(handle: int) -> int:
    return _check(lib().bml_get_resident(handle))


def bml_set_model(handle: int, model: int, coin_seed: int = 0) -> None:
    _check(lib().bml_set_model(handle, model, coin_seed & (2**64 - 1)))


def bml_get_topology(handle: int) -> int:
    return _check(lib().bml_get_topology(handle))


def bml_get_model(handle: int) -> int:
    return _check(lib().bml_get_model(handle))


def bml_step(handle: int, n_steps: int) -> None:
    _check(lib().bml_step(handle, n_steps))


def bml_copy(d_dst, d_src, nbytes: int, stream=None) -> None:
    """Streaming device copy (the bandwidth reference of the benchmarks)."""
    _check(lib().bml_copy(_ptr(d_dst), _ptr(d_src), nbytes, _stream_ptr(stream)))


def bml_step_group(handles, n_steps: int) -> None:
    """Advance several lattices (same size, layout, tuning and stream) in
    joint launches."""
    arr = (_vp * len(handles))(*[int(h) for h in handles])
    _check(lib().bml_step_group(arr, len(handles), n_steps))


def bml_step_group_static(rows: int, cols: int, layout: int, d_state_a, d_state_b, d_stats,
                          stats_cap: int, first_step: int, n_steps: int, t_phases: int,
                          stream=None) -> int:
    """Allocation-free stepping of len(d_state_a) lattices (lists of device
    buffers, one per lattice); returns 1 if the results are in the d_state_b
    buffers, 0 if in d_state_a."""
    count = len(d_state_a)
    if len(d_state_b) != count or len(d_stats) != count:
        raise BmlError(BML_EINVAL, "one state pair and one stats ring per lattice")
    arr = lambda xs: (_vp * count)(*[_ptr(x) for x in xs])  # noqa: E731
    out = _i32()
    _check(lib().bml_step_group_static(count, rows, cols, layout, arr(d_state_a), arr(d_state_b),
                                       arr(d_stats), stats_cap, first_step, n_steps, t_phases,
                                       _stream_ptr(stream), ctypes.byref(out)))
    return int(out.value)


def bml_stats(handle: int, first_step: int, count: int, check: bool = True) -> np.ndarray:
    """Counts of steps first_step .. first_step+count-1 as a STEP_STATS_DTYPE
    array.  With check=False a BML_ECORRUPT result is returned, not raised."""
    out = np.zeros(count, dtype=STEP_STATS_DTYPE)
    rc = lib().bml_stats(handle, first_step, count, out.ctypes.data)
    if rc < 0 and (check or rc != BML_ECORRUPT):
        raise BmlError(rc, bml_last_error())
    return out


def bml_get_cells(handle: int, n: int, cols: int | None = None) -> np.ndarray:
    out = np.empty((n, n if cols is None else cols), dtype=np.uint8)
    _check(lib().bml_get_cells(handle, out.ctypes.data))
    return out


def bml_initial_counts(handle: int) -> tuple[int, int]:
    a, b = _u64(), _u64()
    _check(lib().bml_initial_counts(handle, ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def bml_set_tuning(handle: int, tile_rows: int = -1, t_phases: int = 0,
                   waves_per_block: int = 0) -> None:
    _check(lib().bml_set_tuning(handle, tile_rows, t_phases, waves_per_block))


def bml_get_tuning(handle: int) -> tuple[int, int, int]:
    a, b, c = _i32(), _i32(), _i32()
    _check(lib().bml_get_tuning(handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def bml_step_count(handle: int) -> int:
    return int(lib().bml_step_count(handle))


def bml_current_state(handle: int) -> int:
    return int(lib().bml_current_state(handle) or 0)


def bml_free(handle: int) -> None:
    lib().bml_free(handle)


def bml_pack(n: int, d_cells, d_planes, stream=None) -> None:
    _check(lib().bml_pack(n, _ptr(d_cells), _ptr(d_planes), _stream_ptr(stream)))


def bml_unpack(n: int, d_planes, d_cells, stream=None) -> None:
    _check(lib().bml_unpack(n, _ptr(d_planes), _ptr(d_cells), _stream_ptr(stream)))


# --- batched sweeps -------------------------------------------------------

def bml_batch_arena_bytes(n_list, layout: int) -> int:
    n = np.ascontiguousarray(n_list, dtype=np.int32)
    out = _sz()
    _check(lib().bml_batch_arena_bytes(len(n), n.ctypes.data, layout, ctypes.byref(out)))
    return int(out.value)


def bml_batch_init(n_list, rho_list, seed_list, layout: int, d_arena, arena_bytes: int,
                   d_trace, trace_steps: int, stream) -> int:
    n = np.ascontiguousarray(n_list, dtype=np.int32)
    rho = np.ascontiguousarray(rho_list, dtype=np.float64)
    seed = np.ascontiguousarray([int(s) & (2**64 - 1) for s in seed_list], dtype=np.uint64)
    if not (len(n) == len(rho) == len(seed)):
        raise BmlError(BML_EINVAL, "n, rho and seed must have the same length")
    h = _vp()
    _check(lib().bml_batch_init(ctypes.byref(h), len(n), n.ctypes.data, rho.ctypes.data,
                                seed.ctypes.data, layout, _ptr(d_arena), arena_bytes,
                                _ptr(d_trace), trace_steps, _stream_ptr(stream)))
    return int(h.value)


def bml_batch_set_tuning(handle: int, strip_rows: int = 0, t_phases: int = 0,
                         waves_per_block: int = 0) -> None:
    _check(lib().bml_batch_set_tuning(handle, strip_rows, t_phases, waves_per_block))


def bml_batch_set_resident(handle: int, max_n: int, split_steps: int = 0) -> None:
    _check(lib().bml_batch_set_resident(handle, max_n, split_steps))


def bml_batch_get_resident(handle: int) -> int:
    return _check(lib().bml_batch_get_resident(handle))


def bml_batch_set_active(handle: int, active=None) -> None:
    a = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    _check(lib().bml_batch_set_active(handle, None if a is None else a.ctypes.data))


def bml_batch_run(handle: int, n_steps: int) -> None:
    _check(lib().bml_batch_run(handle, n_steps))


def bml_batch_capture(handle: int, n_steps: int) -> None:
    _check(lib().bml_batch_capture(handle, n_steps))


def bml_batch_replay(handle: int) -> None:
    _check(lib().bml_batch_replay(handle))


def bml_batch_step_count(handle: int) -> int:
    return int(lib().bml_batch_step_count(handle))


def bml_batch_lattice_steps(handle: int, idx: int) -> int:
    out = _i64()
    _check(lib().bml_batch_lattice_steps(handle, idx, ctypes.byref(out)))
    return int(out.value)


def bml_batch_initial_counts(handle: int, idx: int) -> tuple[int, int]:
    a, b = _u64(), _u64()
    _check(lib().bml_batch_initial_counts(handle, idx, ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def bml_batch_get_cells(handle: int, idx: int, n: int) -> np.ndarray:
    out = np.empty((n, n), dtype=np.uint8)
    _check(lib().bml_batch_get_cells(handle, idx, out.ctypes.data))
    return out


def bml_batch_check(handle: int) -> None:
    _check(lib().bml_batch_check(handle))


def bml_batch_free(handle: int) -> None:
    lib().bml_batch_free(handle)


# --- learned early exit -------------------------------------------------------

BML_MLP_INPUTS = 65
BML_MLP_HIDDEN = 64
BML_MLP_PARAMS = 8449
BML_MLP_MAX_BATCH = 256


def bml_features(d_trace, trace_steps: int, count: int, d_cars, d_rho, window: int, d_out,
                 stream=None) -> None:
    _check(lib().bml_features(_ptr(d_trace), trace_steps, count, _ptr(d_cars), _ptr(d_rho),
                              window, _ptr(d_out), _stream_ptr(stream)))


def bml_trace_frozen(d_trace, trace_steps: int, count: int, first_step: int, end_step: int,
                     d_frozen, stream=None) -> None:
    _check(lib().bml_trace_frozen(_ptr(d_trace), trace_steps, count, first_step, end_step,
                                  _ptr(d_frozen), _stream_ptr(stream)))


def bml_trace_mobility(d_trace, trace_steps: int, count: int, d_cars, first_step: int,
                       end_step: int, d_mean, stream=None) -> None:
    _check(lib().bml_trace_mobility(_ptr(d_trace), trace_steps, count, _ptr(d_cars),
                                    first_step, end_step, _ptr(d_mean), _stream_ptr(stream)))


def bml_feature_stats(d_x, n: int, d_mean, d_std, stream=None) -> None:
    _check(lib().bml_feature_stats(_ptr(d_x), n, _ptr(d_mean), _ptr(d_std), _stream_ptr(stream)))


def bml_standardize(d_x, n: int, d_mean, d_std, stream=None) -> None:
    _check(lib().bml_standardize(_ptr(d_x), n, _ptr(d_mean), _ptr(d_std), _stream_ptr(stream)))


def bml_mlp_scratch_bytes() -> int:
    return int(lib().bml_mlp_scratch_bytes())


def bml_mlp_grad(d_params, d_x, d_y, n: int, d_scratch, d_grad, d_loss, stream=None) -> None:
    _check(lib().bml_mlp_grad(_ptr(d_params), _ptr(d_x), _ptr(d_y), n, _ptr(d_scratch),
                              _ptr(d_grad), _ptr(d_loss), _stream_ptr(stream)))


def bml_mlp_train_step(d_params, d_m, d_v, d_grad, t: int, d_x, d_y, d_idx, n: int, lr: float,
                       beta1: float, beta2: float, eps: float, d_scratch, d_loss,
                       stream=None) -> None:
    _check(lib().bml_mlp_train_step(_ptr(d_params), _ptr(d_m), _ptr(d_v), _ptr(d_grad), t,
                                    _ptr(d_x), _ptr(d_y), _ptr(d_idx), n, lr, beta1, beta2, eps,
                                    _ptr(d_scratch), _ptr(d_loss), _stream_ptr(stream)))


def bml_mlp_forward(d_params, d_x, n: int, d_logits, stream=None) -> None:
    _check(lib().bml_mlp_forward(_ptr(d_params), _ptr(d_x), n, _ptr(d_logits),
                                 _stream_ptr(stream)))


def bml_mlp_infer_bf16(d_params, d_x, n: int, d_logits, stream=None) -> None:
    _check(lib().bml_mlp_infer_bf16(_ptr(d_params), _ptr(d_x), n, _ptr(d_logits),
                                    _stream_ptr(stream)))
