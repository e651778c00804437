"""CPU-only checks of the C ABI library: it loads, exports every function
include/bml.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bml.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bml_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def B():
    pkg = pytest.importorskip("paper_1804_07981_amd")
    if not os.path.exists(pkg.library_path()):
        pytest.skip("libbml.so not built")
    return pkg


def test_header_declares_core_entry_points():
    names = declared_functions()
    for n in ("bml_init", "bml_step", "bml_stats", "bml_get_cells", "bml_free",
              "bml_last_error", "bml_state_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol(B):
    lib = ctypes.CDLL(B.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(B):
    assert set(declared_functions()) <= set(B.exported_symbols())


@pytest.mark.parametrize("n,layout,want", [
    (32, 0, 32 * 32), (64, 1, 64 * 64 // 4), (65504, 0, 65504 * 65504),
    (4096, 1, 4096 * 4096 // 4)])
def test_state_bytes(B, n, layout, want):
    assert B.bml_state_bytes(n, layout) == want


@pytest.mark.parametrize("n,layout", [(0, 0), (31, 0), (48, 0), (65536, 0), (64, 2), (-32, 1)])
def test_state_bytes_rejects(B, n, layout):
    with pytest.raises(B.BmlError) as e:
        B.bml_state_bytes(n, layout)
    assert e.value.code == B.BML_EINVAL
    assert B.bml_last_error()


def test_null_handle_is_estate(B):
    lib = B.lib()
    assert lib.bml_step(None, 1) == B.BML_ESTATE
    assert lib.bml_step_count(None) == -1
    assert lib.bml_current_state(None) is None
    lib.bml_free(None)   # ignored


def test_init_rejects_bad_arguments_without_gpu(B):
    lib = B.lib()
    h = ctypes.c_void_p()
    # NULL buffers are rejected before any device call.
    assert lib.bml_init(ctypes.byref(h), 64, 0, 0, 0.3, None, None, None, None, 16, None) \
        == B.BML_EINVAL
    assert lib.bml_init(None, 64, 0, 0, 0.3, None, None, None, None, 16, None) == B.BML_EINVAL
    assert lib.bml_init(ctypes.byref(h), 33, 0, 0, 0.3, None, 256, 512, 1024, 16, None) \
        == B.BML_EINVAL
    # Misaligned buffers.
    assert lib.bml_init(ctypes.byref(h), 64, 0, 0, 0.3, None, 257, 1 << 20, 1 << 21, 16, None) \
        == B.BML_EINVAL
    # Overlapping state buffers.
    assert lib.bml_init(ctypes.byref(h), 64, 0, 0, 0.3, None, 1 << 20, (1 << 20) + 256,
                        1 << 22, 16, None) == B.BML_EINVAL
    # rho out of range, stats_cap out of range.
    assert lib.bml_init(ctypes.byref(h), 64, 0, 0, 1.5, None, 1 << 20, 1 << 21, 1 << 22, 16,
                        None) == B.BML_EINVAL
    assert lib.bml_init(ctypes.byref(h), 64, 0, 0, float("nan"), None, 1 << 20, 1 << 21,
                        1 << 22, 16, None) == B.BML_EINVAL
    assert lib.bml_init(ctypes.byref(h), 64, 0, 0, 0.3, None, 1 << 20, 1 << 21, 1 << 22, 0,
                        None) == B.BML_EINVAL


def test_init_rejects_bad_cell_values_without_gpu(B):
    import numpy as np
    lib = B.lib()
    h = ctypes.c_void_p()
    cells = np.zeros(64 * 64, dtype=np.uint8)
    cells[100] = 4          # 0..2, and 3 (both cars, Model III) are the cell values
    rc = lib.bml_init(ctypes.byref(h), 64, 0, 0, 0.3, cells.ctypes.data, 1 << 20, 1 << 21,
                      1 << 22, 16, None)
    assert rc == B.BML_EINVAL and "value 4" in B.bml_last_error()


def test_step_group_rejects_bad_arguments_without_gpu(B):
    lib = ctypes.CDLL(B.library_path())
    lib.bml_step_group.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                   ctypes.c_int64]
    arr = (ctypes.c_void_p * 9)()
    assert lib.bml_step_group(None, 1, 1) == B.BML_EINVAL
    assert lib.bml_step_group(arr, 0, 1) == B.BML_EINVAL
    assert lib.bml_step_group(arr, 9, 1) == B.BML_EINVAL      # more than 8 lattices
    assert lib.bml_step_group(arr, 2, 1) == B.BML_ESTATE      # NULL handles


def test_copy_rejects_bad_arguments_without_gpu(B):
    lib = ctypes.CDLL(B.library_path())
    lib.bml_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    assert lib.bml_copy(None, None, 16, None) == B.BML_EINVAL
    assert lib.bml_copy(256, 512, 8, None) == B.BML_EINVAL          # not a multiple of 16
    assert lib.bml_copy(256 + 16, 4096, 16, None) == B.BML_EINVAL   # misaligned
    assert lib.bml_copy(4096, 4096 + 256, 512, None) == B.BML_EINVAL  # overlapping


@pytest.mark.parametrize("rows,cols,layout", [(31, 64, 0), (64, 48, 0), (65505, 32, 1),
                                              (64, 65536, 0), (64, 64, 2)])
def test_state_bytes_rect_rejects(B, rows, cols, layout):
    with pytest.raises(B.BmlError) as e:
        B.bml_state_bytes_rect(rows, cols, layout)
    assert e.value.code == B.BML_EINVAL


def test_state_bytes_rect(B):
    assert B.bml_state_bytes_rect(33, 4096, 0) == 33 * 4096
    assert B.bml_state_bytes_rect(33, 4096, 1) == 33 * 4096 // 4
    assert B.bml_state_bytes_rect(64, 64, 1) == B.bml_state_bytes(64, 1)


def test_init_rect_rejects_bad_densities_without_gpu(B):
    lib = B.lib()
    h = ctypes.c_void_p()
    for lr, tb in ((-0.1, 0.2), (0.6, 0.5), (float("nan"), 0.1), (0.1, float("nan"))):
        rc = lib.bml_init_rect(ctypes.byref(h), 64, 64, 0, 1, lr, tb, None, 256, 512 * 1024,
                               1024 * 1024, 8, None)
        assert rc == B.BML_EINVAL, (lr, tb)


def test_topology_calls_reject_null_handle(B):
    lib = B.lib()
    assert lib.bml_set_topology(None, 1) == B.BML_ESTATE
    assert lib.bml_get_topology(None) == B.BML_ESTATE


def test_set_model_rejects_null_handle(B):
    lib = B.lib()
    assert lib.bml_set_model(None, 2, 7) == B.BML_ESTATE
    assert lib.bml_set_model(None, 1, 0) == B.BML_ESTATE


def test_set_model_three_rejects_null_handle(B):
    assert B.lib().bml_set_model(None, 3, 0) == B.BML_ESTATE
    assert B.lib().bml_get_model(None) == B.BML_ESTATE
