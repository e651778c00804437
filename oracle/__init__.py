"""CPU oracle for the Biham-Middleton-Levine (BML) Model I automaton.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The product
library (``paper_1804_07981_amd``) never imports it, and it never imports the
product: the two share no code.

The lattice arithmetic lives in ``bml_oracle.c`` (plain C, optional OpenMP
row split as in the paper's Sec. 4); this module builds it with gcc, loads it
with ctypes and wraps it for numpy arrays.  ``mlp.py`` holds the fp64 oracle
of the learned early-exit classifier (trace features, labels, network,
gradient, Adam and BF16 inference).

Paper: M. Marzolla, "Parallel Implementations of Cellular Automata for
Traffic Models", arXiv:1804.07981 (Sec. 2 model and case tables, Sec. 3
serial update, Sec. 4 OpenMP row split).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

EMPTY, LR, TB = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bml_oracle.c")
_LIB_PATH = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(_HERE, "liboracle.so")
# Plain -O3, no target-specific flags: the library is built once and may run
# on a different host CPU than the one that compiled it.
CFLAGS = ["-O3", "-std=c11", "-fopenmp", "-shared", "-fPIC"]


def build(extra_flags: list[str] | None = None, out: str | None = None) -> str:
    """Compile bml_oracle.c into liboracle.so (always recompiles)."""
    out = out or _LIB_PATH
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), "-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, u64, i32, dbl, vp = (ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_void_p)
        L.bmlo_splitmix64.argtypes = [u64, u64]
        L.bmlo_splitmix64.restype = u64
        L.bmlo_thresholds.argtypes = [dbl, vp, vp]
        L.bmlo_thresholds.restype = None
        L.bmlo_init_cells.argtypes = [i64, i64, u64, dbl, vp]
        L.bmlo_init_cells.restype = None
        L.bmlo_thresholds_asym.argtypes = [dbl, dbl, vp, vp]
        L.bmlo_thresholds_asym.restype = None
        L.bmlo_init_cells_asym.argtypes = [i64, i64, u64, dbl, dbl, vp]
        L.bmlo_init_cells_asym.restype = None
        L.bmlo_phase_h.argtypes = [i64, i64, vp, vp]
        L.bmlo_phase_h.restype = i64
        L.bmlo_phase_v.argtypes = [i64, i64, vp, vp]
        L.bmlo_phase_v.restype = i64
        L.bmlo_count.argtypes = [vp, i64, i32]
        L.bmlo_count.restype = i64
        L.bmlo_run.argtypes = [i64, i64, vp, vp, i64, vp, i32]
        L.bmlo_run.restype = None
        L.bmlo_run_topo.argtypes = [i64, i64, vp, vp, i64, vp, i32, i32]
        L.bmlo_run_topo.restype = None
        L.bmlo_run_model2.argtypes = [i64, i64, vp, vp, i64, i64, u64, vp, i32, i64, i64, i64, i64]
        L.bmlo_run_model2.restype = None
        L.bmlo_run_model3.argtypes = [i64, i64, vp, vp, i64, vp, i32]
        L.bmlo_run_model3.restype = None
        L.bmlo_phase_v_topo.argtypes = [i64, i64, vp, vp, i32]
        L.bmlo_phase_v_topo.restype = i64
        L.bmlo_run_many.argtypes = [i64, vp, vp, vp, vp, vp, i64, i32]
        L.bmlo_run_many.restype = i32
        L.bmlo_pack.argtypes = [i64, i64, vp, vp, vp]
        L.bmlo_pack.restype = None
        L.bmlo_unpack.argtypes = [i64, i64, vp, vp, vp]
        L.bmlo_unpack.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _u8(cells: np.ndarray, allow_both: bool = False) -> np.ndarray:
    a = np.ascontiguousarray(cells, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError("lattice must be 2-D")
    if a.size and int(a.max()) > (3 if allow_both else 2):
        raise ValueError("cell values must be 0..2 (0..3 under Model III)")
    return a


def splitmix64(seed: int, k: int) -> int:
    """k-th output of the SplitMix64 stream started at state `seed`."""
    return int(lib().bmlo_splitmix64(seed & (2**64 - 1), k))


def thresholds(rho: float) -> tuple[int, int]:
    a = ctypes.c_uint64()
    b = ctypes.c_uint64()
    lib().bmlo_thresholds(float(rho), ctypes.byref(a), ctypes.byref(b))
    return int(a.value), int(b.value)


def init_cells(n: int, seed: int, rho: float, cols: int | None = None) -> np.ndarray:
    """Random initial lattice: cell i*cols+j from the (i*cols+j)-th SplitMix64
    output of stream `seed`; LR w.p. rho/2, TB w.p. rho/2, else EMPTY."""
    cols = n if cols is None else cols
    out = np.empty((n, cols), dtype=np.uint8)
    lib().bmlo_init_cells(n, cols, seed & (2**64 - 1), float(rho), _ptr(out))
    return out


def thresholds_asym(rho_lr: float, rho_tb: float) -> tuple[int, int]:
    a = ctypes.c_uint64()
    b = ctypes.c_uint64()
    lib().bmlo_thresholds_asym(float(rho_lr), float(rho_tb), ctypes.byref(a), ctypes.byref(b))
    return int(a.value), int(b.value)


def init_cells_asym(rows: int, cols: int, seed: int, rho_lr: float, rho_tb: float
                    ) -> np.ndarray:
    """Asymmetric random lattice (Sec. 2's unequal LR/TB numbers): cell
    i*cols+j is LR w.p. rho_lr, TB w.p. rho_tb, else EMPTY, from the same
    SplitMix64 draw as init_cells."""
    out = np.empty((rows, cols), dtype=np.uint8)
    lib().bmlo_init_cells_asym(rows, cols, seed & (2**64 - 1), float(rho_lr), float(rho_tb),
                               _ptr(out))
    return out


def phase_h(cells: np.ndarray) -> tuple[np.ndarray, int]:
    """One horizontal phase (Sec. 2 case table); returns (new lattice, moved)."""
    a = _u8(cells)
    out = np.empty_like(a)
    moved = lib().bmlo_phase_h(a.shape[0], a.shape[1], _ptr(a), _ptr(out))
    return out, int(moved)


def phase_v(cells: np.ndarray) -> tuple[np.ndarray, int]:
    """One vertical phase (Sec. 2 case table); returns (new lattice, moved)."""
    a = _u8(cells)
    out = np.empty_like(a)
    moved = lib().bmlo_phase_v(a.shape[0], a.shape[1], _ptr(a), _ptr(out))
    return out, int(moved)


TORUS, KLEIN = 0, 1


def run(cells: np.ndarray, steps: int, n_threads: int = 1, topology: int = TORUS
        ) -> tuple[np.ndarray, np.ndarray]:
    """`steps` steps (H then V each).  Returns (final lattice, stats) with
    stats[s] = (n_lr, moved_lr, n_tb, moved_tb) of step s.  topology KLEIN
    glues the top and bottom edges with a reversal (Klein bottle)."""
    a = _u8(cells).copy()
    tmp = np.empty_like(a)
    stats = np.zeros((max(steps, 0), 4), dtype=np.uint32)
    lib().bmlo_run_topo(a.shape[0], a.shape[1], _ptr(a), _ptr(tmp), int(steps),
                        _ptr(stats), int(n_threads), int(topology))
    return a, stats


def run_model2(cells: np.ndarray, steps: int, coin_seed: int, step0: int = 0,
               n_threads: int = 1, frame: tuple[int, int, int, int] | None = None
               ) -> tuple[np.ndarray, np.ndarray]:
    """Model II (Sec. 2): both car types move in one phase per step; a
    contested empty cell goes to the LR car when the step's counter-based
    coin for that cell is 1 (bit j%32 of SplitMix64 output
    step*rows*W + i*W + j//32 of stream coin_seed, W = ceil(cols/32)).
    step0 is the global index of the first step (it selects the coins).
    frame = (row0, col0, rows_g, cols_g) runs `cells` as the window at
    (row0, col0) of a rows_g x cols_g lattice: every cell draws the coin of
    its position there (the window itself stays periodic, so only cells
    farther than `steps` from its edges match the large lattice's run).
    Parity unpinned against the paper, which gives no Model II values; the
    coin is a reading and the tests pin it."""
    a = _u8(cells).copy()
    tmp = np.empty_like(a)
    stats = np.zeros((max(steps, 0), 4), dtype=np.uint32)
    row0, col0, rows_g, cols_g = frame or (0, 0, a.shape[0], a.shape[1])
    if not (0 <= row0 < rows_g and 0 <= col0 < cols_g):
        raise ValueError("window origin outside the lattice")
    lib().bmlo_run_model2(a.shape[0], a.shape[1], _ptr(a), _ptr(tmp), int(steps), int(step0),
                          coin_seed & (2**64 - 1), _ptr(stats), int(n_threads), int(row0),
                          int(col0), int(rows_g), int(cols_g))
    return a, stats


def run_model3(cells: np.ndarray, steps: int, n_threads: int = 1
               ) -> tuple[np.ndarray, np.ndarray]:
    """Model III (Sec. 2), read as Model II's one-phase update in which an
    EMPTY cell wanted by an LR and a TB car takes both (value 3 = LR | TB);
    any car in a cell blocks cars of either type.  Cells hold 0..3.
    Parity unpinned against the paper (one sentence on Model III): the tests
    pin this reading, not the paper's numbers."""
    a = _u8(cells, allow_both=True).copy()
    tmp = np.empty_like(a)
    stats = np.zeros((max(steps, 0), 4), dtype=np.uint32)
    lib().bmlo_run_model3(a.shape[0], a.shape[1], _ptr(a), _ptr(tmp), int(steps), _ptr(stats),
                          int(n_threads))
    return a, stats


def phase_v_topo(cells: np.ndarray, topology: int) -> tuple[np.ndarray, int]:
    a = _u8(cells)
    out = np.empty_like(a)
    moved = lib().bmlo_phase_v_topo(a.shape[0], a.shape[1], _ptr(a), _ptr(out), int(topology))
    return out, int(moved)


def run_many(lattices: list[np.ndarray], steps: int, n_threads: int = 1
             ) -> tuple[list[np.ndarray], list[np.ndarray]]:
    """Run independent square lattices, one lattice per thread."""
    sizes = np.array([l.shape[0] for l in lattices], dtype=np.int64)
    for l in lattices:
        if l.ndim != 2 or l.shape[0] != l.shape[1]:
            raise ValueError("run_many takes square lattices")
    offsets = np.zeros(len(lattices), dtype=np.int64)
    offsets[1:] = np.cumsum(sizes * sizes)[:-1]
    buf = np.concatenate([np.ascontiguousarray(l, dtype=np.uint8).ravel()
                          for l in lattices]) if lattices else np.zeros(0, np.uint8)
    stats = np.zeros((len(lattices), max(steps, 0), 4), dtype=np.uint32)
    soff = np.arange(len(lattices), dtype=np.int64) * max(steps, 0) * 4
    rc = lib().bmlo_run_many(len(lattices), _ptr(sizes), _ptr(offsets),
                             _ptr(buf), _ptr(soff), _ptr(stats), int(steps),
                             int(n_threads))
    if rc != 0:
        raise MemoryError("oracle run_many could not allocate scratch")
    outs = [buf[o:o + n * n].reshape(n, n).copy() for o, n in zip(offsets, sizes)]
    return outs, [stats[b] for b in range(len(lattices))]


def pack(cells: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """uint8 lattice -> (LR plane, TB plane), rows x cols/32 uint32 each."""
    a = _u8(cells)
    if a.shape[1] % 32:
        raise ValueError("cols must be a multiple of 32")
    lr = np.empty((a.shape[0], a.shape[1] // 32), dtype=np.uint32)
    tb = np.empty_like(lr)
    lib().bmlo_pack(a.shape[0], a.shape[1], _ptr(a), _ptr(lr), _ptr(tb))
    return lr, tb


def unpack(lr: np.ndarray, tb: np.ndarray) -> np.ndarray:
    lr = np.ascontiguousarray(lr, dtype=np.uint32)
    tb = np.ascontiguousarray(tb, dtype=np.uint32)
    rows, words = lr.shape
    out = np.empty((rows, words * 32), dtype=np.uint8)
    lib().bmlo_unpack(rows, words * 32, _ptr(lr), _ptr(tb), _ptr(out))
    return out


def count(cells: np.ndarray, value: int) -> int:
    a = _u8(cells)
    return int(lib().bmlo_count(_ptr(a), a.size, int(value)))
