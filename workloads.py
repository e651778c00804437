"""Seeded synthetic inputs for the BML lattices: workload definitions and
parameter draws, shared by the tests, the benchmark and the examples.

This module holds no automaton arithmetic.  It only says WHICH lattices are
run (sizes, densities, seeds, step counts) and builds a few hand-made
lattices.  The random initial cells themselves are drawn by each
implementation from its own SplitMix64 (cell k of a lattice with seed s is
the k-th output of the stream started at state s); this module only draws
the per-lattice sizes and densities of the sweeps, from a SplitMix64 stream
of its own.

The paper's own workload (Marzolla, arXiv:1804.07981, Sec. 6) is random
lattices of density rho = 0.3, N in {1024, 2048, 4096}, 1024 steps; Fig. 1
uses 256 x 256 lattices at rho = 0.25 / 0.32 / 0.38.  The configurations
below keep that shape of workload and add the sweep cases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

EMPTY, LR, TB = 0, 1, 2
_MASK64 = (1 << 64) - 1


def _splitmix64_stream(state: int, count: int) -> list[int]:
    """First `count` outputs of SplitMix64 started at `state` (Vigna's
    public-domain generator: state += golden gamma; output = finaliser)."""
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out.append(z ^ (z >> 31))
    return out


def _unit(z: int) -> float:
    """53-bit uniform in [0, 1) from a 64-bit output."""
    return (z >> 11) * (1.0 / (1 << 53))


@dataclass(frozen=True)
class Lattice:
    n: int                       # rows (and columns unless `cols` is set)
    rho: float
    seed: int
    cols: int | None = None      # rectangular lattices: columns
    rho_lr: float | None = None  # asymmetric draw: LR / TB probabilities
    rho_tb: float | None = None

    @property
    def cells(self) -> int:
        return self.n * (self.cols or self.n)

    def kwargs(self) -> dict:
        """Keyword arguments of the library's Lattice for this shape and draw."""
        if self.cols is None and self.rho_lr is None:
            return {}
        return {"cols": self.cols or self.n, "rho_lr": self.rho_lr, "rho_tb": self.rho_tb}


@dataclass(frozen=True)
class Workload:
    name: str
    lattices: tuple
    steps: int
    description: str


# Small parity case: 256 x 256, rho 0.30, seed 0, 1024 steps.
SMALL = Workload(
    "bml-256-rho0.30-seed0-1024steps",
    (Lattice(256, 0.30, 0),), 1024,
    "single 256x256 lattice, every cell and count checked after every step")

# Headline single-lattice workload: 4096 x 4096 at four densities, seed k for
# the k-th density, 10000 steps each.
DENSITIES_4096 = (0.25, 0.35, 0.38, 0.45)
MEDIUM = Workload(
    "bml-4096x4096-rho{0.25,0.35,0.38,0.45}-seeds1-4-10000steps",
    tuple(Lattice(4096, r, k + 1) for k, r in enumerate(DENSITIES_4096)),
    10000,
    "four 4096x4096 lattices, uint8 and 2-bitplane forms")
# Tuning-cache name of the four lattices advanced together by joint launches.
MEDIUM_GROUP = "medium4"

# Large single lattice: 32768 x 32768 (1 GiB of uint8 cells), rho 0.30,
# seed 7, 1000 steps.
LARGE = Workload(
    "bml-32768x32768-rho0.30-seed7-1000steps",
    (Lattice(32768, 0.30, 7),), 1000,
    "single lattice far larger than any on-chip cache")


# Rectangular lattice with unequal densities (Sec. 2's asymmetric
# extension): 8192 rows x 32768 columns (256 MiB of uint8 cells), LR 0.20,
# TB 0.10, seed 11, 1000 steps.
RECT = Workload(
    "bml-8192x32768-lr0.20-tb0.10-seed11-1000steps",
    (Lattice(8192, 0.30, 11, cols=32768, rho_lr=0.20, rho_tb=0.10),), 1000,
    "rectangular lattice, unequal LR / TB densities")


SWEEP_STREAM_STATE = 0x5EEDBA7C


def sweep_lattices(count: int = 512, state: int = SWEEP_STREAM_STATE
                   ) -> list[Lattice]:
    """Batched density sweep: lattice L has N log-uniform in [64, 1024]
    rounded to a multiple of 32 and rho uniform in [0.20, 0.50], drawn from
    outputs 2L and 2L+1 of a SplitMix64 stream; its cells use seed L."""
    zs = _splitmix64_stream(state, 2 * count)
    out = []
    for L in range(count):
        ua, ub = _unit(zs[2 * L]), _unit(zs[2 * L + 1])
        n = 32 * int(math.floor(math.exp(math.log(64.0) + ua * math.log(16.0)) / 32.0 + 0.5))
        rho = 0.20 + 0.30 * ub
        out.append(Lattice(n, rho, L))
    return out


SWEEP = Workload("bml-sweep-512-lattices-N64..1024-4096steps",
                 tuple(sweep_lattices()), 4096,
                 "512 lattices of uneven N and rho in one launch")

# Early-exit sweep: 512 x 512, rho_k = (80 + k) / 400 for k = 0..140
# (0.2000 .. 0.5500 step 0.0025), 64 seeds each, seed = 64 k + s.
EE_N = 512
EE_RHO_COUNT = 141
EE_SEEDS = 64
EE_FULL_STEPS = 20000
EE_EXIT_STEP = 512
EE_HELD_OUT = range(51, 64)      # seeds s = 51..63 of every rho: test split
EE_VALIDATION = range(46, 51)    # seeds s = 46..50: validation split


def early_exit_lattices() -> list[tuple[Lattice, int, int]]:
    """(lattice, k, s) for every rho index k and seed index s."""
    out = []
    for k in range(EE_RHO_COUNT):
        rho = (80 + k) / 400.0
        for s in range(EE_SEEDS):
            out.append((Lattice(EE_N, rho, 64 * k + s), k, s))
    return out


def split_of(s: int) -> str:
    if s in EE_HELD_OUT:
        return "test"
    if s in EE_VALIDATION:
        return "val"
    return "train"


# --------------------------------------------------------------------------
# Hand-made and numpy-drawn lattices for tests.
# --------------------------------------------------------------------------

def random_lattice(rng: np.random.Generator, rows: int, cols: int,
                   p_lr: float, p_tb: float) -> np.ndarray:
    """iid cells from a numpy generator: LR w.p. p_lr, TB w.p. p_tb."""
    u = rng.random((rows, cols))
    out = np.zeros((rows, cols), dtype=np.uint8)
    out[u < p_lr] = LR
    out[(u >= p_lr) & (u < p_lr + p_tb)] = TB
    return out


def lone_car(n: int, kind: int, i: int = 0, j: int = 0) -> np.ndarray:
    out = np.zeros((n, n), dtype=np.uint8)
    out[i, j] = kind
    return out


def full_checkerboard(n: int) -> np.ndarray:
    """Every cell occupied, LR where i+j is even, TB where odd."""
    i, j = np.indices((n, n))
    return np.where((i + j) % 2 == 0, LR, TB).astype(np.uint8)


def full_rows(n: int) -> np.ndarray:
    """Every cell occupied by an LR car."""
    return np.full((n, n), LR, dtype=np.uint8)
