"""CPU emulation of the streaming step kernel's skewed level pipeline (no
GPU), row by row in numpy, to check its control flow against the oracle.

A strip of h output rows streams the h + 2K input rows row_a - K .. row_a +
h + K - 1 (periodic).  Level k holds one pending row (after its horizontal
phase) and the TB movers of the row before it; pushed row r, it runs the
horizontal phase of row r, decides the TB movers of row r - 1 (their cell
below, in row r after its horizontal phase, is EMPTY) and emits row r - 1
after the step.  In iteration t level k takes the row level k - 1 emitted
in iteration t - 1 (level 0 the input row t), levels visited from K - 1
down to 0; level K - 1's output is stored for t in [3K - 1, 3K - 1 + h).
Level k is skipped outside 3k <= t <= h + 2K - 1 + k: the test shows the
strips then reproduce K steps of the oracle (cells and all four counts)
and that moving either bound inwards by one breaks them."""
import numpy as np
import pytest

import oracle


def h_phase(L, T):
    """Horizontal phase of one periodic row (boolean planes)."""
    empty = ~(L | T)
    mv = L & np.roll(empty, -1)
    return (L & ~mv) | np.roll(mv, 1), mv


def strip(g0, row_a, h, K, lo=0, hi=0):
    """One strip of the pipeline; lo / hi move the idle-level window's
    lower / upper bound.  Returns (output rows, counts[K][4])."""
    N = g0.shape[0]
    total_in, total_it = h + 2 * K, h + 3 * K - 1
    zero = np.zeros(g0.shape[1], dtype=bool)
    lvL = [zero] * K
    lvT = [zero] * K
    lvM = [zero] * K
    bl = [zero] * K
    bt = [zero] * K
    acc = np.zeros((K, 4), dtype=np.int64)
    out = {}
    for t in range(total_it):
        if t < total_in:
            row = g0[(row_a - K + t) % N]
            L0, T0 = row == 1, row == 2
        else:
            L0, T0 = zero, zero
        for k in range(K - 1, -1, -1):
            if t < 3 * k + lo or t > h + 2 * K - 1 + k + hi:
                continue
            Lin, Tin = (L0, T0) if k == 0 else (bl[k - 1], bt[k - 1])
            L, mv_h = h_phase(Lin, Tin)
            mv = lvT[k] & ~(L | Tin)
            t_new = (lvT[k] & ~mv) | lvM[k]
            oL, oT = lvL[k], t_new
            lvL[k], lvT[k], lvM[k] = L, Tin, mv
            rh = t - 2 * k - K
            if 0 <= rh < h:
                acc[k, 0] += L.sum()
                acc[k, 1] += mv_h.sum()
            if 1 <= rh <= h:
                acc[k, 2] += t_new.sum()
                acc[k, 3] += mv.sum()
            bl[k], bt[k] = oL, oT
        if 3 * K - 1 <= t < 3 * K - 1 + h:
            r = (row_a + t - (3 * K - 1)) % N
            out[r] = np.where(bl[K - 1], 1, np.where(bt[K - 1], 2, 0)).astype(np.uint8)
    return out, acc


def pass_run(g0, K, h, lo=0, hi=0):
    N = g0.shape[0]
    got = np.zeros_like(g0)
    counts = np.zeros((K, 4), dtype=np.int64)
    for row_a in range(0, N, h):
        hh = min(h, N - row_a)
        rows, acc = strip(g0, row_a, hh, K, lo, hi)
        for r, v in rows.items():
            got[r] = v
        counts += acc
    return got, counts


CASES = [(64, 96, 8, 16), (64, 64, 4, 64), (48, 64, 12, 8), (40, 32, 1, 40), (72, 64, 6, 20)]


@pytest.mark.parametrize("n,cols,K,h", CASES)
@pytest.mark.parametrize("rho", [0.3, 0.6])
def test_pipeline_matches_the_oracle(n, cols, K, h, rho):
    g0 = oracle.init_cells(n, 7 * n + K, rho, cols=cols)
    want, wst = oracle.run(g0, K)
    got, counts = pass_run(g0, K, h)
    assert np.array_equal(got, want)
    assert np.array_equal(counts, wst.astype(np.int64))


@pytest.mark.parametrize("n,cols,K,h", CASES[:3])
def test_narrower_window_breaks(n, cols, K, h):
    """Either bound of the idle-level window moved inwards by one: some
    strip's cells or counts differ from the oracle."""
    g0 = oracle.init_cells(n, 11 * n + K, 0.45, cols=cols)
    want, wst = oracle.run(g0, K)
    for lo, hi in ((1, 0), (0, -1)):
        got, counts = pass_run(g0, K, h, lo, hi)
        assert not (np.array_equal(got, want) and np.array_equal(counts, wst.astype(np.int64))), \
            (lo, hi)
