"""CPU emulation of the register-resident tile kernel's decomposition
(no GPU): the lattice is cut into tiles of TW words by slabs of rows (cut
at even rows, as equal as possible), each tile is advanced K steps on its
own with one 32-cell halo word on each side and H halo rows above and
below, as an isolated block with open ends (a car at the block's last
column or row does not move, nothing enters at its first), and only the
tile's own cells and counts are kept.  The rule of Sec. 2 moves a car
only by looking at the next cell in its direction of travel, so what an
isolated block gets wrong enters at its edges and travels at most one
cell (one row) per step: with H >= K and K <= 32 the tiles' own cells and
summed counts equal the whole-lattice oracle.  The bound is tight: one
halo row or one halo cell fewer breaks lattices built to carry a hole
towards the tile at full speed."""
import numpy as np
import pytest

import oracle


def open_step(g):
    """One step of the rule on an isolated block with open ends; returns
    the block and the movers of both phases (at their source cells)."""
    lr = g == 1
    free_right = np.zeros_like(lr)
    free_right[:, :-1] = g[:, 1:] == 0
    mv = lr & free_right
    h = g.copy()
    h[mv] = 0
    h[:, 1:][mv[:, :-1]] = 1
    tb = h == 2
    free_below = np.zeros_like(tb)
    free_below[:-1] = h[1:] == 0
    mvv = tb & free_below
    v = h.copy()
    v[mvv] = 0
    v[1:][mvv[:-1]] = 2
    return h, v, mv, mvv


def slab_cuts(rows, slabs):
    pairs = rows // 2
    return [(pairs * s // slabs * 2, pairs * (s + 1) // slabs * 2) for s in range(slabs)]


def tiled_run(g0, k, tile_words, max_held, halo_rows=None, halo_cells=32):
    """The tile decomposition of k steps; returns (cells, counts[k][4])."""
    rows, cols = g0.shape
    H = k if halo_rows is None else halo_rows
    per = max_held - 2 * H
    slabs = -(-rows // per)
    tw = 32 * tile_words
    assert cols % tw == 0
    out = np.zeros_like(g0)
    counts = np.zeros((k, 4), dtype=np.int64)
    for r0, r1 in slab_cuts(rows, slabs):
        R = r1 - r0
        ri = (r0 - H + np.arange(R + 2 * H)) % rows
        for c0 in range(0, cols, tw):
            ci = (c0 - halo_cells + np.arange(tw + 2 * halo_cells)) % cols
            g = g0[np.ix_(ri, ci)]
            own = (slice(H, H + R), slice(halo_cells, halo_cells + tw))
            for s in range(k):
                h, g, mv, mvv = open_step(g)
                counts[s] += [(h[own] == 1).sum(), mv[own].sum(),
                              (g[own] == 2).sum(), mvv[own].sum()]
            out[r0:r1, c0:c0 + tw] = g[own]
    return out, counts


CASES = [  # rows, cols, tile words, rows a block holds, K
    (64, 128, 2, 96, 32), (64, 128, 2, 96, 7), (96, 192, 3, 128, 20),
    (30, 64, 1, 48, 12), (130, 96, 1, 64, 8), (48, 256, 4, 80, 2)]


@pytest.mark.parametrize("rows,cols,tw,held,k", CASES)
@pytest.mark.parametrize("rho", [0.3, 0.55, 0.8])
def test_tiles_equal_the_oracle(rows, cols, tw, held, k, rho):
    g0 = oracle.init_cells(rows, 1000 + rows + k, rho, cols=cols)
    want, wst = oracle.run(g0, k)
    got, cst = tiled_run(g0, k, tw, held)
    assert np.array_equal(got, want)
    assert np.array_equal(cst, wst.astype(np.int64))


def hole_column(rows, cols, col, hole_row):
    """TB cars filling one column except one hole: the hole climbs one row
    per step (the car above it drops in)."""
    g = np.zeros((rows, cols), dtype=np.uint8)
    g[:, col] = 2
    g[hole_row, col] = 0
    return g


def hole_row(rows, cols, row, hole_col):
    """LR cars filling one row except one hole: the hole moves one cell left
    per step."""
    g = np.zeros((rows, cols), dtype=np.uint8)
    g[row, :] = 1
    g[row, hole_col] = 0
    return g


@pytest.mark.parametrize("k", [4, 9, 16])
def test_one_halo_row_short_fails(k):
    rows, cols, held = 96, 64, 96
    H = k - 1
    per = held - 2 * H
    slabs = -(-rows // per)
    r0, r1 = slab_cuts(rows, slabs)[0]
    # the hole starts just below the first slab's block held with K - 1
    # halo rows: after K steps it sits in the slab's last own row
    g0 = hole_column(rows, cols, 5, (r1 + H) % rows)
    want, _ = oracle.run(g0, k)
    assert np.array_equal(tiled_run(g0, k, 1, held)[0], want)        # K halo rows: exact
    assert not np.array_equal(tiled_run(g0, k, 1, held, halo_rows=H)[0], want)


@pytest.mark.parametrize("k", [4, 9, 32])
def test_one_halo_cell_short_fails(k):
    rows, cols, held = 8, 128, 2 * k + 8
    # the hole starts just right of the first tile's block held with K - 1
    # halo cells: after K steps it sits in the tile's last own cell
    g0 = hole_row(rows, cols, 3, (32 + k - 1) % cols)
    want, _ = oracle.run(g0, k)
    assert np.array_equal(tiled_run(g0, k, 1, held)[0], want)
    assert not np.array_equal(tiled_run(g0, k, 1, held, halo_cells=k - 1)[0], want)
