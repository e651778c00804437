"""Host-side check of the step kernel's launch geometry (no GPU).

Restates the tile, row and lane index arithmetic of the pass kernel and
checks, for every tuning and a spread of lattice sizes, that (1) every load
and store offset lies inside the state buffer, (2) the written (row, word)
pairs cover the lattice exactly once, (3) tile row r holds lattice row
(ty*VR - K + r) mod N and lane l holds word (w0 + l - 1) mod W, and (4) the
XCD-aware block order is a permutation of the waves.
"""
import numpy as np
import pytest

TILE_WORDS = 62
MAX_K = 8


def tile_geometry(n, vr, k, layout):
    words = n // 32
    row_bytes = n if layout == 0 else words * 4
    plane = row_bytes * n
    state = plane if layout == 0 else 2 * plane
    R = vr + 2 * k
    tiles_x = -(-words // TILE_WORDS)
    n_tiles = tiles_x * (n // vr)
    covered = np.zeros((n, words), dtype=np.int32)
    lanes = np.arange(64)
    for t in range(n_tiles):
        ty, tx = divmod(t, tiles_x)
        w0 = tx * TILE_WORDS
        vwords = min(TILE_WORDS, words - w0)
        word = (w0 + lanes - 1 + words) % words
        lane_ok = (lanes >= 1) & (lanes <= vwords)
        voff = word * 32 if layout == 0 else word * 4
        roff0 = ((ty * vr - k + n) % n) * row_bytes
        for r in range(R):
            o = roff0 + r * row_bytes
            for _ in range(3):
                o = o - plane if o >= plane else o
            assert o == ((ty * vr - k + r) % n) * row_bytes
            size = 32 if layout == 0 else 4
            last = o + voff.max() + size + (plane if layout == 1 else 0)
            assert o >= 0 and last <= state
        out0 = ty * vr * row_bytes
        for r in range(k, k + vr):
            ro = out0 + (r - k) * row_bytes
            size = 32 if layout == 0 else 4
            assert ro + voff[lane_ok].max() + size + (plane if layout == 1 else 0) <= state
            covered[ty * vr + r - k, word[lane_ok]] += 1
    assert (covered == 1).all()


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("vr", [32, 64])
@pytest.mark.parametrize("k", [1, 2, 5, 8])
@pytest.mark.parametrize("n", [32, 64, 96, 224, 1984, 2016, 2048, 2144, 4096])
def test_tile_geometry(layout, vr, k, n):
    if n % vr:
        vr = 32   # the library falls back to 32 output rows
    tile_geometry(n, vr, k, layout)


def test_largest_lattice_offsets_fit_32_bits():
    n = 65504
    plane = n * n
    assert plane < 2**32
    k, vr = MAX_K, 32
    roff0 = ((n - 1) % n) * n      # last tile row
    o = roff0 + (vr + 2 * k - 1) * n
    assert o < 2**33               # computed in 64 bits in the kernel
    while o >= plane:
        o -= plane
    assert o + n <= plane


@pytest.mark.parametrize("grid", [8, 16, 1024, 2048])
@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_xcd_block_order_is_permutation(grid, wpb):
    per_xcd = grid // 8
    firsts = [((b % 8) * per_xcd + b // 8) * wpb + w for b in range(grid) for w in range(wpb)]
    assert sorted(firsts) == list(range(grid * wpb))
