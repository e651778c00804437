"""Host-side check of the step kernel's launch geometry (no GPU).

Restates the strip, row and lane index arithmetic of the streaming pass
kernel and checks, for a spread of lattice sizes, strip heights and steps
per pass, that (1) every load and store offset lies inside the state
buffer, (2) the written (row, word) pairs cover the lattice exactly once,
(3) input row t of a strip is lattice row (a - K + t) mod N and lane l holds
word (w0 + l - 1) mod W, and (4) the XCD-aware block order is a permutation
of the waves.
"""
import numpy as np
import pytest

TILE_WORDS = 62


def strip_geometry(n, H, k, layout):
    words = n // 32
    row_bytes = n if layout == 0 else words * 4
    plane = row_bytes * n
    state = plane if layout == 0 else 2 * plane
    size = 32 if layout == 0 else 4
    extra = plane if layout == 1 else 0
    tiles_x = -(-words // TILE_WORDS)
    n_items = tiles_x * -(-n // H)
    covered = np.zeros((n, words), dtype=np.int32)
    lanes = np.arange(64)
    for item in range(n_items):
        sy, tx = divmod(item, tiles_x)
        a = sy * H
        h = min(H, n - a)
        total = h + 2 * k
        w0 = tx * TILE_WORDS
        vwords = min(TILE_WORDS, words - w0)
        word = (w0 + lanes - 1 + words) % words
        lane_ok = (lanes >= 1) & (lanes <= vwords)
        voff = word * 32 if layout == 0 else word * 4
        off = ((a - k + n) % n) * row_bytes
        for t in range(total):
            assert off == ((a - k + t) % n) * row_bytes
            assert 0 <= off and off + voff.max() + size + extra <= state
            off = off + row_bytes
            off = off - plane if off >= plane else off
        st = a * row_bytes
        for t in range(2 * k, total):
            assert st + voff[lane_ok].max() + size + extra <= state
            covered[st // row_bytes, word[lane_ok]] += 1
            st += row_bytes
    assert (covered == 1).all()


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("k", [1, 3, 8])
@pytest.mark.parametrize("n,H", [(32, 8), (32, 32), (64, 24), (96, 40), (224, 64),
                                 (1984, 200), (2016, 8), (2048, 2048), (2144, 96),
                                 (4096, 176)])
def test_strip_geometry(layout, k, n, H):
    strip_geometry(n, H, k, layout)


def test_largest_lattice_offsets_fit_32_bits():
    n = 65504
    plane = n * n
    assert plane < 2**32
    # The last input row offset before a wrap is below the plane size, and
    # one more row (row_bytes = n) stays below 2^32 before the wrap.
    assert (n - 1) * n + n <= 2**32


@pytest.mark.parametrize("grid", [8, 16, 1024, 2048])
@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_xcd_block_order_is_permutation(grid, wpb):
    per_xcd = grid // 8
    firsts = [((b % 8) * per_xcd + b // 8) * wpb + w for b in range(grid) for w in range(wpb)]
    assert sorted(firsts) == list(range(grid * wpb))
