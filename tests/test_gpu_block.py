"""GPU parity of the register-resident tile kernel (bml_set_resident)
against the CPU oracle: cells and all four counts of every step, for tile
and slab counts of one and several, halos from 2 to 32 steps, runs that
are not a whole number of launches, lattices shorter than their halo,
joint launches of several lattices, Model III, the Klein bottle, and the
arguments it refuses."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

from tests.hostinfo import HOST_THREADS  # noqa: E402


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_07981_amd as pkg
    pkg.lib()
    return pkg


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def stats_array(rec):
    return np.stack([rec["n_lr"], rec["moved_lr"], rec["n_tb"], rec["moved_tb"]], axis=1)


def check(lat, want, wst, steps):
    got = lat.cells()
    st = stats_array(lat.stats(0, steps))
    if not np.array_equal(st, wst):
        s0 = int(np.argwhere((st != wst).any(axis=1))[0, 0])
        pytest.fail(f"counts differ from step {s0}: {st[s0]} vs {wst[s0]}")
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        pytest.fail(f"{len(bad)} cells differ, first at {bad[0]}")


# rows x cols, halo steps, steps: one and several tiles and slabs, a lattice
# shorter than its halo (its held block wraps around it several times), runs
# ending inside a launch, slabs cut unevenly (1376 rows at K = 28: four
# slabs of 344; 2336 rows at K = 30: six slabs of 388 or 390 rows), and the
# three tile widths
CASES = [(1024, 1024, 32, 70), (1024, 1024, 16, 37), (1024, 1024, 2, 9),
         (2048, 3072, 32, 65), (96, 1024, 32, 40), (32, 2048, 32, 33),
         (1472, 1024, 24, 50), (512, 4096, 8, 20), (1376, 2048, 28, 61),
         (2336, 1024, 30, 31),
         # narrower tiles: 16 words (4064 x 32768 at K = 2: 256 tiles of 32
         # words would leave CUs idle), 8 words (a lone 4096^2 lattice; 768
         # and 256 columns, which only 8-word tiles divide)
         (4064, 32768, 2, 9), (4096, 4096, 32, 45), (1024, 768, 8, 20), (512, 256, 32, 40)]


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("rows,cols,k,steps", CASES,
                         ids=[f"{r}x{c}_k{k}_s{s}" for r, c, k, s in CASES])
def test_block_matches_oracle(B, layout, rows, cols, k, steps):
    rho_lr, rho_tb = 0.17, 0.19
    seed = rows * 7 + cols + k
    say(f"block {rows}x{cols} k={k} steps={steps} layout={layout}")
    g0 = oracle.init_cells_asym(rows, cols, seed, rho_lr, rho_tb)
    want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS)
    with B.Lattice(rows, seed=seed, layout=layout, cols=cols, rho_lr=rho_lr, rho_tb=rho_tb,
                   stats_cap=steps) as lat:
        lat.set_resident(k)
        assert lat.resident == k
        lat.step(steps)
        check(lat, want, wst, steps)


M3_CASES = [(1024, 1024, 32, 70), (2048, 2048, 28, 57), (96, 1024, 16, 33),
            (1376, 2048, 28, 61)]


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("rows,cols,k,steps", M3_CASES,
                         ids=[f"{r}x{c}_k{k}_s{s}" for r, c, k, s in M3_CASES])
def test_block_model3_matches_oracle(B, layout, rows, cols, k, steps):
    """Model III (one phase; a contested cell takes both cars) in the tile
    kernel: cells (values 0..3) and every count of every step."""
    rho_lr, rho_tb = 0.21, 0.24
    seed = rows + 3 * cols + k
    say(f"block model3 {rows}x{cols} k={k} steps={steps} layout={layout}")
    g0 = oracle.init_cells_asym(rows, cols, seed, rho_lr, rho_tb)
    want, wst = oracle.run_model3(g0, steps, n_threads=HOST_THREADS)
    assert (want == 3).any()                # some cells hold both cars
    with B.Lattice(rows, seed=seed, layout=layout, cols=cols, rho_lr=rho_lr, rho_tb=rho_tb,
                   stats_cap=steps) as lat:
        lat.set_model(3)
        lat.set_resident(k)
        lat.step(steps)
        check(lat, want, wst, steps)


KLEIN_CASES = [(1024, 1024, 32, 70), (2048, 3072, 28, 57), (96, 1024, 16, 33),
               (32, 2048, 32, 33), (1376, 2048, 28, 61), (4096, 4096, 32, 45),
               (1024, 768, 8, 20)]


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("rows,cols,k,steps", KLEIN_CASES,
                         ids=[f"{r}x{c}_k{k}_s{s}" for r, c, k, s in KLEIN_CASES])
def test_block_klein_matches_oracle(B, layout, rows, cols, k, steps):
    """The Klein bottle in the tile kernel (rows across the glued edge held
    mirrored in the first and last slabs; lattices shorter than the halo
    hold rows from across the edge on both sides): cells and every count of
    every step against the oracle's Klein bottle."""
    rho_lr, rho_tb = 0.2, 0.22
    seed = 5 * rows + cols + k
    say(f"block klein {rows}x{cols} k={k} steps={steps} layout={layout}")
    g0 = oracle.init_cells_asym(rows, cols, seed, rho_lr, rho_tb)
    want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS, topology=oracle.KLEIN)
    with B.Lattice(rows, seed=seed, layout=layout, cols=cols, rho_lr=rho_lr, rho_tb=rho_tb,
                   stats_cap=steps) as lat:
        lat.set_topology(B.BML_TOPO_KLEIN)
        lat.set_resident(k)
        lat.step(steps)
        check(lat, want, wst, steps)


def test_block_continues_streaming_runs(B):
    """Runs alternate between the tile kernel (two halos) and the streaming
    kernel on one lattice: the counts ring and the cells follow the oracle."""
    n, rho, seed = 2048, 0.36, 3
    runs = [(32, 40), (0, 11), (16, 21), (0, 3), (32, 32)]
    total = sum(s for _, s in runs)
    want, wst = oracle.run(oracle.init_cells(n, seed, rho), total, n_threads=HOST_THREADS)
    with B.Lattice(n, rho, seed, stats_cap=total) as lat:
        for k, s in runs:
            lat.set_resident(k)
            lat.step(s)
        check(lat, want, wst, total)


@pytest.mark.parametrize("layout", [0, 1])
def test_block_group(B, layout):
    """Three lattices advanced by joint launches of the tile kernel equal
    their oracle runs."""
    import torch
    n, steps = 1024, 45
    specs = [(0.25, 1), (0.38, 2), (0.45, 3)]
    stream = torch.cuda.Stream()
    lats = [B.Lattice(n, rho, seed, layout=layout, stats_cap=steps, stream=stream)
            for rho, seed in specs]
    try:
        for lat in lats:
            lat.set_resident(32)
        B.step_group(lats, steps)
        for lat, (rho, seed) in zip(lats, specs):
            want, wst = oracle.run(oracle.init_cells(n, seed, rho), steps,
                                   n_threads=HOST_THREADS)
            check(lat, want, wst, steps)
    finally:
        for lat in lats:
            lat.close()


def test_block_refusals(B):
    with B.Lattice(1024, 0.3, 1, stats_cap=8) as lat:
        for bad in (-2, 3, 34):
            with pytest.raises(B.BmlError) as e:
                lat.set_resident(bad)
            assert e.value.code == B.BML_EINVAL
        lat.set_resident(32)
        with pytest.raises(B.BmlError) as e:
            lat.set_model(2, 5)                  # Model II: the streaming kernel only
        assert e.value.code == B.BML_EINVAL
        lat.set_model(3)
        lat.set_model(1)
        lat.set_resident(0)
        lat.set_model(2, 5)
        with pytest.raises(B.BmlError) as e:
            lat.set_resident(16)
        assert e.value.code == B.BML_EINVAL
        lat.set_model(1)
        lat.set_resident(32)
        lat.set_topology(B.BML_TOPO_KLEIN)       # the tile kernel runs the Klein bottle too
        with pytest.raises(B.BmlError) as e:
            lat.set_model(3)                     # Model III: the torus only
        assert e.value.code == B.BML_EINVAL
        lat.set_topology(B.BML_TOPO_TORUS)
    with B.Lattice(96, 0.3, 1, stats_cap=8) as lat:  # 96 columns: not whole 256-column tiles
        with pytest.raises(B.BmlError) as e:
            lat.set_resident(16)
        assert e.value.code == B.BML_EINVAL
    with B.Lattice(1024, 0.3, 1, stats_cap=8) as a, B.Lattice(1024, 0.3, 2, stats_cap=8) as b:
        a.set_resident(32)
        with pytest.raises(B.BmlError) as e:     # joint launches need one kernel
            B.step_group([a, b], 4)
        assert e.value.code == B.BML_EINVAL
