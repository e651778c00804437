"""GPU parity of Model II (Sec. 2: every car advances in one phase; an EMPTY
cell targeted by an LR and a TB car goes to one of them by a coin) against
the oracle's Model II run: every cell and every per-step count, bit for bit.

The coins are counter-based (SplitMix64 output step*rows*W + i*W + j/32 of
the handle's coin stream), so the GPU run and the oracle draw the same coin
for the same cell and step whatever the launch shape; cases cover tile and
row widths, every pass length, passes that end mid-pass, step calls that
continue a run, joint launches and lattices with different histories.
"""
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

U8, BP = 0, 1
LAYOUTS = [U8, BP]
from tests.hostinfo import HOST_THREADS  # noqa: E402


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_07981_amd as pkg
    pkg.lib()   # fail loudly if the library is missing
    return pkg


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def stats_array(rec):
    return np.stack([rec["n_lr"], rec["moved_lr"], rec["n_tb"], rec["moved_tb"]], axis=1)


def check_cells(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        pytest.fail(f"{what}: {len(bad)} cells differ, first at {bad[0]}")


M2_CASES = [(32, 64), (96, 96), (256, 256), (200, 2048), (33, 4096), (1000, 96),
            (64, 3008), (40, 32), (130, 4096)]
M2_TUNINGS = [(0, 16, 4), (8, 6, 2), (3, 12, 1), (24, 2, 1), (1, 16, 4), (0, 14, 2)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("rows,cols", M2_CASES, ids=[f"{r}x{c}" for r, c in M2_CASES])
def test_model2_matches_oracle(B, layout, rows, cols):
    rng = np.random.default_rng(rows * 7919 + cols + 31 * layout)
    for tuning in M2_TUNINGS:
        seed = int(rng.integers(0, 2**32))
        coin_seed = int(rng.integers(0, 2**63)) * 2 + 1
        rho_lr, rho_tb = float(rng.uniform(0.05, 0.45)), float(rng.uniform(0.05, 0.45))
        steps = int(rng.integers(1, 2 * tuning[1] + 5))
        say(f"model2 {rows}x{cols} layout={layout} tuning={tuning} steps={steps} seed={seed} "
            f"coin={coin_seed} lr={rho_lr:.3f} tb={rho_tb:.3f}")
        g0 = oracle.init_cells_asym(rows, cols, seed, rho_lr, rho_tb)
        want, wst = oracle.run_model2(g0, steps, coin_seed, n_threads=HOST_THREADS)
        with B.Lattice(rows, seed=seed, cols=cols, rho_lr=rho_lr, rho_tb=rho_tb, layout=layout,
                       stats_cap=64) as lat:
            lat.set_model(2, coin_seed)
            lat.set_tuning(*tuning)
            lat.step(steps)
            check_cells(lat.cells(), want, f"tuning {tuning}")
            assert np.array_equal(stats_array(lat.stats(0, steps)), wst)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_model2_calls_continue_the_coin_stream(B, layout):
    """Step calls of different lengths, a tuning change between them and a
    switch back to the model of Sec. 2 continue one run: the coins of step s
    are those of global step s."""
    rows, cols, seed, coin = 160, 2048, 42, 0x1234_5678_9ABC_DEF1
    g0 = oracle.init_cells_asym(rows, cols, seed, 0.2, 0.2)
    with B.Lattice(rows, seed=seed, cols=cols, rho_lr=0.2, rho_tb=0.2, layout=layout,
                   stats_cap=128) as lat:
        lat.set_model(2, coin)
        done = 0
        want, wst_all = g0, []
        for n, tuning in [(3, (0, 16, 4)), (11, (8, 10, 2)), (1, (0, 2, 4)), (7, (0, 8, 1))]:
            lat.set_tuning(*tuning)
            lat.step(n)
            want, wst = oracle.run_model2(want, n, coin, step0=done, n_threads=HOST_THREADS)
            wst_all.append(wst)
            done += n
            check_cells(lat.cells(), want, f"after {done} steps")
        assert np.array_equal(stats_array(lat.stats(0, done)), np.concatenate(wst_all))
        lat.set_model(1)
        lat.step(4)
        want, _ = oracle.run(want, 4, n_threads=HOST_THREADS)
        check_cells(lat.cells(), want, "model 1 after model 2")


def test_model2_contested_cells_split_both_ways(B):
    """A lattice where every EMPTY cell with an LR car on its left and a TB
    car above is contested: after one step both kinds of winner occur, in
    the places the oracle's coins put them."""
    rows, cols = 64, 2048
    g = np.zeros((rows, cols), np.uint8)
    g[0::2, 0::2] = 1                   # LR cars on even rows, even columns
    g[1::2, 1::2] = 2                   # TB cars above the odd cells of even rows
    g[0, :] = 0
    want, wst = oracle.run_model2(g, 1, 99)
    with B.Lattice(rows, cols=cols, cells=g, stats_cap=4) as lat:
        lat.set_model(2, 99)
        lat.step(1)
        check_cells(lat.cells(), want)
        st = stats_array(lat.stats(0, 1))
    assert np.array_equal(st, wst)
    contested = int((g[1::2, 1::2] == 2).sum() - cols // 2)   # row rows-1 wraps onto row 0
    assert 0 < st[0, 1] < contested and 0 < st[0, 3]


M2_GROUP_CASES = [(4096, BP, (16, 16, 4), 4), (2048, U8, (0, 6, 4), 3), (224, BP, (24, 16, 1), 8),
                  (96, U8, (3, 14, 4), 5)]


@pytest.mark.parametrize("n,layout,tuning,count", M2_GROUP_CASES,
                         ids=[f"n{n}_l{l}_vr{t[0]}_t{t[1]}_w{t[2]}_x{c}"
                              for n, l, t, c in M2_GROUP_CASES])
def test_model2_step_group(B, n, layout, tuning, count):
    """Joint launches of Model II lattices with their own coin streams and
    histories end where the oracle puts each of them."""
    import torch
    rng = np.random.default_rng(n * 13 + layout)
    stream = torch.cuda.Stream()
    rhos = [0.25, 0.35, 0.38, 0.45, 0.9, 0.1, 0.5, 0.3][:count]
    seeds = [int(x) for x in rng.integers(0, 2**32, count)]
    coins = [int(x) for x in rng.integers(0, 2**62, count)]
    pre = [0, 3, 5, 0, 1, 2, 0, 7][:count]
    steps = int(rng.integers(1, 3 * tuning[1]))
    say(f"model2 group n={n} layout={layout} tuning={tuning} count={count} steps={steps}")
    lats = [B.Lattice(n, r, sd, layout=layout, stats_cap=64, stream=stream)
            for r, sd in zip(rhos, seeds)]
    try:
        for lat, p, c in zip(lats, pre, coins):
            lat.set_model(2, c)
            lat.set_tuning(*tuning)
            if p:
                lat.step(p)
        B.step_group(lats, steps)
        for lat, r, sd, p, c in zip(lats, rhos, seeds, pre, coins):
            want, wst = oracle.run_model2(oracle.init_cells(n, sd, r), p + steps, c,
                                          n_threads=HOST_THREADS)
            check_cells(lat.cells(), want, f"rho={r}")
            assert np.array_equal(stats_array(lat.stats(p, steps)), wst[p:])
    finally:
        for lat in lats:
            lat.close()


def test_model2_errors(B):
    import torch
    stream = torch.cuda.Stream()
    a = B.Lattice(64, 0.3, 1, stream=stream)
    b = B.Lattice(64, 0.3, 2, stream=stream)
    try:
        for bad in (0, 4, -1):
            with pytest.raises(B.BmlError) as e:
                a.set_model(bad)
            assert e.value.code == B.BML_EINVAL
        a.set_topology(B.BML_TOPO_KLEIN)
        with pytest.raises(B.BmlError) as e:
            a.set_model(2, 5)
        assert e.value.code == B.BML_EINVAL
        a.set_topology(B.BML_TOPO_TORUS)
        a.set_model(2, 5)
        with pytest.raises(B.BmlError) as e:
            a.set_topology(B.BML_TOPO_KLEIN)
        assert e.value.code == B.BML_EINVAL
        with pytest.raises(B.BmlError) as e:
            B.step_group([a, b], 1)           # models differ
        assert e.value.code == B.BML_EINVAL
        b.set_model(2, 6)
        g0a, g0b = a.cells(), b.cells()
        B.step_group([a, b], 9)
        wa, _ = oracle.run_model2(g0a, 9, 5)
        wb, _ = oracle.run_model2(g0b, 9, 6)
        check_cells(a.cells(), wa, "a")
        check_cells(b.cells(), wb, "b")
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_model2_medium_full_lattice(B, layout):
    """4096 x 4096 at rho 0.38: every cell after 64 Model II steps in the
    default launch shape, and all 64 count rows."""
    import workloads
    w = workloads.MEDIUM.lattices[2]
    g0 = oracle.init_cells(w.n, w.seed, w.rho)
    want, wst = oracle.run_model2(g0, 64, 2024, n_threads=HOST_THREADS)
    with B.Lattice(w.n, w.rho, w.seed, layout=layout, stats_cap=64) as lat:
        lat.set_model(2, 2024)
        lat.step(64)
        check_cells(lat.cells(), want)
        assert np.array_equal(stats_array(lat.stats(0, 64)), wst)


# --- the 32768 x 32768 lattice, sampled windows ------------------------------

def _window(g, i0, j0, size):
    r = np.arange(i0, i0 + size) % g.shape[0]
    c = np.arange(j0, j0 + size) % g.shape[1]
    return g[np.ix_(r, c)]


@pytest.mark.parametrize("layout", LAYOUTS)
def test_model2_large_sampled_windows(B, layout):
    """32768 x 32768, rho 0.30, seed 7, Model II in the launch shape the
    benchmark times (the tuning cache's Model II entry): 24 steps, then 10
    windows of 64 x 64 (corners, edges, interior) against the oracle run on
    padded windows with the coins of their global positions; car counts
    conserved at every step."""
    import bench
    n, rho, seed, steps, W, coin = 32768, 0.30, 7, 24, 64, 0x5EED
    say(f"model2 large sampled n={n} layout={layout}")
    g0 = oracle.init_cells(n, seed, rho)
    with B.Lattice(n, rho, seed, layout=layout, stats_cap=steps) as lat:
        lat.set_model(2, coin)
        tun = bench.load_tuning(layout, n, None, 2)
        if tun:
            lat.set_tuning(*tun)
        lat.step(steps)
        got = lat.cells()
        st = stats_array(lat.stats(0, steps))
    assert (st[:, 0] == oracle.count(g0, 1)).all() and (st[:, 2] == oracle.count(g0, 2)).all()
    rng = np.random.default_rng(72)
    picks = [(0, 0), (0, n - W), (n - W, 0), (n - W, n - W), (n // 2, n // 2 - 32)]
    picks += [tuple(int(x) for x in rng.integers(0, n, size=2)) for _ in range(5)]
    for i0, j0 in picks:
        pad = _window(g0, i0 - steps, j0 - steps, W + 2 * steps)
        ref, _ = oracle.run_model2(pad, steps, coin,
                                   frame=((i0 - steps) % n, (j0 - steps) % n, n, n))
        assert np.array_equal(_window(got, i0, j0, W), ref[steps:steps + W, steps:steps + W]), \
            (i0, j0)
