"""GPU parity of the single-lattice path (libbml through its C ABI) against
the CPU oracle: every cell and every per-step count, bit for bit.

Sizes span several tiles and the periodic wrap; tunings cover every kernel
variant and pass length, including passes that end mid-pass (n_steps not a
multiple of the steps per pass).  Large lattices are checked on sampled
windows using the dependence cone: after s steps a cell depends only on
cells within s rows and s columns of it, so a (W+2s)^2 periodic window of the
initial lattice, run s steps by the oracle, fixes its middle W x W block.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads

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


def make(B, n, rho=0.3, seed=0, layout=U8, cells=None, cap=4096, tuning=None):
    lat = B.Lattice(n, rho, seed, layout=layout, cells=cells, stats_cap=cap)
    if tuning:
        lat.set_tuning(*tuning)
    return lat


# --- initial placement --------------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n,seed,rho", [(32, 0, 0.3), (64, 5, 0.0), (96, 7, 1.0),
                                        (256, 0, 0.3), (512, 12345, 0.45),
                                        (1024, 2**63 + 11, 0.25)])
def test_init_matches_oracle(B, layout, n, seed, rho):
    say(f"init n={n} seed={seed} rho={rho} layout={layout}")
    with make(B, n, rho, seed, layout) as lat:
        want = oracle.init_cells(n, seed, rho)
        assert np.array_equal(lat.cells(), want)
        assert lat.initial_counts() == (oracle.count(want, 1), oracle.count(want, 2))


# --- small lattice, every step --------------------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
def test_small_every_step(B, layout):
    """256 x 256, rho 0.30, seed 0: all cells and counts after each of 1024
    steps."""
    say(f"small every step layout={layout}")
    w = workloads.SMALL
    lt = w.lattices[0]
    ref = oracle.init_cells(lt.n, lt.seed, lt.rho)
    with make(B, lt.n, lt.rho, lt.seed, layout, cap=w.steps) as lat:
        assert np.array_equal(lat.cells(), ref)
        for s in range(w.steps):
            lat.step(1)
            ref, st = oracle.run(ref, 1)
            got = lat.cells()
            if not np.array_equal(got, ref):
                bad = np.argwhere(got != ref)
                pytest.fail(f"step {s}: {len(bad)} cells differ, first at {bad[0]}")
        want = oracle.run(oracle.init_cells(lt.n, lt.seed, lt.rho), w.steps)[1]
        assert np.array_equal(stats_array(lat.stats(0, w.steps)), want)


# --- random sizes, tunings, layouts ---------------------------------------

# (strip rows, phases per pass, waves per block); 0 strip rows = automatic.
TUNINGS = [(0, 2, 4), (8, 2, 4), (32, 4, 1), (64, 8, 2), (0, 16, 4), (40, 16, 1),
           (24, 6, 2), (200, 10, 4), (3, 12, 4)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("tuning", TUNINGS, ids=[f"vr{a}_t{b}_w{c}" for a, b, c in TUNINGS])
def test_random_sizes_all_counts(B, layout, tuning):
    rng = np.random.default_rng(hash((layout,) + tuning) % 2**32)
    for n in (32, 64, 96, 160, 224, 384, 2048 + 96):
        steps = int(rng.integers(1, 40))
        rho = float(rng.choice([0.1, 0.3, 0.38, 0.5, 0.9]))
        seed = int(rng.integers(0, 2**32))
        say(f"random n={n} steps={steps} rho={rho} seed={seed} layout={layout} tuning={tuning}")
        g0 = oracle.init_cells(n, seed, rho)
        want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS)
        with make(B, n, rho, seed, layout, cap=64, tuning=tuning) as lat:
            lat.step(steps)
            assert np.array_equal(lat.cells(), want), (n, steps)
            assert np.array_equal(stats_array(lat.stats(0, steps)), wst), (n, steps)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_hand_made_lattices(B, layout):
    n = 64
    cases = {
        "lone_lr": workloads.lone_car(n, 1, 5, 63),
        "lone_tb": workloads.lone_car(n, 2, 63, 7),
        "checkerboard_full": workloads.full_checkerboard(n),
        "rows_full": workloads.full_rows(n),
        "empty": np.zeros((n, n), np.uint8),
    }
    for name, g in cases.items():
        say(f"hand-made {name} layout={layout}")
        want, wst = oracle.run(g, n + 3)
        with make(B, n, layout=layout, cells=g, cap=256, tuning=(32, 4, 2)) as lat:
            lat.step(n + 3)
            assert np.array_equal(lat.cells(), want), name
            assert np.array_equal(stats_array(lat.stats(0, n + 3)), wst), name


def test_lone_car_returns(B):
    n = 96
    g = workloads.lone_car(n, 1, 40, 95)
    with make(B, n, cells=g, tuning=(32, 16, 4)) as lat:
        lat.step(n)
        assert np.array_equal(lat.cells(), g)
        st = stats_array(lat.stats(0, n))
        assert (st == np.array([1, 1, 0, 0])).all()


# --- invariance -------------------------------------------------------------

def test_tuning_and_layout_invariance(B):
    n, steps = 320, 57
    ref = None
    for layout in LAYOUTS:
        for vr in (0, 8, 64, 320):
            for t in (2, 4, 8, 12, 16):
                for w in (1, 4):
                    say(f"invariance layout={layout} vr={vr} t={t} w={w}")
                    with make(B, n, 0.33, 99, layout, cap=steps, tuning=(vr, t, w)) as lat:
                        lat.step(steps)
                        got = (lat.cells(), stats_array(lat.stats(0, steps)))
                    if ref is None:
                        ref = got
                        want, wst = oracle.run(oracle.init_cells(n, 99, 0.33), steps)
                        assert np.array_equal(ref[0], want) and np.array_equal(ref[1], wst)
                    else:
                        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_step_calls_compose(B):
    """Many small bml_step calls equal one large one (pass boundaries inside
    and across calls)."""
    n = 128
    with make(B, n, 0.35, 3, U8, cap=200, tuning=(32, 8, 4)) as a, \
            make(B, n, 0.35, 3, U8, cap=200, tuning=(32, 8, 4)) as b:
        a.step(101)
        for k in (1, 2, 3, 5, 7, 11, 13, 17, 19, 23):
            b.step(k)
        b.step(0)
        assert b.steps_done == 101
        assert np.array_equal(a.cells(), b.cells())
        assert np.array_equal(stats_array(a.stats(0, 101)), stats_array(b.stats(0, 101)))


def test_checkpoint_resume(B):
    n = 256
    for layout in LAYOUTS:
        with make(B, n, 0.31, 8, layout) as full:
            full.step(150)
            want = full.cells()
            wst = stats_array(full.stats(100, 50))
        with make(B, n, 0.31, 8, layout) as a:
            a.step(100)
            mid = a.cells()
        with make(B, n, layout=layout, cells=mid) as b:
            b.step(50)
            assert np.array_equal(b.cells(), want)
            assert np.array_equal(stats_array(b.stats(0, 50)), wst)


# --- stats ring and errors ----------------------------------------------------

def test_stats_ring_window(B):
    n, cap = 64, 10
    g0 = oracle.init_cells(n, 4, 0.3)
    _, wst = oracle.run(g0, 37)
    with make(B, n, 0.3, 4, U8, cap=cap, tuning=(32, 6, 4)) as lat:
        lat.step(25)
        lat.step(12)
        assert np.array_equal(stats_array(lat.stats(27, 10)), wst[27:37])
        assert np.array_equal(stats_array(lat.stats(30, 5)), wst[30:35])
        for first, count in ((26, 2), (30, 8), (-1, 1)):
            with pytest.raises(B.BmlError) as e:
                lat.stats(first, count)
            assert e.value.code == B.BML_ERANGE


def test_corruption_is_detected(B):
    import torch
    n = 64
    with make(B, n, 0.2, 1, U8) as lat:
        lat.step(3)
        buf = lat.state_tensor()
        cells = buf.view(n, n)
        empty = (cells == 0).nonzero()[0]
        cells[empty[0], empty[1]] = 1    # one extra LR car appears
        torch.cuda.synchronize()
        lat.step(2)
        with pytest.raises(B.BmlError) as e:
            lat.stats(3, 2)
        assert e.value.code == B.BML_ECORRUPT
        rec = lat.stats(3, 2, check=False)
        assert rec["n_lr"][0] == lat.initial_counts()[0] + 1


def test_errors_and_free(B):
    with pytest.raises(B.BmlError) as e:
        make(B, 48)
    assert e.value.code == B.BML_EINVAL
    lat = make(B, 64)
    with pytest.raises(B.BmlError) as e:
        lat.set_tuning(65536, 0, 0)
    assert e.value.code == B.BML_EINVAL
    with pytest.raises(B.BmlError):
        lat.set_tuning(0, 3, 0)
    with pytest.raises(B.BmlError):
        lat.set_tuning(0, 0, 8)
    with pytest.raises(B.BmlError):
        lat.step(-1)
    h = lat.handle
    lat.close()
    with pytest.raises(B.BmlError) as e:
        B.bml_step(h, 1)
    assert e.value.code == B.BML_ESTATE


def test_pack_unpack_roundtrip(B):
    import torch
    n = 192
    g = workloads.random_lattice(np.random.default_rng(5), n, n, 0.3, 0.3)
    d_cells = torch.from_numpy(g).cuda()
    d_planes = torch.empty(n * n // 4, dtype=torch.uint8, device="cuda")
    d_back = torch.empty_like(d_cells)
    B.bml_pack(n, d_cells, d_planes)
    B.bml_unpack(n, d_planes, d_back)
    torch.cuda.synchronize()
    lr, tb = oracle.pack(g)
    planes = d_planes.cpu().numpy().view(np.uint32)
    assert np.array_equal(planes[: n * n // 32].reshape(n, n // 32), lr)
    assert np.array_equal(planes[n * n // 32:].reshape(n, n // 32), tb)
    assert np.array_equal(d_back.cpu().numpy(), g)


# --- row mode: N = 2048 and 4096 (a whole row per wavefront) ----------------

ROW_TUNINGS = [(0, 2, 4), (8, 4, 4), (16, 16, 4), (24, 10, 2), (4096, 12, 1), (40, 14, 4),
               (8, 16, 1), (0, 6, 2), (1, 16, 4), (3, 8, 2)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", [2048, 4096])
@pytest.mark.parametrize("tuning", ROW_TUNINGS, ids=[f"vr{a}_t{b}_w{c}" for a, b, c in ROW_TUNINGS])
def test_row_mode_all_counts(B, layout, n, tuning):
    """Row lengths of 64 and 128 words put a whole row in one wavefront with
    wrapping lane moves; strips of several heights (some not dividing N),
    every pass length, and runs that end mid-pass."""
    rng = np.random.default_rng(hash((layout, n) + tuning) % 2**32)
    steps = int(rng.integers(1, 3 * tuning[1]))
    rho = float(rng.choice([0.1, 0.3, 0.38, 0.5, 0.9]))
    seed = int(rng.integers(0, 2**32))
    say(f"row mode n={n} steps={steps} rho={rho} seed={seed} layout={layout} tuning={tuning}")
    g0 = oracle.init_cells(n, seed, rho)
    want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS)
    with make(B, n, rho, seed, layout, cap=64, tuning=tuning) as lat:
        lat.step(steps)
        got = lat.cells()
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            pytest.fail(f"{len(bad)} cells differ, first at {bad[0]}")
        assert np.array_equal(stats_array(lat.stats(0, steps)), wst)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", [2048, 4096])
def test_row_mode_wrap_cars(B, layout, n):
    """Cars that cross the periodic seam (last word of the row, lane 63, to
    the first, lane 0) and the seam between a lane's two words: a lone LR car
    starting at the right edge and a lone TB car at the bottom edge are back
    home after N steps, and a jam across the seam matches the oracle."""
    say(f"row mode wrap n={n} layout={layout}")
    g = np.zeros((n, n), np.uint8)
    g[5, n - 1] = 1          # LR car about to wrap in x
    g[n - 1, 37] = 2         # TB car about to wrap in y
    g[100, 2046:2051] = 1    # cars across lanes 31/32 (n = 4096: word seam)
    g[101, 63:66] = 2
    g[200, n - 3:] = 1
    g[200, :2] = 2           # blocked by a TB car just across the x seam
    want, wst = oracle.run(g, 3 * n // 2, n_threads=HOST_THREADS)
    with make(B, n, layout=layout, cells=g, cap=64) as lat:
        lat.step(n)
        lat.step(n // 2)
        assert np.array_equal(lat.cells(), want)
        assert np.array_equal(stats_array(lat.stats(3 * n // 2 - 64, 64)), wst[-64:])
    lone = np.zeros((n, n), np.uint8)
    lone[7, n - 1] = 1
    lone[n - 1, 9] = 2
    with make(B, n, layout=layout, cells=lone, cap=8) as lat:
        lat.step(n)
        assert np.array_equal(lat.cells(), lone)


# --- joint launches of several lattices (bml_step_group) -------------------

GROUP_CASES = [(4096, BP, (16, 16, 4), 4), (4096, U8, (8, 12, 2), 4), (2144, U8, (0, 6, 4), 3),
               (224, BP, (24, 16, 1), 8), (2048, U8, (0, 2, 4), 2), (96, U8, (3, 14, 4), 5)]


@pytest.mark.parametrize("n,layout,tuning,count", GROUP_CASES,
                         ids=[f"n{n}_l{l}_vr{t[0]}_t{t[1]}_w{t[2]}_x{c}"
                              for n, l, t, c in GROUP_CASES])
def test_step_group_matches_each_alone(B, n, layout, tuning, count):
    """Lattices advanced together in joint launches, with different
    histories (some stepped alone first) and stats rings of different sizes,
    end where the oracle puts each of them, and each ring holds that
    lattice's own counts."""
    import torch
    rng = np.random.default_rng(n * 31 + layout)
    stream = torch.cuda.Stream()
    rhos = [0.25, 0.35, 0.38, 0.45, 0.9, 0.1, 0.5, 0.3][:count]
    seeds = [int(x) for x in rng.integers(0, 2**32, count)]
    caps = [64, 30, 64, 7, 64, 5, 64, 64][:count]
    pre = [0, 3, 5, 0, 1, 2, 0, 7][:count]
    steps = int(rng.integers(1, 3 * tuning[1]))
    say(f"group n={n} layout={layout} tuning={tuning} count={count} steps={steps}")
    lats = [B.Lattice(n, r, sd, layout=layout, stats_cap=c, stream=stream)
            for r, sd, c in zip(rhos, seeds, caps)]
    try:
        for lat, p in zip(lats, pre):
            lat.set_tuning(*tuning)
            if p:
                lat.step(p)
        B.step_group(lats, steps)
        for lat, r, sd, c, p in zip(lats, rhos, seeds, caps, pre):
            want, wst = oracle.run(oracle.init_cells(n, sd, r), p + steps, n_threads=HOST_THREADS)
            assert lat.steps_done == p + steps
            got = lat.cells()
            if not np.array_equal(got, want):
                bad = np.argwhere(got != want)
                pytest.fail(f"rho={r}: {len(bad)} cells differ, first at {bad[0]}")
            m = min(c, steps)
            assert np.array_equal(stats_array(lat.stats(p + steps - m, m)), wst[-m:]), r
    finally:
        for lat in lats:
            lat.close()


def test_step_group_rejects_mismatches(B):
    import torch
    stream = torch.cuda.Stream()
    a = B.Lattice(64, 0.3, 1, stream=stream)
    b = B.Lattice(64, 0.3, 2, stream=stream)
    c = B.Lattice(96, 0.3, 3, stream=stream)
    d = B.Lattice(64, 0.3, 4, layout=BP, stream=stream)
    e = B.Lattice(64, 0.3, 5, stream=torch.cuda.Stream())
    try:
        for bad in ([a, a], [a, c], [a, d], [a, e]):
            with pytest.raises(B.BmlError) as err:
                B.step_group(bad, 1)
            assert err.value.code == B.BML_EINVAL
        b.set_tuning(-1, 4, 0)
        with pytest.raises(B.BmlError) as err:
            B.step_group([a, b], 1)
        assert err.value.code == B.BML_EINVAL
        assert a.steps_done == 0 and b.steps_done == 0
        b.set_tuning(-1, a.tuning()[1], 0)
        B.step_group([a, b], 0)
        B.step_group([a, b], 2)
        assert a.steps_done == 2 and b.steps_done == 2
    finally:
        for lat in (a, b, c, d, e):
            lat.close()


# --- rectangular lattices, unequal LR / TB densities ---------------------

RECT_CASES = [(32, 64, 0.1, 0.3), (96, 160, 0.3, 0.1), (200, 2048, 0.2, 0.15),
              (33, 4096, 0.05, 0.4), (1000, 96, 0.0, 0.5), (64, 3008, 0.45, 0.45),
              (517, 224, 0.25, 0.0)]
RECT_TUNINGS = [(0, 16, 4), (8, 6, 2), (24, 2, 1)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("rows,cols,rho_lr,rho_tb", RECT_CASES,
                         ids=[f"{r}x{c}_lr{a}_tb{b}" for r, c, a, b in RECT_CASES])
def test_rect_asym_matches_oracle(B, layout, rows, cols, rho_lr, rho_tb):
    """rows x cols lattices (rows not a multiple of 32, row-mode widths with
    rows != cols, tile-mode widths) with unequal LR / TB densities: the
    initial draw, then every cell and count after runs under several
    tunings, against the oracle's asymmetric draw and run."""
    rng = np.random.default_rng(rows * 7919 + cols + layout)
    seed = int(rng.integers(0, 2**32))
    g0 = oracle.init_cells_asym(rows, cols, seed, rho_lr, rho_tb)
    for tuning in RECT_TUNINGS:
        steps = int(rng.integers(1, 2 * tuning[1] + 3))
        say(f"rect {rows}x{cols} lr={rho_lr} tb={rho_tb} layout={layout} tuning={tuning} "
            f"steps={steps} seed={seed}")
        want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS)
        with B.Lattice(rows, seed=seed, cols=cols, rho_lr=rho_lr, rho_tb=rho_tb, layout=layout,
                       stats_cap=64) as lat:
            assert np.array_equal(lat.cells(), g0)
            assert lat.initial_counts() == (oracle.count(g0, 1), oracle.count(g0, 2))
            lat.set_tuning(*tuning)
            lat.step(steps)
            got = lat.cells()
            if not np.array_equal(got, want):
                bad = np.argwhere(got != want)
                pytest.fail(f"{len(bad)} cells differ, first at {bad[0]}")
            assert np.array_equal(stats_array(lat.stats(0, steps)), wst)


def test_rect_equal_halves_is_the_square_draw(B):
    with B.Lattice(256, 0.37, 11) as a, \
            B.Lattice(256, seed=11, cols=256, rho_lr=0.37 / 2, rho_tb=0.37 / 2) as b:
        assert np.array_equal(a.cells(), b.cells())


def test_rect_group_and_host_cells(B):
    """Rectangular lattices in joint launches, one of them from host cells."""
    import torch
    rows, cols, steps = 300, 2048, 21
    stream = torch.cuda.Stream()
    g1 = oracle.init_cells_asym(rows, cols, 5, 0.2, 0.25)
    hand = np.zeros((rows, cols), np.uint8)
    hand[7, cols - 1] = 1
    hand[rows - 1, 9] = 2
    hand[100, 1000:1010] = 1
    lats = [B.Lattice(rows, seed=5, cols=cols, rho_lr=0.2, rho_tb=0.25, stream=stream),
            B.Lattice(rows, cols=cols, cells=hand, layout=U8, stream=stream)]
    try:
        B.step_group(lats, steps)
        for lat, g in zip(lats, (g1, hand)):
            want, wst = oracle.run(g, steps, n_threads=HOST_THREADS)
            assert np.array_equal(lat.cells(), want)
            assert np.array_equal(stats_array(lat.stats(0, steps)), wst)
    finally:
        for lat in lats:
            lat.close()


# --- Klein bottle (top and bottom edges glued with a reversal) ------------

KLEIN_CASES = [(32, 64), (96, 160), (200, 2048), (33, 4096), (1000, 96), (64, 3008), (40, 32)]
KLEIN_TUNINGS = [(0, 16, 4), (8, 6, 2), (3, 12, 1), (24, 2, 1), (1, 16, 4)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("rows,cols", KLEIN_CASES, ids=[f"{r}x{c}" for r, c in KLEIN_CASES])
def test_klein_matches_oracle(B, layout, rows, cols):
    """Klein-bottle lattices (strips whose halo crosses the glued edge at the
    top, the bottom or both; tile and row widths): every cell and count
    against the oracle's Klein run, under several tunings."""
    rng = np.random.default_rng(rows * 104729 + cols + 17 * layout)
    for tuning in KLEIN_TUNINGS:
        seed = int(rng.integers(0, 2**32))
        rho_lr, rho_tb = float(rng.uniform(0.05, 0.4)), float(rng.uniform(0.05, 0.4))
        steps = int(rng.integers(1, 2 * tuning[1] + 5))
        say(f"klein {rows}x{cols} layout={layout} tuning={tuning} steps={steps} seed={seed} "
            f"lr={rho_lr:.3f} tb={rho_tb:.3f}")
        g0 = oracle.init_cells_asym(rows, cols, seed, rho_lr, rho_tb)
        want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS, topology=oracle.KLEIN)
        with B.Lattice(rows, seed=seed, cols=cols, rho_lr=rho_lr, rho_tb=rho_tb, layout=layout,
                       stats_cap=64) as lat:
            lat.set_topology(B.BML_TOPO_KLEIN)
            lat.set_tuning(*tuning)
            lat.step(steps)
            got = lat.cells()
            if not np.array_equal(got, want):
                bad = np.argwhere(got != want)
                pytest.fail(f"{len(bad)} cells differ, first at {bad[0]}")
            assert np.array_equal(stats_array(lat.stats(0, steps)), wst)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_klein_lone_tb_car_mirrored_then_home(B, layout):
    rows, cols = 64, 2048
    g = np.zeros((rows, cols), np.uint8)
    g[5, 3] = 2
    g[9, 40] = 1
    with B.Lattice(rows, cols=cols, cells=g, layout=layout, stats_cap=8) as lat:
        lat.set_topology(B.BML_TOPO_KLEIN)
        assert lat.topology == B.BML_TOPO_KLEIN
        lat.step(rows)
        want, _ = oracle.run(g, rows, topology=oracle.KLEIN)
        assert want[5, cols - 1 - 3] == 2
        assert np.array_equal(lat.cells(), want)
        lat.step(rows)
        want2, _ = oracle.run(want, rows, topology=oracle.KLEIN)
        assert np.array_equal(lat.cells(), want2)


def test_klein_errors_and_torus_switch(B):
    import torch
    stream = torch.cuda.Stream()
    a = B.Lattice(64, 0.3, 1, stream=stream)
    b = B.Lattice(64, 0.3, 2, stream=stream)
    try:
        with pytest.raises(B.BmlError) as e:
            a.set_topology(2)
        assert e.value.code == B.BML_EINVAL
        a.set_topology(B.BML_TOPO_KLEIN)
        with pytest.raises(B.BmlError) as e:
            B.step_group([a, b], 1)
        assert e.value.code == B.BML_EINVAL
        b.set_topology(B.BML_TOPO_KLEIN)
        g0a, g0b = a.cells(), b.cells()
        B.step_group([a, b], 5)
        a.set_topology(B.BML_TOPO_TORUS)
        a.step(3)
        wa, _ = oracle.run(g0a, 5, topology=oracle.KLEIN)
        wa, _ = oracle.run(wa, 3)
        wb, _ = oracle.run(g0b, 5, topology=oracle.KLEIN)
        assert np.array_equal(a.cells(), wa) and np.array_equal(b.cells(), wb)
    finally:
        a.close()
        b.close()


# --- the 4096 x 4096 workload, whole lattice --------------------------------

@pytest.mark.parametrize("layout", LAYOUTS)
def test_medium_full_lattice(B, layout):
    """4096 x 4096 at rho 0.38 (seed 3 as in the four-density workload),
    default tuning: every cell and count after 120 steps."""
    n, rho, seed, steps = 4096, 0.38, 3, 120
    say(f"medium full n={n} layout={layout}")
    g0 = oracle.init_cells(n, seed, rho)
    want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS)
    with make(B, n, rho, seed, layout, cap=steps) as lat:
        lat.step(steps)
        assert np.array_equal(lat.cells(), want)
        assert np.array_equal(stats_array(lat.stats(0, steps)), wst)


# --- the four-lattice 4096 x 4096 workload in the benchmark's launch shape ---

MEDIUM_CHECK_STEPS = 1000


@pytest.fixture(scope="module")
def medium_reference():
    """The oracle's run of the four 4096 x 4096 lattices (rho .25/.35/.38/.45,
    seeds 1-4): final cells and every step's counts, on all host threads."""
    w = workloads.MEDIUM
    out = []
    for lt in w.lattices:
        say(f"oracle: 4096^2 rho={lt.rho} seed={lt.seed}, {MEDIUM_CHECK_STEPS} steps, "
            f"{HOST_THREADS} threads")
        out.append(oracle.run(oracle.init_cells(lt.n, lt.seed, lt.rho), MEDIUM_CHECK_STEPS,
                              n_threads=HOST_THREADS))
    return out


@pytest.mark.parametrize("layout", LAYOUTS)
def test_medium_bench_shape(B, layout, medium_reference):
    """The four lattices advanced together by joint launches in the tuned
    shape the benchmark times (bench.load_tuning(layout, 4096, "medium4")),
    1000 steps: every count of every step and every final cell."""
    import torch
    import bench
    w = workloads.MEDIUM
    tun = bench.load_tuning(layout, 4096, workloads.MEDIUM_GROUP)
    res = bench.load_resident_steps(layout, 4096, workloads.MEDIUM_GROUP)
    say(f"medium bench shape layout={layout} tuning={tun} resident={res}")
    stream = torch.cuda.Stream()
    lats = [B.Lattice(lt.n, lt.rho, lt.seed, layout=layout, stats_cap=MEDIUM_CHECK_STEPS,
                      stream=stream) for lt in w.lattices]
    try:
        for lat in lats:
            if tun:
                lat.set_tuning(*tun)
            if res:
                lat.set_resident(res)
        B.step_group(lats, MEDIUM_CHECK_STEPS)
        for lat, lt, (want, wst) in zip(lats, w.lattices, medium_reference):
            got = lat.cells()
            if not np.array_equal(got, want):
                bad = np.argwhere(got != want)
                pytest.fail(f"rho={lt.rho}: {len(bad)} cells differ, first at {bad[0]}")
            st = stats_array(lat.stats(0, MEDIUM_CHECK_STEPS))
            if not np.array_equal(st, wst):
                s0 = int(np.argwhere((st != wst).any(axis=1))[0, 0])
                pytest.fail(f"rho={lt.rho}: counts differ from step {s0}: {st[s0]} vs {wst[s0]}")
    finally:
        for lat in lats:
            lat.close()


# --- the 32768 x 32768 workload, whole lattice ------------------------------

LARGE_CHECK_STEPS = 64


@pytest.fixture(scope="module")
def large_reference():
    """The oracle's run of the 32768 x 32768 lattice (rho 0.30, seed 7) for
    64 steps: initial and final cells and every step's counts."""
    lt = workloads.LARGE.lattices[0]
    say(f"oracle: 32768^2 init + {LARGE_CHECK_STEPS} steps, {HOST_THREADS} threads")
    g0 = oracle.init_cells(lt.n, lt.seed, lt.rho)
    want, wst = oracle.run(g0, LARGE_CHECK_STEPS, n_threads=HOST_THREADS)
    return g0, want, wst


@pytest.mark.parametrize("layout", LAYOUTS)
def test_large_whole_lattice(B, layout, large_reference):
    """32768 x 32768 in the tuned launch shape the benchmark times (the
    streaming kernel's, or the tile kernel's when it was faster): 64 steps,
    every cell and all 64 count rows against
    the whole-lattice oracle."""
    import bench
    lt = workloads.LARGE.lattices[0]
    g0, want, wst = large_reference
    tun = bench.load_tuning(layout, lt.n)
    res = bench.load_resident_steps(layout, lt.n)
    say(f"large whole lattice layout={layout} tuning={tun} resident={res}")
    with make(B, lt.n, lt.rho, lt.seed, layout, cap=LARGE_CHECK_STEPS, tuning=tun) as lat:
        if res:
            lat.set_resident(res)
        lat.step(LARGE_CHECK_STEPS)
        st = stats_array(lat.stats(0, LARGE_CHECK_STEPS))
        got = lat.cells()
    if not np.array_equal(st, wst):
        s0 = int(np.argwhere((st != wst).any(axis=1))[0, 0])
        pytest.fail(f"counts differ from step {s0}: {st[s0]} vs {wst[s0]}")
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        pytest.fail(f"{len(bad)} cells differ, first at {bad[0]}")


# --- the 32768 x 32768 workload, sampled windows --------------------------

def window(g, i0, j0, size):
    n = g.shape[0]
    rows = np.arange(i0, i0 + size) % n
    cols = np.arange(j0, j0 + size) % n
    return g[np.ix_(rows, cols)]


@pytest.mark.parametrize("layout", LAYOUTS)
def test_large_sampled_windows(B, layout, large_reference):
    """32768 x 32768, rho 0.30, seed 7, in the launch shape the benchmark
    times: 48 steps, then 12 windows of 64 x 64 (corners, edges, interior)
    checked against the oracle on padded windows, and every step's counts
    against the whole-lattice oracle."""
    n, rho, seed, steps, W = 32768, 0.30, 7, 48, 64
    say(f"large sampled n={n} layout={layout}")
    g0, _, wst = large_reference
    import bench
    with make(B, n, rho, seed, layout, cap=steps, tuning=bench.load_tuning(layout, n)) as lat:
        res = bench.load_resident_steps(layout, n)
        if res:
            lat.set_resident(res)
        lat.step(steps)
        got = lat.cells()
        st = stats_array(lat.stats(0, steps))
    assert np.array_equal(st, wst[:steps])
    rng = np.random.default_rng(7)
    picks = [(0, 0), (0, n - W), (n - W, 0), (n - W, n - W), (n // 2, n // 2 - 32)]
    picks += [tuple(int(x) for x in rng.integers(0, n, size=2)) for _ in range(7)]
    for i0, j0 in picks:
        pad = window(g0, i0 - steps, j0 - steps, W + 2 * steps)
        ref, _ = oracle.run(pad, steps)
        assert np.array_equal(window(got, i0, j0, W), ref[steps:steps + W, steps:steps + W]), \
            (i0, j0)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_klein_large(B, layout, large_reference):
    """32768 x 32768 Klein bottle in the benchmark's launch shape (the tile
    kernel's when it was faster), 40 steps: every cell and every step's
    counts against the whole-lattice Klein oracle; every row keeps its LR
    cars and every column pair (j, N-1-j) its TB cars (a TB car crossing
    the glued edge changes column j for N-1-j)."""
    import bench
    n, rho, seed, steps = 32768, 0.30, 7, 40
    g0 = large_reference[0]
    tun = bench.load_tuning(layout, n)
    res = bench.load_resident_steps(layout, n, None, 1, B.BML_TOPO_KLEIN)
    say(f"klein large n={n} layout={layout} tuning={tun} resident={res}")
    with make(B, n, rho, seed, layout, cap=steps) as lat:
        lat.set_topology(B.BML_TOPO_KLEIN)
        if tun:
            lat.set_tuning(*tun)
        if res:
            lat.set_resident(res)
        lat.step(steps)
        got = lat.cells()
        st = stats_array(lat.stats(0, steps))
    assert (st[:, 0] == oracle.count(g0, 1)).all() and (st[:, 2] == oracle.count(g0, 2)).all()
    assert np.array_equal((got == 1).sum(axis=1), (g0 == 1).sum(axis=1))
    tb_got, tb0 = (got == 2).sum(axis=0), (g0 == 2).sum(axis=0)
    assert np.array_equal(tb_got + tb_got[::-1], tb0 + tb0[::-1])
    assert not np.array_equal(tb_got, tb0)      # some TB cars crossed the glued edge
    say(f"oracle: 32768^2 Klein {steps} steps, {HOST_THREADS} threads")
    want, wst = oracle.run(g0, steps, n_threads=HOST_THREADS, topology=oracle.KLEIN)
    if not np.array_equal(st, wst):
        s0 = int(np.argwhere((st != wst).any(axis=1))[0, 0])
        pytest.fail(f"counts differ from step {s0}: {st[s0]} vs {wst[s0]}")
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        pytest.fail(f"{len(bad)} cells differ, first at {bad[0]}")


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rect_large_sampled_windows(B, layout):
    """The rectangular workload (8192 rows x 32768 columns, rho_LR 0.20,
    rho_TB 0.10, seed 11) in the benchmark's tuned launch shape, 40 steps:
    windows of 64 x 64 (corners, edges, interior) against the oracle on
    padded windows; per-row LR and per-column TB counts conserved."""
    import bench
    lt = workloads.RECT.lattices[0]
    rows, cols, steps, W = lt.n, lt.cols, 40, 64
    say(f"rect large {rows}x{cols} layout={layout}")
    g0 = oracle.init_cells_asym(rows, cols, lt.seed, lt.rho_lr, lt.rho_tb)
    with B.Lattice(rows, seed=lt.seed, cols=cols, rho_lr=lt.rho_lr, rho_tb=lt.rho_tb,
                   layout=layout, stats_cap=steps) as lat:
        tun = bench.load_tuning(layout, f"{rows}x{cols}")
        if tun:
            lat.set_tuning(*tun)
        res = bench.load_resident_steps(layout, f"{rows}x{cols}")
        if res:
            lat.set_resident(res)
        lat.step(steps)
        got = lat.cells()
        st = stats_array(lat.stats(0, steps))
    assert (st[:, 0] == oracle.count(g0, 1)).all() and (st[:, 2] == oracle.count(g0, 2)).all()
    assert np.array_equal((got == 1).sum(axis=1), (g0 == 1).sum(axis=1))
    assert np.array_equal((got == 2).sum(axis=0), (g0 == 2).sum(axis=0))

    def win(g, i0, j0, h, w):
        return g[np.ix_(np.arange(i0, i0 + h) % rows, np.arange(j0, j0 + w) % cols)]

    rng = np.random.default_rng(75)
    picks = [(0, 0), (0, cols - W), (rows - W, 0), (rows - W, cols - W)]
    picks += [(int(rng.integers(0, rows)), int(rng.integers(0, cols))) for _ in range(6)]
    for i0, j0 in picks:
        pad = win(g0, i0 - steps, j0 - steps, W + 2 * steps, W + 2 * steps)
        ref, _ = oracle.run(pad, steps)
        assert np.array_equal(win(got, i0, j0, W, W), ref[steps:steps + W, steps:steps + W]), \
            (i0, j0)


@pytest.fixture(scope="module")
def max_lattice():
    """The largest lattice the library takes, 65504 x 65504 (4.3 GB of byte
    cells), initial state from the oracle."""
    return oracle.init_cells(65504, 99, 0.3)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_maximum_size_lattice(B, layout, max_lattice):
    """65504 x 65504 (every byte offset just below 2^32): the initial state
    and 16 steps in the default launch shape, checked on windows at the
    corners, the edges and inside against the oracle on padded windows;
    counts conserved at every step and per row / column."""
    n, steps, W = 65504, 16, 64
    g0 = max_lattice
    say(f"maximum size n={n} layout={layout}")
    with make(B, n, 0.3, 99, layout, cap=steps) as lat:
        init = lat.cells()
        assert np.array_equal(init[:W, :W], g0[:W, :W])
        assert np.array_equal(init[-W:, -W:], g0[-W:, -W:])
        assert np.array_equal(init[::4097], g0[::4097])
        del init
        lat.step(steps)
        got = lat.cells()
        st = stats_array(lat.stats(0, steps))
    assert (st[:, 0] == oracle.count(g0, 1)).all() and (st[:, 2] == oracle.count(g0, 2)).all()
    assert np.array_equal((got == 1).sum(axis=1), (g0 == 1).sum(axis=1))
    assert np.array_equal((got == 2).sum(axis=0), (g0 == 2).sum(axis=0))
    picks = [(0, 0), (0, n - W), (n - W, 0), (n - W, n - W), (n // 2, n // 2), (12345, 60000)]
    for i0, j0 in picks:
        pad = window(g0, i0 - steps, j0 - steps, W + 2 * steps)
        ref, _ = oracle.run(pad, steps)
        assert np.array_equal(window(got, i0, j0, W), ref[steps:steps + W, steps:steps + W]), \
            (i0, j0)


def test_copy_reference_kernel(B):
    """The bandwidth reference copy moves every byte, including a tail that
    is not a multiple of the grid's stride."""
    import torch
    for nbytes in (16, 4096 + 48, (1 << 24) + 16 * 12345):
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
        B.bml_copy(dst, src, nbytes, torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert torch.equal(dst[:nbytes], src)
        assert int(dst[nbytes:].sum()) == 0


def test_autotuner_candidates_match_the_oracle(B):
    """The autotuner's gate with the oracle's run as its reference: every
    candidate launch shape (strip rows, phases per pass, waves per block) of
    a joint four-lattice group must reproduce it, or tune_group raises."""
    from paper_1804_07981_amd import autotune
    specs = [(512, 0.25, 1), (512, 0.35, 2), (512, 0.38, 3), (512, 0.45, 4)]
    steps = 48
    ref = []
    for n, rho, seed in specs:
        want, wst = oracle.run(oracle.init_cells(n, seed, rho), steps, n_threads=HOST_THREADS)
        ref.append((want, wst))
    for layout in LAYOUTS:
        r = autotune.tune_group(specs, layout, "oracle-gate", strip_rows=(0, 8, 24),
                                t_phases=(2, 10, 16), waves=(1, 4), steps=steps,
                                log=say, reference=ref)
        assert len(r["all"]) == 18
