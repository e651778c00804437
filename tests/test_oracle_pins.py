"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test pins the oracle to something other than itself: a second
formulation printed in the paper, a car-centric brute force, a textbook
special case (elementary CA rule 184), symmetries and invariants of the
model, closed-form trajectories, and the published SplitMix64 outputs.
Paper: Marzolla, arXiv:1804.07981 (Sec. 2 model and case tables, Sec. 3
synchronous update and layout, Sec. 5 select-and-mask formulation).
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import workloads
from tests import brute

EMPTY, LR, TB = 0, 1, 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- local rule ---------------------------------------------------------

def _select_and_mask(left, center, right, mover):
    """Sec. 5's branch-free form: masks are 0 or -1, combined bitwise."""
    m = lambda b: -1 if b else 0
    mask_in = m(left == mover) & m(center == EMPTY)
    mask_out = m(center == mover) & m(right == EMPTY)
    mask_keep = ~(mask_in | mask_out)
    return (mask_in & mover) | (mask_out & EMPTY) | (mask_keep & center)


@pytest.mark.parametrize("l,c,r", list(itertools.product((0, 1, 2), repeat=3)))
def test_h_rule_matches_select_and_mask(l, c, r):
    row = np.array([[l, c, r]], dtype=np.uint8)  # periodic 1x3: c sees l, r
    out, _ = oracle.phase_h(row)
    assert out[0, 1] == _select_and_mask(l, c, r, LR)


@pytest.mark.parametrize("t,c,b", list(itertools.product((0, 1, 2), repeat=3)))
def test_v_rule_matches_select_and_mask(t, c, b):
    col = np.array([[t], [c], [b]], dtype=np.uint8)
    out, _ = oracle.phase_v(col)
    assert out[1, 0] == _select_and_mask(t, c, b, TB)


# --- brute force on tiny lattices ----------------------------------------

def _check_against_brute(grid, steps):
    g = np.array(grid, dtype=np.uint8)
    bg, bstats = brute.run(grid, steps)
    og, ostats = oracle.run(g, steps)
    assert np.array_equal(og, np.array(bg, dtype=np.uint8))
    assert [tuple(int(x) for x in s) for s in ostats] == bstats


@pytest.mark.parametrize("n", range(1, 9))
def test_brute_force_random(n):
    rng = np.random.default_rng(1000 + n)
    for trial in range(40):
        p = rng.random()
        q = rng.random() * (1 - p)
        g = workloads.random_lattice(rng, n, n, p, q)
        _check_against_brute(g.tolist(), 6)


@pytest.mark.parametrize("rows,cols", [(2, 3), (3, 2), (1, 5), (5, 1), (4, 7), (7, 3)])
def test_brute_force_rectangular(rows, cols):
    rng = np.random.default_rng(rows * 31 + cols)
    for _ in range(30):
        g = workloads.random_lattice(rng, rows, cols, 0.35, 0.35)
        _check_against_brute(g.tolist(), 5)


def test_brute_force_exhaustive_2x2_and_3x3_one_step():
    for n in (2,):
        for cells in itertools.product((0, 1, 2), repeat=n * n):
            _check_against_brute(np.array(cells).reshape(n, n).tolist(), 2)
    rng = np.random.default_rng(7)
    all3 = list(itertools.product((0, 1, 2), repeat=9))
    for idx in rng.choice(len(all3), 1500, replace=False):
        _check_against_brute(np.array(all3[idx]).reshape(3, 3).tolist(), 1)


def test_brute_force_8x8_init_lattices():
    for seed in range(20):
        for rho in (0.0, 0.2, 0.3, 0.5, 0.8, 1.0):
            g = oracle.init_cells(8, seed, rho)
            _check_against_brute(g.tolist(), 12)


# --- elementary CA rule 184 ---------------------------------------------

def _rule184(ring):
    n = len(ring)
    return [(184 >> (4 * ring[(j - 1) % n] + 2 * ring[j] + ring[(j + 1) % n])) & 1
            for j in range(n)]


def test_lr_only_rows_follow_rule_184():
    """An LR-only row under the H phase is Wolfram's elementary rule 184."""
    rng = np.random.default_rng(184)
    for _ in range(200):
        n = int(rng.integers(1, 40))
        ring = (rng.random(n) < rng.random()).astype(int).tolist()
        out, moved = oracle.phase_h(np.array([ring], dtype=np.uint8) * LR)
        assert (out[0] // LR).tolist() == _rule184(ring)


def test_rule_184_stationary_flux():
    """Rule 184 on a ring of n cells with k cars reaches a state where
    exactly min(k, n-k) cars move every step (traffic flow of rule 184)."""
    rng = np.random.default_rng(1840)
    for _ in range(100):
        n = int(rng.integers(2, 48))
        k = int(rng.integers(0, n + 1))
        row = np.zeros((1, n), dtype=np.uint8)
        row[0, rng.choice(n, k, replace=False)] = LR
        _, stats = oracle.run(row, 2 * n + 4)
        assert all(int(m) == min(k, n - k) for m in stats[n:, 1])


# --- symmetries and invariants -------------------------------------------

def _tau(g):
    """Transpose and swap LR <-> TB."""
    t = g.T.copy()
    out = t.copy()
    out[t == LR] = TB
    out[t == TB] = LR
    return out


def test_vertical_is_transposed_horizontal():
    rng = np.random.default_rng(11)
    for _ in range(200):
        r, c = (int(x) for x in rng.integers(1, 12, size=2))
        g = workloads.random_lattice(rng, r, c, rng.random() * 0.5, rng.random() * 0.5)
        v, mv = oracle.phase_v(g)
        h, mh = oracle.phase_h(_tau(g))
        assert np.array_equal(v, _tau(h)) and mv == mh


def test_translation_equivariance():
    rng = np.random.default_rng(12)
    for _ in range(60):
        n = int(rng.integers(2, 24))
        g = workloads.random_lattice(rng, n, n + int(rng.integers(0, 5)), 0.2, 0.2)
        a, b = (int(x) for x in rng.integers(0, 30, size=2))
        s1, st1 = oracle.run(np.roll(g, (a, b), axis=(0, 1)), 7)
        s2, st2 = oracle.run(g, 7)
        assert np.array_equal(s1, np.roll(s2, (a, b), axis=(0, 1)))
        assert np.array_equal(st1, st2)


def test_conservation_per_row_and_column():
    rng = np.random.default_rng(13)
    for n in (5, 16, 33, 64):
        g = workloads.random_lattice(rng, n, n, 0.2, 0.2)
        out, stats = oracle.run(g, 50)
        assert np.array_equal((out == LR).sum(axis=1), (g == LR).sum(axis=1))
        assert np.array_equal((out == TB).sum(axis=0), (g == TB).sum(axis=0))
        assert (stats[:, 0] == (g == LR).sum()).all()
        assert (stats[:, 2] == (g == TB).sum()).all()


@pytest.mark.parametrize("kind", [LR, TB])
@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 32])
def test_lone_car_returns_after_n_steps(kind, n):
    g = workloads.lone_car(n, kind, n // 2, n // 3)
    out, stats = oracle.run(g, n)
    assert np.array_equal(out, g)
    moving = 1 if n > 1 else 0
    want = (1, moving, 0, 0) if kind == LR else (0, 0, 1, moving)
    assert all(tuple(int(x) for x in s) == want for s in stats)
    if n > 2:
        mid, _ = oracle.run(g, 1)
        i, j = n // 2, n // 3
        expect = (i, (j + 1) % n) if kind == LR else ((i + 1) % n, j)
        assert mid[expect] == kind and mid.sum() == kind


@pytest.mark.parametrize("lattice", ["checkerboard", "rows", "rho1"])
def test_full_lattice_is_fixed_point(lattice):
    n = 12
    g = {"checkerboard": workloads.full_checkerboard(n),
         "rows": workloads.full_rows(n),
         "rho1": oracle.init_cells(n, 3, 1.0)}[lattice]
    assert (g != EMPTY).all()
    out, stats = oracle.run(g, 20)
    assert np.array_equal(out, g)
    assert (stats[:, 1] == 0).all() and (stats[:, 3] == 0).all()


def test_zero_moves_means_fixed_point_forever():
    """If a step moves nothing, the next state equals the current one, so the
    lattice is frozen for good; checked on lattices that jam."""
    for seed in range(6):
        g = oracle.init_cells(32, seed, 0.7)
        out, stats = oracle.run(g, 400)
        zero = np.nonzero((stats[:, 1] == 0) & (stats[:, 3] == 0))[0]
        if len(zero) == 0:
            continue
        t = int(zero[0])
        assert (stats[t:, 1] == 0).all() and (stats[t:, 3] == 0).all()
        at_t, _ = oracle.run(g, t + 1)
        assert np.array_equal(at_t, out)


def test_car_train_only_front_moves():
    row = np.array([[LR, LR, LR, EMPTY, EMPTY, EMPTY]], dtype=np.uint8)
    out, moved = oracle.phase_h(row)
    assert out.tolist() == [[LR, LR, EMPTY, LR, EMPTY, EMPTY]] and moved == 1
    col = row.T.copy() * 2
    out, moved = oracle.phase_v(col)
    assert out.T.tolist() == [[TB, TB, EMPTY, TB, EMPTY, EMPTY]] and moved == 1


def test_h_then_v_order():
    # LR at (0,0) wants (0,1); TB at (1,1)... a TB above (0,1) at (n-1,1)
    # wants (0,1) too.  H goes first, so the LR car takes the cell.
    n = 4
    g = np.zeros((n, n), dtype=np.uint8)
    g[0, 0] = LR
    g[n - 1, 1] = TB
    out, stats = oracle.run(g, 1)
    assert out[0, 1] == LR and out[n - 1, 1] == TB
    assert tuple(int(x) for x in stats[0]) == (1, 1, 1, 0)


def test_thread_count_does_not_change_result():
    g = oracle.init_cells(96, 5, 0.33)
    a, sa = oracle.run(g, 40, n_threads=1)
    for t in (2, 3, 8):
        b, sb = oracle.run(g, 40, n_threads=t)
        assert np.array_equal(a, b) and np.array_equal(sa, sb)


def test_run_many_matches_run():
    lats = [oracle.init_cells(n, n, 0.3) for n in (8, 32, 20)]
    outs, stats = oracle.run_many(lats, 30, n_threads=3)
    for g, o, s in zip(lats, outs, stats):
        a, sa = oracle.run(g, 30)
        assert np.array_equal(a, o) and np.array_equal(sa, s)


def test_checkpoint_resume():
    g = oracle.init_cells(40, 9, 0.35)
    full, sf = oracle.run(g, 70)
    mid, s1 = oracle.run(g, 30)
    end, s2 = oracle.run(mid, 40)
    assert np.array_equal(full, end)
    assert np.array_equal(sf, np.concatenate([s1, s2]))


# --- initial placement ---------------------------------------------------

def test_splitmix64_published_outputs():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_state0.txt"))
            if l.strip() and not l.startswith("#")]
    for k, hexval in rows:
        assert oracle.splitmix64(0, int(k)) == int(hexval, 16)


def test_init_cell_k_uses_kth_output():
    rho = 0.4
    thr_lr, thr_tb = oracle.thresholds(rho)
    assert thr_lr == int(rho / 2 * 2**53) and thr_tb == int(rho * 2**53)
    g = oracle.init_cells(8, 12345, rho, cols=16)
    for k in range(g.size):
        u = oracle.splitmix64(12345, k) >> 11
        want = LR if u < thr_lr else (TB if u < thr_tb else EMPTY)
        assert g.ravel()[k] == want


@pytest.mark.parametrize("rho", [0.0, 0.1, 0.3, 0.55, 1.0])
def test_init_fractions(rho):
    g = oracle.init_cells(256, 99, rho)
    n = g.size
    for kind in (LR, TB):
        p = rho / 2
        frac = (g == kind).sum() / n
        sigma = np.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(frac - p) <= 5 * sigma + 1e-12


# --- Klein bottle (top and bottom edges glued with a reversal) ------------

KLEIN = oracle.KLEIN


@pytest.mark.parametrize("rows,cols", [(1, 5), (2, 3), (3, 2), (4, 7), (5, 5), (6, 4), (8, 8),
                                       (7, 1)])
def test_klein_matches_brute_force(rows, cols):
    rng = np.random.default_rng(rows * 131 + cols)
    for _ in range(25):
        p = rng.random()
        q = rng.random() * (1 - p)
        g = workloads.random_lattice(rng, rows, cols, p, q)
        og, ost = oracle.run(g, 6, topology=KLEIN)
        bg, bst = brute.run(g.tolist(), 6, klein=True)
        assert np.array_equal(og, np.array(bg, dtype=np.uint8))
        assert [tuple(int(x) for x in s) for s in ost] == bst


@pytest.mark.parametrize("rows,cols,i,j", [(8, 8, 3, 1), (5, 12, 0, 11), (16, 9, 15, 4)])
def test_klein_lone_tb_car_comes_back_mirrored_then_home(rows, cols, i, j):
    g = np.zeros((rows, cols), np.uint8)
    g[i, j] = TB
    once, st = oracle.run(g, rows, topology=KLEIN)
    want = np.zeros_like(g)
    want[i, cols - 1 - j] = TB
    assert np.array_equal(once, want)
    assert (st[:, 3] == 1).all() and (st[:, 1] == 0).all()
    twice, _ = oracle.run(once, rows, topology=KLEIN)
    assert np.array_equal(twice, g)


def test_klein_conservation_per_row_and_column_pair():
    rng = np.random.default_rng(77)
    g = workloads.random_lattice(rng, 24, 19, 0.3, 0.3)
    out, _ = oracle.run(g, 40, topology=KLEIN)
    assert np.array_equal((out == LR).sum(axis=1), (g == LR).sum(axis=1))
    pair = lambda x: (x == TB).sum(axis=0) + (x == TB).sum(axis=0)[::-1]   # noqa: E731
    assert np.array_equal(pair(out), pair(g))


def test_klein_without_tb_cars_is_the_torus():
    rng = np.random.default_rng(5)
    g = workloads.random_lattice(rng, 12, 10, 0.5, 0.0)
    assert np.array_equal(oracle.run(g, 9, topology=KLEIN)[0], oracle.run(g, 9)[0])


# --- Model II (Sec. 2): one phase per step, random winner on conflicts ----

@pytest.mark.parametrize("rows,cols", [(1, 4), (2, 2), (3, 5), (4, 4), (5, 3), (6, 7), (8, 8),
                                       (3, 40)])
def test_model2_matches_brute_force(rows, cols):
    rng = np.random.default_rng(rows * 977 + cols)
    for trial in range(20):
        p = rng.random()
        q = rng.random() * (1 - p)
        g = workloads.random_lattice(rng, rows, cols, p, q)
        seed, step0 = int(rng.integers(0, 2**63)), int(rng.integers(0, 1000))
        og, ost = oracle.run_model2(g, 5, seed, step0)
        bg, bst = brute.run_model2(g.tolist(), 5, seed, step0)
        assert np.array_equal(og, np.array(bg, dtype=np.uint8))
        assert [tuple(int(x) for x in s) for s in ost] == bst


def test_model2_without_conflicts_is_one_phase_of_model1():
    """With only one car type nothing is ever contested: a Model II step is
    a horizontal (LR only) or vertical (TB only) phase of Model I."""
    rng = np.random.default_rng(9)
    for kind in (LR, TB):
        g = workloads.random_lattice(rng, 12, 20, 0.45 if kind == LR else 0.0,
                                     0.45 if kind == TB else 0.0)
        got, st = oracle.run_model2(g, 1, 5)
        want, moved = (oracle.phase_h if kind == LR else oracle.phase_v)(g)
        assert np.array_equal(got, want)
        assert int(st[0, 1] + st[0, 3]) == moved


def test_model2_contested_cells_get_exactly_one_car_and_a_fair_coin():
    """LR cars at (2a+1, 2b) and TB cars at (2a, 2b+1) make every cell
    (2a+1, 2b+1) an empty cell claimed by both: each step exactly one of the
    two enters, and the LR share over many steps is 1/2 within 5 sigma."""
    rows, cols = 64, 64
    lr_wins = trials = 0
    for step0 in range(0, 40, 4):
        g = np.zeros((rows, cols), np.uint8)
        g[1::2, 0::2] = LR        # left of each target
        g[0::2, 1::2] = TB        # above each target
        out, st = oracle.run_model2(g, 1, 0xC0FFEE, step0)
        targets = out[1::2, 1::2]
        assert ((targets == LR) | (targets == TB)).all()
        lr_wins += int((targets == LR).sum())
        trials += targets.size
        assert int(st[0, 1] + st[0, 3]) == targets.size
    p = lr_wins / trials
    assert abs(p - 0.5) <= 5 * np.sqrt(0.25 / trials)


def test_model2_conserves_cars_per_row_and_column():
    rng = np.random.default_rng(21)
    g = workloads.random_lattice(rng, 30, 26, 0.3, 0.3)
    out, st = oracle.run_model2(g, 50, 77)
    assert np.array_equal((out == LR).sum(axis=1), (g == LR).sum(axis=1))
    assert np.array_equal((out == TB).sum(axis=0), (g == TB).sum(axis=0))
    assert (st[:, 0] == (g == LR).sum()).all() and (st[:, 2] == (g == TB).sum()).all()


def test_model2_step_index_selects_the_coins():
    """Running 3 + 4 steps with the global step carried over equals 7 steps."""
    rng = np.random.default_rng(4)
    g = workloads.random_lattice(rng, 16, 40, 0.35, 0.35)
    a, sa = oracle.run_model2(g, 7, 11)
    b1, s1 = oracle.run_model2(g, 3, 11)
    b2, s2 = oracle.run_model2(b1, 4, 11, step0=3)
    assert np.array_equal(a, b2) and np.array_equal(sa, np.concatenate([s1, s2]))


@pytest.mark.parametrize("i0,j0", [(0, 0), (37, 70), (90, 150), (5, 180)])
def test_model2_window_with_global_coins_matches_the_whole_lattice(i0, j0):
    """After s steps a cell depends only on cells within s rows and columns
    of it, so a padded window run with the coins of its global positions
    reproduces the whole lattice's run in its middle (windows that cross the
    lattice's edges included)."""
    rows, cols, steps, w = 96, 192, 6, 24
    rng = np.random.default_rng(i0 * 31 + j0)
    g = workloads.random_lattice(rng, rows, cols, 0.3, 0.3)
    full, _ = oracle.run_model2(g, steps, 0xABCDEF, step0=11)
    r = np.arange(i0 - steps, i0 + w + steps) % rows
    c = np.arange(j0 - steps, j0 + w + steps) % cols
    pad = g[np.ix_(r, c)]
    frame = ((i0 - steps) % rows, (j0 - steps) % cols, rows, cols)
    win, _ = oracle.run_model2(pad, steps, 0xABCDEF, step0=11, frame=frame)
    want = full[np.ix_(r[steps:steps + w], c[steps:steps + w])]
    assert np.array_equal(win[steps:steps + w, steps:steps + w], want)
    # the window's own coins (no frame) generally differ
    own, _ = oracle.run_model2(pad, steps, 0xABCDEF, step0=11)
    assert (i0, j0) == (0, 0) or not np.array_equal(own, win)


# --- Model III (Sec. 2): a cell may hold an LR and a TB car at once --------

BOTH = LR | TB


def _with_both(rng, g, frac):
    g = g.copy()
    g[rng.random(g.shape) < frac] = BOTH
    return g


@pytest.mark.parametrize("rows,cols", [(1, 4), (2, 2), (3, 5), (4, 4), (5, 3), (6, 7), (8, 8),
                                       (3, 40)])
def test_model3_matches_brute_force(rows, cols):
    rng = np.random.default_rng(rows * 683 + cols)
    for trial in range(20):
        p = rng.random()
        q = rng.random() * (1 - p)
        g = _with_both(rng, workloads.random_lattice(rng, rows, cols, p, q), rng.random() * 0.3)
        og, ost = oracle.run_model3(g, 6)
        bg, bst = brute.run_model3(g.tolist(), 6)
        assert np.array_equal(og, np.array(bg, dtype=np.uint8))
        assert [tuple(int(x) for x in s) for s in ost] == bst


def test_model3_one_type_is_rule_184():
    """LR cars alone: every row is elementary CA rule 184 (Wolfram's
    numbering, bit n of 184 = new centre for neighbourhood n = 4l + 2c + r);
    TB cars alone: every column is."""
    rng = np.random.default_rng(31)
    rule = [(184 >> n) & 1 for n in range(8)]
    for kind in (LR, TB):
        g = workloads.random_lattice(rng, 14, 18, 0.5 if kind == LR else 0.0,
                                     0.5 if kind == TB else 0.0)
        got, _ = oracle.run_model3(g, 1)
        lines = (g == kind).astype(int) if kind == LR else (g == kind).astype(int).T
        want = np.zeros_like(lines)
        for r, line in enumerate(lines):
            n = len(line)
            for c in range(n):
                want[r, c] = rule[4 * line[c - 1] + 2 * line[c] + line[(c + 1) % n]]
        out = (got == kind).astype(int) if kind == LR else (got == kind).astype(int).T
        assert np.array_equal(out, want)


def test_model3_without_contested_cells_is_model2():
    """A step with no EMPTY cell wanted by both types is the same under
    Models II and III (whatever the coins)."""
    rng = np.random.default_rng(17)
    for trial in range(30):
        g = workloads.random_lattice(rng, 10, 12, 0.3, 0.3)
        while True:          # drop the TB car above each contested cell
            contested = (g == EMPTY) & (np.roll(g, 1, axis=1) == LR) & (np.roll(g, 1, axis=0) == TB)
            if not contested.any():
                break
            g[np.roll(contested, -1, axis=0)] = EMPTY
        a, sa = oracle.run_model3(g, 1)
        b, sb = oracle.run_model2(g, 1, int(rng.integers(0, 2**63)))
        assert np.array_equal(a, b) and np.array_equal(sa, sb)


def test_model3_contested_cells_take_both_cars():
    rows, cols = 32, 32
    g = np.zeros((rows, cols), np.uint8)
    g[1::2, 0::2] = LR
    g[0::2, 1::2] = TB
    out, st = oracle.run_model3(g, 1)
    assert (out[1::2, 1::2] == BOTH).all()
    assert (out[1::2, 0::2] == EMPTY).all() and (out[0::2, 1::2] == EMPTY).all()
    assert tuple(int(x) for x in st[0]) == (rows * cols // 4, rows * cols // 4,
                                            rows * cols // 4, rows * cols // 4)


def test_model3_doubly_occupied_cell_blocks_both_types_and_empties_one_car_at_a_time():
    g = np.zeros((5, 6), np.uint8)
    g[2, 2] = BOTH
    g[2, 1] = LR            # blocked by the double cell on its right
    g[1, 2] = TB            # blocked by the double cell below
    g[3, 2] = LR            # blocks the double cell's TB car
    out, st = oracle.run_model3(g, 1)
    want = np.zeros_like(g)
    want[2, 1] = LR
    want[1, 2] = TB
    want[2, 2] = TB         # its LR car left, its TB car is blocked
    want[2, 3] = LR
    want[3, 3] = LR
    assert np.array_equal(out, want)
    assert tuple(int(x) for x in st[0]) == (3, 2, 2, 0)


def test_model3_conserves_cars_per_row_and_column():
    rng = np.random.default_rng(23)
    g = _with_both(rng, workloads.random_lattice(rng, 30, 26, 0.3, 0.3), 0.05)
    out, st = oracle.run_model3(g, 60)
    assert np.array_equal((out & LR > 0).sum(axis=1), (g & LR > 0).sum(axis=1))
    assert np.array_equal((out & TB > 0).sum(axis=0), (g & TB > 0).sum(axis=0))
    assert (st[:, 0] == (g & LR > 0).sum()).all() and (st[:, 2] == (g & TB > 0).sum()).all()


# --- asymmetric placement (unequal LR and TB numbers, Sec. 2 extensions) ---

def _floor_times_2_53(x: float) -> int:
    """floor(x * 2^53) in exact rational arithmetic."""
    from fractions import Fraction
    return int(Fraction(x) * 2**53)


@pytest.mark.parametrize("rho_lr,rho_tb", [(0.1, 0.3), (0.3, 0.1), (0.0, 0.45), (0.25, 0.0),
                                           (0.6, 0.4), (1 / 3, 1 / 7)])
def test_asym_thresholds_and_cells(rho_lr, rho_tb):
    thr_lr, thr_tb = oracle.thresholds_asym(rho_lr, rho_tb)
    assert thr_lr == _floor_times_2_53(rho_lr)
    assert thr_tb == _floor_times_2_53(rho_lr + rho_tb)     # the sum rounded as IEEE double
    g = oracle.init_cells_asym(6, 40, 777, rho_lr, rho_tb)
    for k in range(g.size):
        u = oracle.splitmix64(777, k) >> 11
        want = LR if u < thr_lr else (TB if u < thr_tb else EMPTY)
        assert g.ravel()[k] == want


@pytest.mark.parametrize("rho", [0.0, 0.17, 0.37, 0.5, 1.0])
def test_asym_with_equal_halves_is_the_symmetric_draw(rho):
    assert oracle.thresholds_asym(rho / 2, rho / 2) == oracle.thresholds(rho)
    assert np.array_equal(oracle.init_cells_asym(40, 96, 3, rho / 2, rho / 2),
                          oracle.init_cells(40, 3, rho, cols=96))


@pytest.mark.parametrize("rho_lr,rho_tb", [(0.05, 0.3), (0.35, 0.15), (0.0, 0.2), (0.5, 0.5)])
def test_asym_fractions(rho_lr, rho_tb):
    g = oracle.init_cells_asym(256, 384, 41, rho_lr, rho_tb)
    n = g.size
    for kind, p in ((LR, rho_lr), (TB, rho_tb)):
        frac = (g == kind).sum() / n
        sigma = np.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(frac - p) <= 5 * sigma + 1e-12
    if rho_lr == 0:
        assert not (g == LR).any()
    if rho_lr + rho_tb == 1:
        assert not (g == EMPTY).any()


# --- bitplane definition ---------------------------------------------------

def test_pack_layout_and_roundtrip():
    g = np.zeros((2, 64), dtype=np.uint8)
    g[0, 0] = LR      # word 0 bit 0 (leftmost cell = least significant bit)
    g[0, 33] = TB     # word 1 bit 1
    g[1, 31] = LR     # row 1 word 0 bit 31
    lr, tb = oracle.pack(g)
    assert lr.tolist() == [[1, 0], [1 << 31, 0]]
    assert tb.tolist() == [[0, 2], [0, 0]]
    rng = np.random.default_rng(3)
    r = workloads.random_lattice(rng, 17, 96, 0.3, 0.3)
    assert np.array_equal(oracle.unpack(*oracle.pack(r)), r)


# --- physics sanity (qualitative) -----------------------------------------

@pytest.mark.slow
def test_fig1_free_flow_and_jam():
    """Fig. 1: at 256 x 256 after 4096 steps, rho = 0.25 flows freely and
    rho = 0.38 is jammed (most seeds; both phases can coexist near the
    critical density, so a majority of three seeds is asked for)."""
    def mean_v(rho, seed):
        g = oracle.init_cells(256, seed, rho)
        _, st = oracle.run(g, 4096, n_threads=os.cpu_count() or 1)
        cars = st[-100:, 0].astype(float) + st[-100:, 2]
        return float(((st[-100:, 1] + st[-100:, 3]) / cars).mean())
    free = [mean_v(0.25, s) for s in range(3)]
    jam = [mean_v(0.38, s) for s in range(3)]
    assert sum(v > 0.9 for v in free) >= 2
    assert sum(v < 0.05 for v in jam) >= 2
