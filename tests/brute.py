"""Car-centric brute-force BML evaluator in pure Python (tiny lattices only).

Independent of the oracle's cell-centric loops: it lists the cars, decides
from the pre-phase lattice which of them move (a car moves iff the cell in
its direction of travel is EMPTY, Marzolla arXiv:1804.07981 Sec. 2), checks
that no two cars target the same cell, then applies every move at once
(synchronous update, Sec. 3).
"""
EMPTY, LR, TB = 0, 1, 2


def target(i, j, kind, rows, cols, klein=False):
    """The cell a car at (i, j) drives into.  On the Klein bottle a TB car
    leaving the bottom row re-enters the top row in the mirrored column."""
    if kind == LR:
        return i, (j + 1) % cols
    if klein and i == rows - 1:
        return 0, cols - 1 - j
    return (i + 1) % rows, j


def phase(grid, kind, klein=False):
    rows, cols = len(grid), len(grid[0])
    moves = []
    for i in range(rows):
        for j in range(cols):
            if grid[i][j] != kind:
                continue
            ti, tj = target(i, j, kind, rows, cols, klein)
            if grid[ti][tj] == EMPTY:
                moves.append(((i, j), (ti, tj)))
    targets = [t for _, t in moves]
    assert len(set(targets)) == len(targets), "two cars share a target"
    new = [list(r) for r in grid]
    for (si, sj), _ in moves:
        new[si][sj] = EMPTY
    for _, (ti, tj) in moves:
        assert new[ti][tj] == EMPTY
        new[ti][tj] = kind
    return new, len(moves)


def step(grid, klein=False):
    """One step: every LR car, then every TB car.  Returns (grid, counts)
    with counts = (n_lr, moved_lr, n_tb, moved_tb)."""
    g1, mlr = phase(grid, LR)
    n_lr = sum(c == LR for r in g1 for c in r)
    g2, mtb = phase(g1, TB, klein)
    n_tb = sum(c == TB for r in g2 for c in r)
    return g2, (n_lr, mlr, n_tb, mtb)


def run(grid, steps, klein=False):
    grid = [list(r) for r in grid]
    stats = []
    for _ in range(steps):
        grid, c = step(grid, klein)
        stats.append(c)
    return grid, stats


# --- Model II (Sec. 2): both types in one phase, random winner on conflict ---

_M64 = (1 << 64) - 1


def splitmix64(state, k):
    """k-th output of the SplitMix64 stream started at `state` (Steele, Lea
    and Flood's generator, written out here independently of the oracle)."""
    z = (state + (k + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def model2_coin(seed, step, rows, cols, i, j):
    words = (cols + 31) // 32
    z = splitmix64(seed, step * rows * words + i * words + j // 32) & 0xFFFFFFFF
    return (z >> (j % 32)) & 1          # 1: the LR car takes the contested cell


def model2_step(grid, seed, step):
    """Cars list their targets on the pre-step lattice; a target claimed by
    an LR and a TB car goes to one of them by the coin; every winner moves at
    once.  Returns (grid, (n_lr, moved_lr, n_tb, moved_tb))."""
    rows, cols = len(grid), len(grid[0])
    claims = {}
    for i in range(rows):
        for j in range(cols):
            kind = grid[i][j]
            if kind == EMPTY:
                continue
            t = target(i, j, kind, rows, cols)
            if grid[t[0]][t[1]] == EMPTY:
                claims.setdefault(t, []).append(((i, j), kind))
    moves = []
    for (ti, tj), cars in claims.items():
        assert len(cars) <= 2
        if len(cars) == 2:
            want = LR if model2_coin(seed, step, rows, cols, ti, tj) else TB
            cars = [c for c in cars if c[1] == want]
        moves.append((cars[0][0], (ti, tj), cars[0][1]))
    new = [list(r) for r in grid]
    for (si, sj), _, _ in moves:
        new[si][sj] = EMPTY
    for _, (ti, tj), kind in moves:
        new[ti][tj] = kind
    n_lr = sum(c == LR for r in new for c in r)
    n_tb = sum(c == TB for r in new for c in r)
    mlr = sum(1 for m in moves if m[2] == LR)
    return new, (n_lr, mlr, n_tb, len(moves) - mlr)


def run_model2(grid, steps, seed, step0=0):
    grid = [list(r) for r in grid]
    stats = []
    for s in range(steps):
        grid, c = model2_step(grid, seed, step0 + s)
        stats.append(c)
    return grid, stats


# --- Model III (Sec. 2): a cell may hold an LR and a TB car at once ----------

def model3_step(grid):
    """Cells hold a set of cars as bits (1 LR, 2 TB).  Every car lists its
    target on the pre-step lattice and moves iff the target holds no car;
    then all moves happen at once, so a target wanted by one car of each
    type ends with both.  Returns (grid, (n_lr, moved_lr, n_tb, moved_tb))."""
    rows, cols = len(grid), len(grid[0])
    moves = []
    for i in range(rows):
        for j in range(cols):
            for kind in (LR, TB):
                if grid[i][j] & kind:
                    ti, tj = target(i, j, kind, rows, cols)
                    if grid[ti][tj] == EMPTY:
                        moves.append(((i, j), (ti, tj), kind))
    new = [list(r) for r in grid]
    for (si, sj), _, kind in moves:
        new[si][sj] &= ~kind
    for _, (ti, tj), kind in moves:
        assert not new[ti][tj] & kind, "two cars of one type share a target"
        new[ti][tj] |= kind
    n_lr = sum(1 for r in new for c in r if c & LR)
    n_tb = sum(1 for r in new for c in r if c & TB)
    mlr = sum(1 for m in moves if m[2] == LR)
    return new, (n_lr, mlr, n_tb, len(moves) - mlr)


def run_model3(grid, steps):
    grid = [list(r) for r in grid]
    stats = []
    for _ in range(steps):
        grid, c = model3_step(grid)
        stats.append(c)
    return grid, stats
