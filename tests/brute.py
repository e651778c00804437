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
