"""GPU checks of the allocation-free entry point, bml_step_group_static: the
same launches as bml_step_group with the stats-reduction scratch in a
static device array.  Two calls in a row (the second on fewer, smaller
lattices, starting at a later step, with a ring that wraps) must give the
cells and the counts of the handle-based entry point bit for bit."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_07981_amd as pkg
    return pkg


def say(msg):
    print(msg, flush=True)


def run_both(B, n, layout, seeds, rho, pre_steps, steps, t_phases, cap):
    """Steps len(seeds) lattices of n x n by `steps` after `pre_steps`, once
    through handles (bml_step_group) and once through bml_step_group_static
    on copies of the same states; returns both results."""
    import torch
    say(f"no-alloc case: n={n} layout={layout} lattices={len(seeds)} pre={pre_steps} "
        f"steps={steps} t_phases={t_phases} cap={cap}")
    stream = torch.cuda.current_stream()
    lats = [B.Lattice(n, rho, s, layout=layout, stats_cap=cap) for s in seeds]
    for lat in lats:
        lat.set_tuning(0, t_phases, 4)
    if pre_steps:
        B.step_group(lats, pre_steps)
    torch.cuda.synchronize()
    a = [lat.state_tensor().clone() for lat in lats]
    b = [torch.empty_like(x) for x in a]
    rings = [torch.full((cap * 4,), -1, dtype=torch.int32, device="cuda") for _ in seeds]
    torch.cuda.synchronize()
    B.step_group(lats, steps)
    in_b = B.bml_step_group_static(n, n, layout, a, b, rings, cap, pre_steps, steps, t_phases,
                                   stream)
    torch.cuda.synchronize()
    want_cells = [lat.cells() for lat in lats]
    keep = min(steps, cap)
    want_stats = [lat.stats(pre_steps + steps - keep, keep) for lat in lats]
    got_cells, got_stats = [], []
    for i in range(len(seeds)):
        res = (b if in_b else a)[i]
        if layout == B.BML_LAYOUT_U8:
            cells = res.cpu().numpy().reshape(n, n)
        else:
            out = torch.empty(n * n, dtype=torch.uint8, device="cuda")
            B.bml_unpack(n, res, out, stream)
            torch.cuda.synchronize()
            cells = out.cpu().numpy().reshape(n, n)
        got_cells.append(cells)
        ring = rings[i].cpu().numpy().view(np.uint32).reshape(cap, 4)
        first = pre_steps + steps - keep
        slots = [(first + j) % cap for j in range(keep)]
        got_stats.append(ring[slots])
    for lat in lats:
        lat.close()
    return want_cells, want_stats, got_cells, got_stats


def check(want_cells, want_stats, got_cells, got_stats):
    for wc, ws, gc, gs in zip(want_cells, want_stats, got_cells, got_stats):
        assert np.array_equal(gc, wc)
        ws = np.stack([ws["n_lr"], ws["moved_lr"], ws["n_tb"], ws["moved_tb"]], axis=1)
        assert np.array_equal(gs, ws)


def test_static_matches_step_group_twice(B):
    # first call: three 1024^2 byte lattices, 37 steps (passes of 4 and a
    # last pass of 1), every count kept
    check(*run_both(B, 1024, B.BML_LAYOUT_U8, [3, 4, 5], 0.33, 0, 37, 8, 64))
    # second call, smaller: one 256^2 bitplane lattice from step 5, 21 steps
    # in passes of 8 into a ring of 8 slots (it wraps)
    check(*run_both(B, 256, B.BML_LAYOUT_BITPLANE, [9], 0.4, 5, 21, 16, 8))


def test_static_rejects_bad_arguments(B):
    import torch
    n = 64
    bufs = [torch.empty(n * n, dtype=torch.uint8, device="cuda") for _ in range(2)]
    ring = torch.zeros(16, dtype=torch.int32, device="cuda")
    for count in (0, 9):
        with pytest.raises(B.BmlError) as e:
            B.bml_step_group_static(n, n, 0, [bufs[0]] * count, [bufs[1]] * count,
                                    [ring] * count, 4, 0, 1, 2)
        assert e.value.code == B.BML_EINVAL
    with pytest.raises(B.BmlError) as e:   # odd phase count
        B.bml_step_group_static(n, n, 0, [bufs[0]], [bufs[1]], [ring], 4, 0, 1, 3)
    assert e.value.code == B.BML_EINVAL
    with pytest.raises(B.BmlError) as e:   # same buffer twice
        B.bml_step_group_static(n, n, 0, [bufs[0]], [bufs[0]], [ring], 4, 0, 1, 2)
    assert e.value.code == B.BML_EINVAL
