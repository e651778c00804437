"""GPU parity of the batched sweep (bml_batch_* through the C ABI) against the
CPU oracle: every lattice's cells and its per-step moved counts (the trace),
for mixed lattice sizes, both layouts, several tunings, graph capture and
replay, and lattices switched off mid-run."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads

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


def oracle_runs(ns, rhos, seeds, steps):
    lats = [oracle.init_cells(n, s, r) for n, r, s in zip(ns, rhos, seeds)]
    return oracle.run_many(lats, steps, n_threads=HOST_THREADS)


def check_batch(bt, ns, want_cells, want_stats, first_step=0):
    tr = bt.trace()
    for b, n in enumerate(ns):
        assert np.array_equal(bt.cells(b), want_cells[b]), f"lattice {b} (n={n}) cells"
        steps = want_stats[b].shape[0]
        got = tr[b, first_step:first_step + steps]
        assert np.array_equal(got[:, 0], want_stats[b][:, 1]), f"lattice {b} LR moved"
        assert np.array_equal(got[:, 1], want_stats[b][:, 3]), f"lattice {b} TB moved"
    bt.check()


MIXED = [32, 64, 96, 160, 256, 320, 992, 1024, 2048 + 96]


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("tuning", [(0, 0, 0), (8, 2, 4), (32, 8, 2), (64, 16, 4), (40, 6, 1)])
def test_mixed_sizes(B, layout, tuning):
    rng = np.random.default_rng(hash(tuning) % 2**32 + layout)
    ns = MIXED
    rhos = [float(x) for x in rng.uniform(0.15, 0.6, len(ns))]
    seeds = [int(x) for x in rng.integers(0, 2**40, len(ns))]
    steps = int(rng.integers(20, 70))
    say(f"batch mixed layout={layout} tuning={tuning} steps={steps}")
    want, wst = oracle_runs(ns, rhos, seeds, steps)
    with B.Batch(ns, rhos, seeds, layout=layout, trace_steps=128) as bt:
        bt.set_tuning(*tuning)
        bt.run(steps)
        check_batch(bt, ns, want, wst)
        for b in range(len(ns)):
            assert bt.lattice_steps(b) == steps


def test_graph_replays_match_eager(B):
    """A captured run replayed several times, with eager work and
    synchronisations in between, equals the eager runs step for step."""
    import torch
    ns = [64, 128, 224, 512]
    rhos = [0.3, 0.36, 0.42, 0.33]
    seeds = [1, 2, 3, 4]
    per, reps = 24, 4
    want, wst = oracle_runs(ns, rhos, seeds, per * reps + 5)
    with B.Batch(ns, rhos, seeds, trace_steps=256) as g:
        g.set_tuning(32, 8, 4)
        g.capture(per)
        for r in range(reps):
            g.replay()
            g.synchronize()
            x = torch.ones(1000, device="cuda").sum().item()   # eager work in between
            assert x == 1000.0
            torch.cuda.synchronize()
            want_r, wst_r = oracle_runs(ns, rhos, seeds, per * (r + 1))
            check_batch(g, ns, want_r, wst_r)
        g.run(5)   # eager continuation after the replays
        check_batch(g, ns, want, wst)


def test_set_active_freezes_lattices(B):
    ns = [96, 128, 320, 64]
    rhos = [0.3, 0.5, 0.25, 0.4]
    seeds = [7, 8, 9, 10]
    with B.Batch(ns, rhos, seeds, trace_steps=200) as bt:
        bt.set_tuning(16, 6, 2)
        bt.run(13)
        bt.set_active([1, 0, 1, 0])
        bt.run(21)
        bt.set_active([1, 1, 0, 1])
        bt.run(8)
        expect_steps = [42, 21, 34, 21]
        for b in range(len(ns)):
            assert bt.lattice_steps(b) == expect_steps[b]
            want, wst = oracle.run(oracle.init_cells(ns[b], seeds[b], rhos[b]), expect_steps[b])
            assert np.array_equal(bt.cells(b), want), b
        tr = bt.trace()
        # lattice 1 ran steps 0..12 and 34..41 of the batch; 13..33 are 0.
        _, w1 = oracle.run(oracle.init_cells(ns[1], seeds[1], rhos[1]), 21)
        assert np.array_equal(tr[1, :13, 0], w1[:13, 1])
        assert (tr[1, 13:34] == 0).all()
        assert np.array_equal(tr[1, 34:42, 0], w1[13:21, 1])
        bt.check()


def test_sweep_workload_first_steps(B):
    """The 512-lattice sweep (N log-uniform 64..1024, rho 0.2..0.5): every
    lattice's cells and moved counts after 48 steps."""
    lats = workloads.SWEEP.lattices
    ns = [l.n for l in lats]
    rhos = [l.rho for l in lats]
    seeds = [l.seed for l in lats]
    steps = 48
    want, wst = oracle_runs(ns, rhos, seeds, steps)
    with B.Batch(ns, rhos, seeds, trace_steps=steps) as bt:
        bt.run(steps)
        check_batch(bt, ns, want, wst)


def test_sweep_workload_full_length_sample(B):
    """Six lattices of the sweep (two smallest, two middle, two largest) run
    the full 4096 steps inside the whole 512-lattice batch."""
    lats = workloads.SWEEP.lattices
    ns = [l.n for l in lats]
    order = np.argsort(ns, kind="stable")
    pick = [int(order[0]), int(order[1]), int(order[255]), int(order[256]),
            int(order[-2]), int(order[-1])]
    steps = workloads.SWEEP.steps
    with B.Batch(ns, [l.rho for l in lats], [l.seed for l in lats], trace_steps=steps) as bt:
        bt.capture(512)
        for _ in range(steps // 512):
            bt.replay()
        bt.synchronize()
        tr = bt.trace()
        for b in pick:
            say(f"sweep full-length lattice {b} n={ns[b]}")
            want, wst = oracle.run(oracle.init_cells(ns[b], lats[b].seed, lats[b].rho), steps,
                                   n_threads=HOST_THREADS)
            assert np.array_equal(bt.cells(b), want), b
            assert np.array_equal(tr[b, :, 0], wst[:, 1]) and np.array_equal(tr[b, :, 1], wst[:, 3])
        bt.check()


def test_batch_errors(B):
    with pytest.raises(B.BmlError) as e:
        B.bml_batch_arena_bytes([64, 48], 1)
    assert e.value.code == B.BML_EINVAL
    with B.Batch([64], [0.3], [1], trace_steps=8) as bt:
        with pytest.raises(B.BmlError):
            bt.set_tuning(0, 3, 0)
        with pytest.raises(B.BmlError):
            bt.replay()          # nothing captured
        with pytest.raises(B.BmlError):
            bt.run(-1)
        bt.run(20)               # past the trace: not recorded, still stepped
        assert bt.lattice_steps(0) == 20
        want, _ = oracle.run(oracle.init_cells(64, 1, 0.3), 20)
        assert np.array_equal(bt.cells(0), want)


# --- register-resident runs (one launch per run, lattices in VGPRs) ---------

# every width W = N / 32 from 1 to 32 (odd W: a half wavefront at the
# bottom of each lattice), twice, plus 17 lattices of 64 x 64 (more than the
# 16 one-wave lattices a workgroup holds)
EVERY_WIDTH = [32 * w for w in range(1, 33)] * 2 + [64] * 17


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("split", [0, 16, 64])
def test_resident_every_width(B, layout, split):
    """Every width, whole lattices or (split > 0) the most expensive ones cut
    into slabs with `split` halo rows; 37 steps (with slabs: launches of
    `split` steps and a shorter last one)."""
    rng = np.random.default_rng(77 + layout + split)
    ns = EVERY_WIDTH
    rhos = [float(x) for x in rng.uniform(0.1, 0.7, len(ns))]
    seeds = [int(x) for x in rng.integers(0, 2**40, len(ns))]
    steps = 37
    say(f"resident every width layout={layout} split={split} lattices={len(ns)} steps={steps}")
    want, wst = oracle_runs(ns, rhos, seeds, steps)
    with B.Batch(ns, rhos, seeds, layout=layout, trace_steps=64) as bt:
        bt.set_resident(1024, split)
        assert bt.resident
        bt.run(steps)
        check_batch(bt, ns, want, wst)
        assert all(bt.lattice_steps(b) == steps for b in range(len(ns)))


def test_resident_and_streaming_agree_in_runs(B):
    """Runs of several lengths alternate between the register-resident and
    the streaming kernel on the same batch; the result is the oracle's."""
    ns = [96, 352, 608, 1024, 736]
    rhos = [0.33, 0.38, 0.29, 0.41, 0.36]
    seeds = [11, 12, 13, 14, 15]
    runs = [(1024, 9), (0, 14), (1024, 1), (0, 3), (1024, 30)]
    total = sum(k for _, k in runs)
    want, wst = oracle_runs(ns, rhos, seeds, total)
    with B.Batch(ns, rhos, seeds, trace_steps=total) as bt:
        for max_n, k in runs:
            bt.set_resident(max_n)
            assert bt.resident == (max_n >= 1024)
            bt.run(k)
        check_batch(bt, ns, want, wst)


def test_resident_slabs_on_the_sweep(B):
    """The 512-lattice sweep with its largest lattices cut into slabs of
    32 halo rows: 100 steps (launches of 32, 32, 32 and 4), every lattice's
    cells and moved counts."""
    lats = workloads.SWEEP.lattices
    ns = [l.n for l in lats]
    rhos = [l.rho for l in lats]
    seeds = [l.seed for l in lats]
    steps = 100
    want, wst = oracle_runs(ns, rhos, seeds, steps)
    with B.Batch(ns, rhos, seeds, trace_steps=steps) as bt:
        bt.set_resident(1024, 32)
        bt.run(steps)
        check_batch(bt, ns, want, wst)
    with B.Batch([64], [0.3], [1], trace_steps=8) as bt:
        for bad in (-16, 8, 24, 256):
            with pytest.raises(B.BmlError) as e:
                bt.set_resident(1024, bad)
            assert e.value.code == B.BML_EINVAL


def test_resident_mode_boundary(B):
    """The mode follows the largest lattice: 1024 runs resident, 1056 does
    not; a lower limit switches a batch back to streaming.  Both sides match
    the oracle."""
    for ns, limit, resident in (([1024, 64], 1024, True), ([1056, 64], 1024, False),
                                ([544, 512], 512, False), ([512, 480], 512, True)):
        rhos = [0.35] * len(ns)
        seeds = [3, 4]
        want, wst = oracle_runs(ns, rhos, seeds, 11)
        with B.Batch(ns, rhos, seeds, trace_steps=16) as bt:
            bt.set_resident(limit)
            assert bt.resident == resident, (ns, limit)
            bt.run(11)
            check_batch(bt, ns, want, wst)
    with B.Batch([64], [0.3], [1], trace_steps=8) as bt:
        for bad in (-1, 1056):
            with pytest.raises(B.BmlError) as e:
                bt.set_resident(bad)
            assert e.value.code == B.BML_EINVAL


@pytest.mark.parametrize("split", [0, 32])
def test_resident_graph_with_retired_lattices(B, split):
    """A captured resident run keeps its grid while lattices retire: the
    active ones are re-binned, the rest padded.  Replays, eager runs and an
    empty active set all match the oracle (with slabs: 16-step replays of
    one launch each, 5 eager steps)."""
    ns = [64] * 20 + [96, 96, 480, 1024, 992]
    rng = np.random.default_rng(5)
    rhos = [float(x) for x in rng.uniform(0.2, 0.5, len(ns))]
    seeds = list(range(100, 100 + len(ns)))
    per = 16
    with B.Batch(ns, rhos, seeds, trace_steps=128) as bt:
        bt.set_resident(1024, split)
        assert bt.resident
        bt.capture(per)
        bt.replay()
        active = [1 if (b % 3) else 0 for b in range(len(ns))]
        bt.set_active(active)
        bt.replay()
        bt.set_active([0] * len(ns))
        bt.replay()                      # nothing active: states unchanged
        bt.set_active(None)
        bt.run(5)
        bt.synchronize()
        steps = [per + (per if active[b] else 0) + 5 for b in range(len(ns))]
        tr = bt.trace()
        for b in range(len(ns)):
            assert bt.lattice_steps(b) == steps[b]
            want, wst = oracle.run(oracle.init_cells(ns[b], seeds[b], rhos[b]), steps[b])
            assert np.array_equal(bt.cells(b), want), b
            assert np.array_equal(tr[b, :per, 0], wst[:per, 1]), b
            assert np.array_equal(tr[b, :per, 1], wst[:per, 3]), b
            if active[b]:
                assert np.array_equal(tr[b, per:2 * per, 0], wst[per:2 * per, 1]), b
                assert np.array_equal(tr[b, per:2 * per, 1], wst[per:2 * per, 3]), b
            else:
                assert (tr[b, per:2 * per] == 0).all(), b
            assert (tr[b, 2 * per:3 * per] == 0).all(), b
            assert np.array_equal(tr[b, 3 * per:3 * per + 5, 0], wst[-5:, 1]), b
        bt.check()


def test_resident_density_extremes(B):
    """Empty, nearly empty (single cars crossing every wavefront boundary
    and the periodic edges), nearly full and full lattices, with wide and
    narrow rows and half-wavefront bottoms."""
    ns, rhos = [], []
    for n in (1024, 992, 96, 32, 64):
        for rho in (0.0, 0.002, 0.95, 1.0):
            ns.append(n)
            rhos.append(rho)
    seeds = list(range(len(ns)))
    steps = 150
    want, wst = oracle_runs(ns, rhos, seeds, steps)
    with B.Batch(ns, rhos, seeds, trace_steps=steps) as bt:
        assert bt.resident
        bt.run(steps)
        check_batch(bt, ns, want, wst)


def test_resident_tuner_gate_with_the_oracle(B):
    """The resident autotuner's gate with the oracle as its reference: every
    slab halo candidate must reproduce the oracle's moved counts and cells
    of a batch with lattices taller than a workgroup, or tune_resident
    raises."""
    from paper_1804_07981_amd import autotune
    ns = [1024, 544, 96, 768, 64]
    rhos = [0.3, 0.36, 0.4, 0.33, 0.5]
    seeds = [21, 22, 23, 24, 25]
    steps = 40
    want, wst = oracle_runs(ns, rhos, seeds, 2 * steps)
    trace = np.zeros((len(ns), 2 * steps, 2), dtype=np.uint32)
    for b in range(len(ns)):
        trace[b, :, 0] = wst[b][:, 1]
        trace[b, :, 1] = wst[b][:, 3]
    ref = (trace, [want[0], want[len(ns) // 2], want[-1]])
    r = autotune.tune_resident(ns, rhos, seeds, "oracle-gate", splits=(16, 48, 112),
                               steps=steps, log=say, reference=ref)
    assert len(r["all"]) == 3 and all(x["exact"] for x in r["all"])
