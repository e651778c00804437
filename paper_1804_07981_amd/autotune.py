"""Autotuner for the BML step kernels.

For a lattice size and layout (or a batch of lattices) it times candidate
launch shapes -- strip height, phases per HBM pass (temporal-block depth)
and waves per block -- with HIP events on the library's stream, and keeps
the fastest.  Every candidate must reproduce a reference -- final cells and
every per-step count, bit for bit (the bit-exactness gate).  The caller
passes the reference (the test suite passes the CPU oracle's run); without
one, the first candidate's run is the reference.  The launch shape never
changes the result, so a candidate that differs from the reference, or
whose car counts are not conserved (BML_ECORRUPT), is a bug: the tuner
writes what it knows (failures.dump_corruption) and raises instead of
moving on to the next candidate.  Results go to a JSON cache keyed by GPU
architecture, layout and size, which `Lattice`/`Batch` users (and bench.py)
read back.

For the register-resident batch kernel it picks the slab halo (split_steps)
of lattices taller than a workgroup.

Usage: python -m paper_1804_07981_amd.autotune --sizes 4096 32768 [--medium] [--batch]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys

import numpy as np
import torch

from . import _lib as L
from .batch import Batch
from .failures import dump_corruption
from .lattice import Lattice, step_group


class TuningMismatch(RuntimeError):
    """A candidate launch shape gave other cells or counts than the reference."""


CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
MODEL2_COIN_SEED = 0x5EED       # coin stream of the Model II candidates


def arch() -> str:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def key(layout: int, n, model: int = 1, topology: int = 0) -> str:
    """Cache key: arch/layout/size, with a /model2 or /model3 suffix for
    Models II and III and /klein for the Klein bottle."""
    return (f"{arch()}/{'u8' if layout == L.BML_LAYOUT_U8 else 'bp'}/{n}"
            + (f"/model{model}" if model != 1 else "")
            + ("/klein" if topology != 0 else ""))


def load(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(cache: dict, path: str = CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(layout: int, n, path: str = CACHE):
    """(tile_rows, t_phases, waves_per_block) from the cache, or None."""
    e = load(path).get(key(layout, n))
    if not e:
        return None
    return int(e["tile_rows"]), int(e["t_phases"]), int(e["waves_per_block"])


def _stats_array(rec):
    return np.stack([rec["n_lr"], rec["moved_lr"], rec["n_tb"], rec["moved_tb"]], axis=1)


def _checked_run(lat, steps: int, where: str, extra: dict):
    """(cells, counts) of a lattice after its run; on BML_ECORRUPT the
    evidence is written and the error re-raised."""
    try:
        return lat.cells(), _stats_array(lat.stats(0, steps))
    except L.BmlError as e:
        if e.code == L.BML_ECORRUPT:
            dump_corruption(e, lat, where, extra)
        raise


def _same(a, b) -> bool:
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _candidates(strip_rows, t_phases, waves, resident):
    """Launch shapes to time: the streaming kernel's (tile_rows, t_phases,
    waves_per_block), then the register-resident tile kernel's steps per
    launch."""
    return ([("stream", c) for c in itertools.product(strip_rows, t_phases, waves)]
            + [("resident", k) for k in resident])


def _best(results):
    """The fastest streaming tuning, with resident_steps = the tile kernel's
    steps per launch when one of those candidates is faster still (else 0)."""
    stream = [r for r in results if "resident_steps" not in r]
    res = [r for r in results if "resident_steps" in r]
    best = dict(max(stream, key=lambda r: r["gcups"])) if stream else {}
    best["resident_steps"] = 0
    if res:
        rb = max(res, key=lambda r: r["gcups"])
        best["resident_gcups"] = rb["gcups"]
        if not stream or rb["gcups"] > best["gcups"]:
            best["resident_steps"] = rb["resident_steps"]
    return best


def tune_lattice(n: int, layout: int, strip_rows=(0, 8, 16, 32, 64, 128, 256),
                 t_phases=(2, 4, 8, 12, 16), waves=(2, 4), steps: int | None = None,
                 rho: float = 0.3, seed: int = 7, log=print, shape: dict | None = None,
                 model: int = 1, reference=None, resident=(), topology: int = 0) -> dict:
    """Fastest (tile_rows, t_phases, waves_per_block) for an n x n lattice, or
    n rows x shape["cols"] with the draw in `shape` (Lattice keywords), under
    update rule `model` (1, 2 for Model II, 3 for Model III) on `topology`
    (BML_TOPO_TORUS or BML_TOPO_KLEIN), and whether the
    register-resident tile kernel with one of the steps per launch in
    `resident` beats it.  `reference`: the (cells, counts[steps][4]) every
    candidate must reproduce (default: the first candidate's run)."""
    shape = shape or {}
    cells = n * shape.get("cols", n)
    if steps is None:
        # about 4e9 cell-steps per measurement, at least 48 steps
        steps = int(max(48, min(2000, 4e9 / cells)))
        steps -= steps % 48
    ref = reference
    results = []
    size = f"{n}x{shape['cols']}" if "cols" in shape else f"{n}"
    for kind, cand in _candidates(strip_rows, t_phases, waves, resident):
        with Lattice(n, rho, seed, layout=layout, stats_cap=steps, **shape) as lat:
            if topology != 0:
                lat.set_topology(topology)
            if model != 1:
                lat.set_model(model, MODEL2_COIN_SEED)
            if kind == "stream":
                tr, tp, w = cand
                lat.set_tuning(tr, tp, w)
                desc = f"rows={tr} T={tp} w={w}"
            else:
                lat.set_resident(cand)
                desc = f"resident K={cand}"
            lat.step(steps)                      # warm-up (and the checked run)
            got = _checked_run(lat, steps, f"tune-{size}",
                               {"candidate": list(cand) if kind == "stream" else ["resident", cand], "rho": rho, "seed": seed})
            if ref is None:
                ref = got
            if not _same(got, ref):
                raise TuningMismatch(f"n={size} layout={layout}: candidate {desc} differs "
                                     "from the reference")
            # timed: whole launches of the candidate
            timed = steps if kind == "stream" else -(-steps // cand) * cand
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(lat.stream)
            lat.step(timed)
            e1.record(lat.stream)
            torch.cuda.synchronize()
            dt = e0.elapsed_time(e1) / 1e3
        gcups = cells * timed / dt / 1e9
        results.append({"tile_rows": tr, "t_phases": tp, "waves_per_block": w,
                        "gcups": gcups, "exact": True} if kind == "stream" else
                       {"resident_steps": cand, "gcups": gcups, "exact": True})
        log(f"  n={size} layout={layout} {desc}: {gcups:.0f} GCUPS")
    return {"best": _best(results), "all": results, "steps": steps}


def tune_group(specs, layout: int, name: str, strip_rows=(0, 4, 8, 12, 16, 24, 32, 48),
               t_phases=(8, 10, 12, 14, 16), waves=(2, 4), steps: int = 480, log=print,
               model: int = 1, reference=None, make_lattice=Lattice, step=step_group,
               resident=(), topology: int = 0) -> dict:
    """Fastest common tuning for lattices (n, rho, seed) of one size that are
    advanced together by joint launches (bml_step_group): a launch spreads
    the strips of all of them over the device, so the best strip height
    differs from a lone lattice's.  `reference`: one (cells, counts[steps][4])
    pair per lattice, the run every candidate must reproduce (default: the
    first candidate's).  `resident`: steps per launch of the register-resident
    tile kernel to try as well.  A candidate whose counts are not conserved,
    or that differs from the reference, stops the tuning (see the module
    docstring).
    make_lattice / step: the Lattice constructor and the joint step (stand-ins
    in the host-side tests)."""
    ref = reference
    results = []
    cells = float(sum(n * n for n, _, _ in specs))
    for kind, cand in _candidates(strip_rows, t_phases, waves, resident):
        stream = torch.cuda.Stream() if torch.cuda.is_available() else None
        lats = [make_lattice(n, rho, seed, layout=layout, stats_cap=steps, stream=stream)
                for n, rho, seed in specs]
        try:
            for lat in lats:
                if topology != 0:
                    lat.set_topology(topology)
                if model != 1:
                    lat.set_model(model, MODEL2_COIN_SEED)
                if kind == "stream":
                    tr, tp, w = cand
                    lat.set_tuning(tr, tp, w)
                    desc = f"rows={tr} T={tp} w={w}"
                else:
                    lat.set_resident(cand)
                    desc = f"resident K={cand}"
            step(lats, steps)                        # warm-up (and the checked run)
            got = [_checked_run(lat, steps, f"tune-{name}",
                                {"candidate": list(cand) if kind == "stream" else ["resident", cand], "lattice_index": i,
                                 "spec": list(specs[i]), "group": [list(x) for x in specs]})
                   for i, lat in enumerate(lats)]
            if ref is None:
                ref = got
            for i, (a, b) in enumerate(zip(got, ref)):
                if not _same(a, b):
                    raise TuningMismatch(
                        f"group {name} layout={layout}: candidate {desc} differs from the "
                        f"reference on lattice {i} {specs[i]}")
            # timed: whole launches of the candidate
            timed = steps if kind == "stream" else -(-steps // cand) * cand
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            step(lats, timed)
            e1.record(stream)
            torch.cuda.synchronize()
            dt = e0.elapsed_time(e1) / 1e3
        finally:
            for lat in lats:
                lat.close()
        gcups = cells * timed / dt / 1e9
        results.append({"tile_rows": tr, "t_phases": tp, "waves_per_block": w,
                        "gcups": gcups, "exact": True} if kind == "stream" else
                       {"resident_steps": cand, "gcups": gcups, "exact": True})
        log(f"  group {name} layout={layout} {desc}: {gcups:.0f} GCUPS")
    return {"best": _best(results), "all": results, "steps": steps}


def tune_batch(ns, rhos, seeds, name: str, strip_rows=(16, 32, 64, 128),
               t_phases=(4, 8, 12, 16), waves=(2, 4), steps: int = 256, log=print,
               reference=None) -> dict:
    """Fastest batch tuning for a set of lattices.  Every candidate's trace
    (per-step moved counts of every lattice over 2 x steps) and the cells of
    three lattices must equal `reference` (default: the first candidate's);
    car counts are recounted after the run (bml_batch_check)."""
    ref = reference
    results = []
    cells = float(np.sum(np.asarray(ns, dtype=np.float64) ** 2))
    for sr, tp, w in itertools.product(strip_rows, t_phases, waves):
        with Batch(ns, rhos, seeds, trace_steps=2 * steps) as bt:
            bt.set_resident(0)           # the streaming kernel's launch shapes
            bt.set_tuning(sr, tp, w)
            bt.run(steps)
            bt.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(bt.stream)
            bt.run(steps)
            e1.record(bt.stream)
            bt.synchronize()
            dt = e0.elapsed_time(e1) / 1e3
            bt.check()
            got = (bt.trace(), [bt.cells(b) for b in (0, len(ns) // 2, len(ns) - 1)])
        if ref is None:
            ref = got
        if not (np.array_equal(got[0], ref[0])
                and all(np.array_equal(a, b) for a, b in zip(got[1], ref[1]))):
            raise TuningMismatch(f"batch {name}: candidate rows={sr} T={tp} w={w} differs "
                                 "from the reference")
        gcups = cells * steps / dt / 1e9
        results.append({"tile_rows": sr, "t_phases": tp, "waves_per_block": w,
                        "gcups": gcups, "exact": True})
        log(f"  batch {name} rows={sr} T={tp} w={w}: {gcups:.0f} GCUPS")
    return {"best": max(results, key=lambda r: r["gcups"]), "all": results, "steps": steps}


def resident_key(name: str) -> str:
    return f"{arch()}/resident/{name}"


def tune_resident(ns, rhos, seeds, name: str, splits=(32, 48, 64, 80, 96),
                  steps: int = 512, log=print, reference=None) -> dict:
    """Fastest slab halo (split_steps) of the register-resident batch kernel
    for a set of lattices.  Every candidate's trace over 2 x steps and the
    cells of three lattices must equal `reference` (default: the first
    candidate's); car counts are recounted (bml_batch_check)."""
    ref = reference
    results = []
    cells = float(np.sum(np.asarray(ns, dtype=np.float64) ** 2))
    for sp in splits:
        with Batch(ns, rhos, seeds, trace_steps=2 * steps) as bt:
            bt.set_resident(1024, sp)
            if not bt.resident:
                raise ValueError(f"batch {name}: lattices too large for the resident kernel")
            bt.run(steps)
            bt.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(bt.stream)
            bt.run(steps)
            e1.record(bt.stream)
            bt.synchronize()
            dt = e0.elapsed_time(e1) / 1e3
            bt.check()
            got = (bt.trace(), [bt.cells(b) for b in (0, len(ns) // 2, len(ns) - 1)])
        if ref is None:
            ref = got
        if not (np.array_equal(got[0], ref[0])
                and all(np.array_equal(a, b) for a, b in zip(got[1], ref[1]))):
            raise TuningMismatch(f"batch {name}: resident candidate split={sp} differs from "
                                 "the reference")
        gcups = cells * steps / dt / 1e9
        results.append({"split": sp, "gcups": gcups, "exact": True})
        log(f"  resident {name} split={sp}: {gcups:.0f} GCUPS")
    return {"best": max(results, key=lambda r: r["gcups"]), "all": results, "steps": steps}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="tune the BML step kernels")
    ap.add_argument("--sizes", type=int, nargs="*", default=[4096, 32768])
    ap.add_argument("--layouts", nargs="*", default=["u8", "bp"])
    ap.add_argument("--batch", action="store_true", help="also tune the 512-lattice sweep")
    ap.add_argument("--rect", action="store_true",
                    help="also tune the rectangular, asymmetric workload lattice")
    ap.add_argument("--medium", action="store_true",
                    help="also tune the four 4096x4096 lattices advanced by joint launches")
    ap.add_argument("--cache", default=CACHE)
    ap.add_argument("--quick", action="store_true", help="fewer candidates")
    ap.add_argument("--model", type=int, choices=[1, 2, 3], default=1,
                    help="update rule of the tuned runs: 1, 2 (Model II) or 3 (Model III)")
    ap.add_argument("--klein", action="store_true",
                    help="tune on the Klein bottle (the model of Sec. 2 only)")
    args = ap.parse_args(argv)
    m = args.model
    topo = L.BML_TOPO_KLEIN if args.klein else L.BML_TOPO_TORUS
    if args.klein and m != 1:
        ap.error("--klein: the model of Sec. 2 only")
    torch.cuda.set_device(0)
    cache = load(args.cache)
    kw = dict(strip_rows=(0, 64, 256), t_phases=(4, 8, 16), waves=(4,)) if args.quick else {}
    # the register-resident tile kernel: the model of Sec. 2 and Model III,
    # 1024-column tiles
    res = (16, 24, 28, 32) if m in (1, 3) else ()
    tiles = lambda rows, cols: res if rows % 32 == 0 and cols % 256 == 0 else ()  # noqa: E731
    for n in args.sizes:
        for lay in args.layouts:
            layout = L.BML_LAYOUT_U8 if lay == "u8" else L.BML_LAYOUT_BITPLANE
            r = tune_lattice(n, layout, model=m, resident=tiles(n, n), topology=topo, **kw)
            cache[key(layout, n, m, topo)] = dict(r["best"], steps=r["steps"])
            print(json.dumps({"key": key(layout, n, m, topo), **r["best"]}), flush=True)
    if args.rect:
        import workloads
        lt = workloads.RECT.lattices[0]
        for lay in args.layouts:
            layout = L.BML_LAYOUT_U8 if lay == "u8" else L.BML_LAYOUT_BITPLANE
            r = tune_lattice(lt.n, layout, rho=lt.rho, seed=lt.seed, shape=lt.kwargs(),
                             model=m, resident=tiles(lt.n, lt.cols or lt.n), topology=topo,
                             **kw)
            k = key(layout, f"{lt.n}x{lt.cols}", m, topo)
            cache[k] = dict(r["best"], steps=r["steps"])
            print(json.dumps({"key": k, **r["best"]}), flush=True)
    if args.medium:
        import workloads
        specs = [(l.n, l.rho, l.seed) for l in workloads.MEDIUM.lattices]
        for lay in args.layouts:
            layout = L.BML_LAYOUT_U8 if lay == "u8" else L.BML_LAYOUT_BITPLANE
            r = tune_group(specs, layout, workloads.MEDIUM_GROUP, model=m,
                           resident=tiles(specs[0][0], specs[0][0]), topology=topo)
            k = key(layout, workloads.MEDIUM_GROUP, m, topo)
            cache[k] = dict(r["best"], steps=r["steps"])
            print(json.dumps({"key": k, **r["best"]}), flush=True)
    if args.batch:
        import workloads
        lats = workloads.SWEEP.lattices
        r = tune_batch([l.n for l in lats], [l.rho for l in lats], [l.seed for l in lats],
                       "sweep512")
        cache[key(L.BML_LAYOUT_BITPLANE, "sweep512")] = dict(r["best"], steps=r["steps"])
        print(json.dumps({"key": key(L.BML_LAYOUT_BITPLANE, "sweep512"), **r["best"]}),
              flush=True)
        r = tune_resident([l.n for l in lats], [l.rho for l in lats], [l.seed for l in lats],
                          "sweep512")
        cache[resident_key("sweep512")] = dict(r["best"], steps=r["steps"])
        print(json.dumps({"key": resident_key("sweep512"), **r["best"]}), flush=True)
    save(cache, args.cache)
    return 0


if __name__ == "__main__":
    sys.exit(main())
