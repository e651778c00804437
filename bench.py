#!/usr/bin/env python3
"""Benchmark of the MI355X BML step library (one GPU).

Default workload: one 32768 x 32768 lattice (rho 0.30, seed 7), 1000 steps,
uint8 cells, in the autotuned launch shape (several steps per HBM pass).  One
benchmark step is that whole job: the lattice advanced 1000 steps with every
per-step count recorded.  The initial lattice is resident in HBM before the
timed region starts (1 GiB per state buffer: far beyond the 256 MB Infinity
Cache, so the step kernel's traffic is HBM traffic).

Prints one JSON line: GCUPS (cell updates per second, one update = one cell
advanced one full step, horizontal + vertical phase), the HBM roofline of the
step kernel, the unblocked one-step-per-pass kernel on the same lattice
(`t2`), the bitplane form, the four 4096 x 4096 lattices (`medium`, bound by
the ALU and on-chip caches, not HBM), the 512-lattice density sweep, the
learned early exit, and the CPU oracle timed on the host cores.
`--workload medium|rect|sweep|early-exit` times those workloads alone.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
PROFILES = os.path.join(ROOT, "profiles")
# the sources of the streaming pass kernel, and of the register-resident
# tile kernel: a stored counter summary holds only while its kernel's hash
# is unchanged
KERNEL_SOURCES = ["paper_1804_07981_amd/csrc/bml_pass.hpp",
                  "paper_1804_07981_amd/csrc/bml_tile.hpp"]
BLOCK_SOURCES = ["paper_1804_07981_amd/csrc/bml_block.hpp"]


def kernel_hash(resident: bool = False) -> str:
    h = hashlib.sha256()
    for p in (BLOCK_SOURCES if resident else KERNEL_SOURCES):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def bytes_per_cell_step(layout: int, k: int) -> float:
    """Algorithmic HBM bytes per cell-step of one pass of k steps: the state
    is read once and written once per pass (1 byte per cell for uint8, 2 bits
    for bitplanes), shared by the k steps of the pass."""
    per_cell_pass = 2.0 if layout == 0 else 0.5
    return per_cell_pass / k


# gfx950 vector ALU: 256 CUs x 128 lanes per clock x 2.4 GHz, the rate of
# the published fp32 vector peak (157.3 TFLOP/s with an FMA counted as two).
# The unit is a full-rate 32-bit lane-op slot: plain logic ops (and, or,
# xor, three-input bit ops, moves) take one; popcount (v_bcnt_u32_b32) and
# the funnel shift (v_alignbit_b32) issue at half that rate on this chip and
# take two (profiles/valu_issue_rates.md).
ALU_PEAK_LANE_OPS = 256 * 128 * 2.4e9
# Slots per 32-cell word and step of the rule of Sec. 2: horizontal phase
# occupancy or, the right neighbour's occupancy across the word boundary (a
# funnel shift), movers and-not, arrivals (a funnel shift), update xor3;
# vertical phase emptiness nor, movers and, update xor3: 6 logic ops + 2
# funnel shifts = 10 slots; the four per-step counts are four popcount-adds
# = 8 slots.
RULE_SLOTS = 6 + 2 * 2
COUNT_SLOTS = 4 * 2
# Byte cells <-> bitplanes, in registers, per 32-cell word and pass: gather
# bit 0 and bit 1 of 32 bytes into two words and rotate the bit index
# (about 64 logic ops), and the inverse.
CONVERT_SLOTS = 128

# The paper's fastest measured runs (Sec. 7, table of mean execution times:
# rho 0.3, 1024 steps, times read as seconds), with their machines: context
# for the numbers here, not a baseline of the same workload or hardware.
PAPER_RUNS = [
    ("CUDA", "GeForce GTX 1070 (1920 cores, 1.80 GHz)", 4096, 0.768),
    ("CUDA", "GeForce GTX 1070 (1920 cores, 1.80 GHz)", 1024, 0.052),
    ("OpenMP+SIMD, 12 cores", "Xeon E5-2603 (12 cores, 1.7 GHz)", 4096, 2.292),
    ("OpenMP+SIMD, 4 cores", "Xeon E3-1220 (4 cores, 3.5 GHz)", 2048, 0.339),
    ("CUDA", "Quadro K620 (384 cores, 1.12 GHz)", 4096, 5.970),
]


def paper_context() -> dict:
    """The paper's runs above with GCUPS = N^2 * 1024 / t (derived)."""
    return {"source": "arXiv:1804.07981 Sec. 7, mean execution times, rho 0.3, 1024 steps "
                      "(seconds); GCUPS derived as N^2*1024/t",
            "runs": [{"implementation": impl, "machine": m, "n": n, "seconds": t,
                      "gcups": round(n * n * 1024 / t / 1e9, 2)}
                     for impl, m, n, t in PAPER_RUNS]}


def alu_roofline(layout: int, k: int, gcups: float, model: int = 1) -> dict:
    """Algorithmic full-rate lane-op slots per cell-step over the achieved
    GCUPS, against ALU_PEAK_LANE_OPS.  Model I and Model III (one phase of
    the same op count): RULE_SLOTS + COUNT_SLOTS per word-step.  Model II:
    about 27 logic ops for the contested-cell masks and both moves in one
    phase (two of them funnel shifts, +2), the counts, and about 38 slots
    for the word's coin hash (a 64-bit SplitMix64 output in 32-bit lane ops,
    its three multiplies at quarter rate).  The byte layout adds
    CONVERT_SLOTS per word per pass of k steps."""
    per_word = (27 + 2 + COUNT_SLOTS + 38) if model == 2 else RULE_SLOTS + COUNT_SLOTS
    per_cell_step = (per_word + (CONVERT_SLOTS / k if layout == 0 else 0.0)) / 32
    achieved = gcups * 1e9 * per_cell_step
    return {"bound": "alu", "achieved": round(achieved / 1e12, 2),
            "peak": round(ALU_PEAK_LANE_OPS / 1e12, 2), "unit": "Tlane-op/s",
            "frac": round(achieved / ALU_PEAK_LANE_OPS, 4),
            "lane_ops_per_cell_step": round(per_cell_step, 4)}


def size_key(lt):
    """Tuning-cache size key of a workload lattice: N, or ROWSxCOLS."""
    return lt.n if lt.cols is None else f"{lt.n}x{lt.cols}"


def load_tuning(layout: int, n, group: str | None = None, model: int = 1):
    """Autotuned (tile_rows, t_phases, waves_per_block): the entry for the
    group of lattices run together (e.g. the four concurrent 4096 lattices),
    else the one for a lone lattice of side n, else None.  Models II and III
    use their own entries (a /model2 or /model3 suffix) when they exist."""
    path = os.path.join(ROOT, "paper_1804_07981_amd", "tune_cache.json")
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
            lay = "u8" if layout == 0 else "bp"
            keys = ([f"gfx950/{lay}/{group}"] if group else []) + [f"gfx950/{lay}/{n}"]
            if model != 1:
                keys = [k + f"/model{model}" for k in keys] + keys
            for key in keys:
                if key in cache:
                    t = cache[key]
                    return int(t["tile_rows"]), int(t["t_phases"]), int(t["waves_per_block"])
        except (OSError, ValueError, KeyError):
            pass
    return None


def load_resident_steps(layout: int, n, group: str | None = None, model: int = 1,
                        topology: int = 0) -> int:
    """Autotuned steps per launch of the register-resident tile kernel for
    the lattice (or group) the tuning cache entry names (0: the streaming
    kernel is faster, or no entry).  Model III reads only its own (/model3)
    entries, the Klein bottle (topology 1) its own (/klein); Model II, which
    the tile kernel does not run: always 0."""
    if model == 2 or (model == 3 and topology != 0):
        return 0
    path = os.path.join(ROOT, "paper_1804_07981_amd", "tune_cache.json")
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        return 0
    lay = "u8" if layout == 0 else "bp"
    suffix = "/model3" if model == 3 else "/klein" if topology != 0 else ""
    for key in ([f"gfx950/{lay}/{group}{suffix}"] if group else []) + [f"gfx950/{lay}/{n}{suffix}"]:
        if key in cache:
            return int(cache[key].get("resident_steps", 0))
    return 0


def load_resident_split(group: str) -> int:
    """Autotuned slab halo of the register-resident batch kernel for a
    batch (0: whole lattices) from the tuning cache, else 0."""
    path = os.path.join(ROOT, "paper_1804_07981_amd", "tune_cache.json")
    try:
        with open(path) as f:
            return int(json.load(f).get(f"gfx950/resident/{group}", {}).get("split", 0))
    except (OSError, ValueError, AttributeError):
        return 0


def traffic_from_profile(name: str, tuning, launches_bytes: float, profiles: str = PROFILES,
                         resident: int = 0):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source with the same tuning (for the
    register-resident tile kernel: the same steps per launch); else None."""
    if resident:
        path = os.path.join(profiles, name.replace("pass_", "block_", 1)
                            + f"_k{resident}.traffic.json")
        try:
            with open(path) as f:
                d = json.load(f)
        except (OSError, ValueError):
            return None
        if d.get("kernel_hash") != kernel_hash(resident=True) or \
                int(d.get("probe", {}).get("resident", 0)) != resident:
            return None
        return d.get("hbm_bytes_per_launch")
    path = os.path.join(profiles, f"{name}_t{tuning[1]}.traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    p = d.get("probe", {})
    if (p.get("tile_rows"), p.get("t_phases"), p.get("waves_per_block")) != tuple(tuning):
        return None
    return d.get("hbm_bytes_per_launch")


def _pmc_per_dispatch(csv_dir: str, counter: str) -> dict:
    """{dispatch id: (kernel name, summed counter value)} from a rocprofv3
    --pmc output directory."""
    import csv
    out = {}
    for root, _, files in os.walk(csv_dir):
        for fn in files:
            if not fn.endswith("counter_collection.csv"):
                continue
            with open(os.path.join(root, fn)) as f:
                for r in csv.DictReader(f):
                    if r["Counter_Name"] != counter:
                        continue
                    d = int(r["Dispatch_Id"])
                    name, v = out.get(d, (r["Kernel_Name"], 0.0))
                    out[d] = (name, v + float(r["Counter_Value"]))
    return out


def pmc_summary(probe_log: str, fetch_dir: str, write_dir: str, profiles: str = PROFILES) -> int:
    """HBM bytes per launch of the step kernel from FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch), each scaled so that the 1 GiB copy the probe runs
    first reads as 1 GiB fetched and 1 GiB written."""
    probe = None
    with open(probe_log) as f:
        for line in f:
            if line.startswith("{") and '"probe"' in line:
                probe = json.loads(line)
    if probe is None:
        print("no probe line in " + probe_log, file=sys.stderr)
        return 1
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = _pmc_per_dispatch(d, counter)
        step_kernel = "block_kernel" if probe.get("resident") else "pass_kernel"
        copies = [v for name, v in disp.values() if "copy" in name.lower()]
        passes = [v for name, v in disp.values() if step_kernel in name]
        if not copies or not passes:
            print(f"{counter}: copy or {step_kernel} dispatches missing", file=sys.stderr)
            return 1
        copy_kib = max(copies)
        res[counter] = {"copy_kib": copy_kib, "scale": (1 << 20) / copy_kib,
                        "pass_kib_per_dispatch": sum(passes) / len(passes),
                        "dispatches": len(passes)}
    layout = 0 if probe["layout"] == "u8" else 1
    resident = int(probe.get("resident", 0))
    k = resident or probe["t_phases"] // 2
    alg = bytes_per_cell_step(layout, k) * probe["cells_per_launch"] * k
    hbm = sum(r["pass_kib_per_dispatch"] * 1024 * r["scale"] for r in res.values())
    kernel = "block_kernel" if resident else "pass_kernel"
    out = {"kernel": f"{kernel}<{probe['layout']}, K={k}>", "probe": probe,
           "kernel_hash": probe["kernel_hash"],
           "fetch_kib_per_dispatch": res["FETCH_SIZE"]["pass_kib_per_dispatch"],
           "write_kib_per_dispatch": res["WRITE_SIZE"]["pass_kib_per_dispatch"],
           "copy_calibration": {"bytes": 1 << 30,
                                "fetch_kib": res["FETCH_SIZE"]["copy_kib"],
                                "write_kib": res["WRITE_SIZE"]["copy_kib"],
                                "fetch_scale": res["FETCH_SIZE"]["scale"],
                                "write_scale": res["WRITE_SIZE"]["scale"]},
           "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": alg,
           "ratio_to_algorithmic": hbm / alg,
           "dispatches": res["FETCH_SIZE"]["dispatches"]}
    stem = (f"block_{probe['layout']}_{probe['n']}_k{resident}" if resident else
            f"pass_{probe['layout']}_{probe['n']}_t{probe['t_phases']}")
    path = os.path.join(profiles, stem + ".traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
    return 0


def copy_ceiling(B, dev, nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """GB/s (bytes read + bytes written) of a 1 GiB device copy, by torch and
    by the library's streaming copy kernel, on this device."""
    import torch
    a = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("torch_copy", lambda: b.copy_(a)),
                     ("bml_copy", lambda: B.bml_copy(b, a, nbytes,
                                                      torch.cuda.current_stream(dev)))):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def host_threads() -> int:
    """Threads the oracle may use: OMP_NUM_THREADS when set (this process's
    share of the host), else every CPU the process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "").strip()
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(lt, target_s: float = 10.0, model: int = 1, coin_seed: int = 0):
    """The oracle on a bounded sample of the workload's first lattice -- its
    first rows (at most about 3.4e7 cells), run as a periodic lattice of
    their own -- timed on all host threads and on one thread, about
    `target_s` seconds each."""
    import oracle

    def run(g, steps, threads):
        if model == 2:
            return oracle.run_model2(g, steps, coin_seed, n_threads=threads)
        if model == 3:
            return oracle.run_model3(g, steps, n_threads=threads)
        return oracle.run(g, steps, n_threads=threads)

    cols = lt.cols or lt.n
    rows = 1
    while rows * 2 * cols <= int(3.4e7) and rows * 2 <= lt.n:
        rows *= 2
    if lt.cols is None and lt.rho_lr is None:
        g = oracle.init_cells(rows, lt.seed, lt.rho, cols=cols)
    else:
        g = oracle.init_cells_asym(rows, cols, lt.seed, lt.rho_lr, lt.rho_tb)

    def timed(threads):
        t0 = time.perf_counter()
        g1, _ = run(g, 2, threads)
        cal = (time.perf_counter() - t0) / 2
        steps = max(2, min(int(target_s / max(cal, 1e-6)), 5000))
        t0 = time.perf_counter()
        run(g1, steps, threads)
        dt = time.perf_counter() - t0
        return rows * cols * steps / dt / 1e9, steps, dt

    threads = host_threads()
    v_all, s_all, t_all = timed(threads)
    v_one, s_one, t_one = timed(1)
    rule = {1: "", 2: ", Model II", 3: ", Model III"}[model]
    draw = (f"rho={lt.rho}" if lt.rho_lr is None
            else f"rho_lr={lt.rho_lr} rho_tb={lt.rho_tb}")
    return {"value": round(v_all, 3), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"first {rows} rows of the {lt.n}x{cols} lattice ({draw}, seed "
                      f"{lt.seed}) run as a periodic {rows}x{cols} lattice: {s_all} steps "
                      f"on {threads} threads in {t_all:.1f} s (plain C oracle, gcc -O3, "
                      f"OpenMP row split{rule})",
            "single_thread": {"value": round(v_one, 4), "unit": "GCUPS", "cores": 1,
                              "steps": s_one, "seconds": round(t_one, 2)},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def sweep_measure(B, workloads, dev, steps: int, warmup: int, plain_sample,
                  resident_max_n: int = 1024, split: int | None = None) -> dict:
    """512 lattices of uneven N and rho, 4096 steps each, in one batch: a
    captured 512-step graph replayed 8 times (mean of `steps` timed runs
    after `warmup`); against plain per-lattice runs through the
    single-lattice API (all lattices, or an evenly spaced sample scaled to
    all by cell count; plain_sample=0 skips them).  resident_max_n: the
    batch's register-resident limit (1024: every lattice of the sweep stays
    in registers; 0: the streaming kernel, one launch per pass); split: the
    resident slab halo (0: whole lattices, one launch per replay; None: the
    autotuned value)."""
    import numpy as np
    import torch
    wl = workloads.SWEEP
    ns = [l.n for l in wl.lattices]
    rhos = [l.rho for l in wl.lattices]
    seeds = [l.seed for l in wl.lattices]
    cells = float(np.sum(np.asarray(ns, dtype=np.float64) ** 2))
    chunk = 512
    tun = load_tuning(1, "sweep512")
    if split is None:
        split = load_resident_split("sweep512")
    times = []
    for rep in range(warmup + steps):
        with B.Batch(ns, rhos, seeds, layout=1, trace_steps=wl.steps, device=dev) as bt:
            if tun:
                bt.set_tuning(*tun)
            bt.set_resident(resident_max_n, split)
            resident = bt.resident
            bt.capture(chunk)
            bt.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(bt.stream)
            for _ in range(wl.steps // chunk):
                bt.replay()
            e1.record(bt.stream)
            bt.synchronize()
            if rep >= warmup:
                times.append(e0.elapsed_time(e1) / 1e3)
            bt.check()
    batch_s = float(np.mean(times))
    gcups = cells * wl.steps / batch_s / 1e9
    out = {"workload": wl.name, "lattices": len(ns), "steps_per_lattice": wl.steps,
           "graph_steps": chunk,
           "kernel": ("resident_kernel (registers, " + (f"slabs with {split} halo rows, "
                      f"launches of {split} steps)" if split else "one launch per replay)"))
           if resident else "batch_kernel (streaming, one launch per pass)",
           "tuning": {"resident_split": split} if resident else tun, "gcups": gcups,
           "batched_wall_s": batch_s,
           # the sweep's lattices live in registers / on-chip caches; the
           # rule's bit operations bound it
           "roofline": alu_roofline(1, 1, gcups)}
    if plain_sample == 0:
        return out
    idx = list(range(len(ns))) if plain_sample is None else list(
        np.linspace(0, len(ns) - 1, plain_sample).astype(int))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_cells = 0.0
    for b in idx:
        with B.Lattice(ns[b], rhos[b], seeds[b], layout=1, stats_cap=wl.steps, device=dev) as lat:
            lat.step(wl.steps)
            lat.stats(0, wl.steps)
        plain_cells += float(ns[b]) ** 2
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) * (cells / plain_cells)
    out.update({"plain_per_lattice_wall_s": plain_s, "plain_measured_lattices": len(idx),
                "gain": plain_s / batch_s})
    return out


def bench_sweep(args, B, workloads, dev) -> int:
    """The density sweep as its own benchmark line (GCUPS of the batch)."""
    sw = sweep_measure(B, workloads, dev, args.steps, args.warmup, args.plain_sample,
                       resident_max_n=args.resident_max_n, split=args.split)
    out = {"metric": "GCUPS (cell updates/s); density-sweep time vs plain",
           "value": round(sw["gcups"], 1),
           "unit": "GCUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(sw["batched_wall_s"] * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bitplane",
           "data": "synthetic (SplitMix64 iid lattices)",
           "config": {"workload": sw["workload"], "lattices": sw["lattices"],
                      "steps_per_lattice": sw["steps_per_lattice"],
                      "graph_steps": sw["graph_steps"], "kernel": sw["kernel"],
                      "tuning": sw["tuning"]},
           "roofline": sw["roofline"],
           "sweep": {k: sw.get(k) for k in ("batched_wall_s", "plain_per_lattice_wall_s",
                                            "plain_measured_lattices", "gain")}}
    print(json.dumps(out), flush=True)
    return 0


def bench_early_exit(args) -> int:
    """The learned early-exit density sweep (512 x 512 lattices, 141
    densities x 64 seeds, 20000 steps): labels, GPU training, held-out
    error and wall time against plain runs and the exact stop rule."""
    from paper_1804_07981_amd import early_exit as ee
    ns, rhos, seeds, split = ee.c4_lattices()
    rep = ee.experiment(ns, rhos, seeds, split, plain_sample=args.plain_sample or 96,
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    t3 = rep["batch_exact_stop_mlp"]["wall_s"]
    out = {"metric": "density-sweep wall time vs plain per-lattice full runs", "value":
           round(rep["gain_vs_plain"], 2), "unit": "x faster", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": round(t3 * 1e3, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bitplane+fp32/bf16",
           "data": "synthetic (SplitMix64 iid lattices)",
           "config": {"workload": "bml-early-exit-512x512-141rho-64seeds-20000steps"},
           "early_exit": rep}
    print(json.dumps(out), flush=True)
    return 0


def load_for(args):
    """Tuning lookup honouring --tuning."""
    if args.tuning:
        forced = tuple(args.tuning)
        return lambda lay, n, grp=None: forced
    return lambda lay, n, grp=None: load_tuning(lay, n, grp, args.model)


def measure(B, dev, wl, layout: int, steps: int, warmup: int, mode: str, load, configure,
            tuning=None, resident=None) -> dict:
    """Times `steps` runs of the whole workload (each lattice wl.steps steps)
    after `warmup` untimed ones.  mode "joint": every lattice on one stream,
    advanced together by joint launches (bml_step_group); "streams": one
    stream per lattice, their launches overlapping; "single": the current
    stream.  resident: steps per launch of the register-resident tile kernel
    (0: the streaming kernel; None: the autotuned choice).  Busy time per
    stream from HIP events on that stream; every recorded count is checked
    against the initial car numbers afterwards (a mismatch writes its
    evidence and raises)."""
    import torch
    from paper_1804_07981_amd.failures import dump_corruption
    group = workloads_mod().MEDIUM_GROUP if len(wl.lattices) > 1 else None
    lats = []
    shared = torch.cuda.Stream(dev) if mode == "joint" else None
    for lt in wl.lattices:
        stream = (shared if mode == "joint" else
                  torch.cuda.Stream(dev) if mode == "streams" else
                  torch.cuda.current_stream(dev))
        lat = B.Lattice(lt.n, lt.rho, lt.seed, layout=layout, stats_cap=wl.steps, device=dev,
                        stream=stream, **lt.kwargs())
        tun = tuning or load(layout, size_key(lt), group if mode == "joint" else None)
        if tun:
            lat.set_tuning(*tun)
        configure(lat)
        res_k = resident
        if res_k is None:
            res_k = 0 if tuning else load_resident_steps(
                layout, size_key(lt), group if mode == "joint" else None, lat.model,
                lat.topology)
        if res_k:
            lat.set_resident(res_k)
        lats.append(lat)

    def run_job():
        if mode == "joint":
            B.step_group(lats, wl.steps)
        else:
            for lat in lats:
                lat.step(wl.steps)

    for _ in range(warmup):
        run_job()
    torch.cuda.synchronize()
    streams = list({id(lat.stream): lat.stream for lat in lats}.values())
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in streams]
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    for st, (e0, _) in zip(streams, evs):
        e0.record(st)
    marks[0].record(streams[0])
    for i in range(steps):
        run_job()
        marks[i + 1].record(streams[0])
    for st, (_, e1) in zip(streams, evs):
        e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(steps))
    per_stream = [e0.elapsed_time(e1) / 1e3 for e0, e1 in evs]
    gpu_s = max(per_stream)
    for lat in lats:
        try:
            lat.stats(lat.steps_done - wl.steps, wl.steps)
        except B.BmlError as e:
            if e.code == B.BML_ECORRUPT:
                path = dump_corruption(e, lat, "bench", {"workload": wl.name, "mode": mode})
                print(f"car counts not conserved; evidence in {path}", file=sys.stderr,
                      flush=True)
            raise
    tr, tp, wpb = lats[0].tuning()
    res_k = lats[0].resident
    k = res_k or tp // 2
    passes = -(-wl.steps // k) * steps
    launches = passes if mode == "joint" else passes * len(lats)
    cells = sum(lt.cells for lt in wl.lattices)
    for lat in lats:
        lat.close()
    return {"gpu_s": gpu_s, "wall_s": wall, "k": k, "tile_rows": tr, "wpb": wpb,
            "resident": res_k,
            "launches": launches, "cells": cells, "mode": mode,
            "lattices_per_launch": len(lats) if mode == "joint" else 1,
            "lattices_total": len(lats),
            "avg_launch_s": sum(per_stream) / launches, "step_ms": step_ms,
            "gcups": cells * wl.steps * steps / gpu_s / 1e9}


def workloads_mod():
    import workloads
    return workloads


def hbm_roofline(res: dict, layout: int, kname: str, extra: dict | None = None) -> dict:
    """HBM roofline of the step kernel from one measure() result: algorithmic
    bytes of one launch (state read once and written once per pass) over the
    average launch duration; `traffic` = HBM bytes per launch from the
    committed counter summary when it was taken on this kernel source with
    this launch shape, else None."""
    k = res["k"]
    launch_cells = res["cells"] / res["lattices_total"] * res["lattices_per_launch"]
    alg = bytes_per_cell_step(layout, k) * launch_cells * k
    per_launch = res["avg_launch_s"]
    achieved = alg / per_launch / 1e9
    traffic = traffic_from_profile(kname, (res["tile_rows"], 2 * k, res["wpb"]), alg,
                                   resident=res.get("resident", 0))
    lay = "u8" if layout == 0 else "bitplane"
    if res.get("resident"):
        kernel = (f"block_kernel<{lay}, K={k}> (register-resident tiles of 1024, 512 or 256 "
                  f"columns by launch size x up to {512 - 2 * k} rows with {k} halo rows, "
                  f"4 waves/block, {res['lattices_per_launch']} lattice(s) per launch)")
    else:
        kernel = (f"pass_kernel<{lay}, K={k}> (strip rows {res['tile_rows'] or 'auto'}, "
                  f"{res['wpb']} waves/block, {res['lattices_per_launch']} lattice(s) per "
                  "launch)")
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": kernel,
           "algorithmic_bytes_per_launch": alg,
           "avg_launch_us": round(per_launch * 1e6, 2),
           "traffic_gbs": round(traffic / per_launch / 1e9, 1) if traffic else None,
           "traffic_over_algorithmic": round(traffic / alg, 4) if traffic else None}
    out.update(extra or {})
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "medium", "rect", "sweep", "early-exit"],
                    default="large")
    ap.add_argument("--plain-sample", type=int, default=None,
                    help="sweep/early-exit: time plain per-lattice runs on this many "
                         "lattices and scale to all")
    ap.add_argument("--layout", choices=["u8", "bitplane"], default="u8")
    ap.add_argument("--resident-max-n", type=int, default=1024,
                    help="sweep: the batch's register-resident limit (0: the streaming "
                         "kernel)")
    ap.add_argument("--split", type=int, default=None,
                    help="sweep: the resident slab halo (0: whole lattices; default: "
                         "autotuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the secondary measurements")
    ap.add_argument("--probe", action="store_true",
                    help="for counter runs: a 1 GiB device copy (the calibration kernel "
                         "of known traffic), then --steps BML steps of the workload")
    ap.add_argument("--topology", choices=["torus", "klein"], default="torus",
                    help="medium/large/rect: periodic in both directions, or the Klein "
                         "bottle (top and bottom edges glued with a reversal)")
    ap.add_argument("--model", type=int, choices=[1, 2, 3], default=1,
                    help="medium/large/rect: the model of Sec. 2 (1), Model II (2: one "
                         "phase per step, a coin on contested cells) or Model III (3: one "
                         "phase, a contested cell takes both cars)")
    ap.add_argument("--coin-seed", type=int, default=0x5EED,
                    help="Model II: the coin stream's seed")
    ap.add_argument("--tuning", type=int, nargs=3, metavar=("TILE_ROWS", "T_PHASES", "WPB"),
                    help="medium/large/rect: run this tuning instead of the autotuned one")
    ap.add_argument("--resident", type=int, default=None,
                    help="medium/large/rect: steps per launch of the register-resident tile "
                         "kernel (0: the streaming kernel; default: the autotuned choice)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("PROBE_LOG", "FETCH_DIR", "WRITE_DIR"),
                    help="no GPU: turn two rocprofv3 --pmc runs of --probe (FETCH_SIZE, "
                         "WRITE_SIZE) into profiles/pass_<layout>_<n>_t<T>.traffic.json "
                         "(block_<layout>_<n>_k<K>.traffic.json for the tile kernel)")
    args = ap.parse_args()

    if args.pmc_summary:
        return pmc_summary(*args.pmc_summary)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "row-slab decomposition is a design, not built.", file=sys.stderr)
        return 2

    import torch

    import paper_1804_07981_amd as B
    import workloads

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.workload == "sweep":
        return bench_sweep(args, B, workloads, dev)
    if args.workload == "early-exit":
        return bench_early_exit(args)
    wl = {"medium": workloads.MEDIUM, "large": workloads.LARGE,
          "rect": workloads.RECT}[args.workload]
    load = load_for(args)
    layout = 0 if args.layout == "u8" else 1
    topology = B.BML_TOPO_KLEIN if args.topology == "klein" else B.BML_TOPO_TORUS
    if args.model != 1 and args.topology != "torus":
        print("Models II and III run on the torus only", file=sys.stderr)
        return 2

    def configure(lat):
        lat.set_topology(topology)
        if args.model != 1:
            lat.set_model(args.model, args.coin_seed)

    group = workloads.MEDIUM_GROUP if len(wl.lattices) > 1 else None
    if args.probe:
        a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)                       # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
        # the launch shape the benchmark times: all lattices of the workload
        # in joint launches, with the same tuning
        stream = torch.cuda.Stream(dev)
        lats = [B.Lattice(lt.n, lt.rho, lt.seed, layout=layout, stats_cap=max(args.steps, 1),
                          device=dev, stream=stream, **lt.kwargs()) for lt in wl.lattices]
        tun = load(layout, size_key(wl.lattices[0]), group)
        res_k = args.resident if args.resident is not None else (
            0 if args.tuning else load_resident_steps(layout, size_key(wl.lattices[0]), group,
                                                      args.model, topology))
        for lat in lats:
            if tun:
                lat.set_tuning(*tun)
            configure(lat)
            if res_k:
                lat.set_resident(res_k)
        B.step_group(lats, args.steps)
        torch.cuda.synchronize()
        tr, tp, wpb = lats[0].tuning()
        print(json.dumps({"probe": wl.name, "layout": args.layout, "steps": args.steps,
                          "n": (wl.lattices[0].n if wl.lattices[0].cols is None
                                else f"{wl.lattices[0].n}x{wl.lattices[0].cols}"),
                          "lattices_per_launch": len(lats),
                          "cells_per_launch": sum(lt.cells for lt in wl.lattices),
                          "t_phases": tp, "tile_rows": tr, "waves_per_block": wpb,
                          "resident": lats[0].resident,
                          "kernel_hash": kernel_hash(resident=bool(lats[0].resident))}),
              flush=True)
        for lat in lats:
            lat.close()
        return 0

    def kname_of(w, lay):
        lt0 = w.lattices[0]
        name = (f"pass_{'u8' if lay == 0 else 'bitplane'}_{lt0.n}" if lt0.cols is None
                else f"pass_{'u8' if lay == 0 else 'bitplane'}_{lt0.n}x{lt0.cols}")
        return name + ("_klein" if args.topology == "klein" else "") + (
            f"_model{args.model}" if args.model != 1 else "")

    main_mode = "joint" if len(wl.lattices) > 1 else "single"
    res = measure(B, dev, wl, layout, args.steps, args.warmup, main_mode, load, configure,
                  resident=args.resident)
    value = res["gcups"]
    ms_per_step = res["gpu_s"] * 1e3 / args.steps
    alu = alu_roofline(layout, res["k"], value, args.model)
    if args.workload == "medium":
        # four lattices of 16 MiB (uint8): resident in the 256 MB Infinity
        # Cache, so the launches are bound by the ALU and on-chip caches,
        # not by HBM; the bytes they would move are reported alongside
        roofline = dict(alu, kernel=hbm_roofline(res, layout, kname_of(wl, layout))["kernel"],
                        avg_launch_us=round(res["avg_launch_s"] * 1e6, 2),
                        cache_resident_gbs=hbm_roofline(res, layout,
                                                        kname_of(wl, layout))["achieved"])
    elif res["resident"]:
        # the register-resident tile kernel reads and writes the state once
        # per K steps: its lane operations (the rule, the counts, the byte
        # conversion once per launch) bind it, with its HBM rate alongside
        hbm = hbm_roofline(res, layout, kname_of(wl, layout),
                           {"copy_ceiling_gbs": copy_ceiling(B, dev)})
        roofline = dict(alu, kernel=hbm["kernel"], traffic=hbm["traffic"],
                        avg_launch_us=hbm["avg_launch_us"],
                        algorithmic_bytes_per_launch=hbm["algorithmic_bytes_per_launch"],
                        hbm=hbm, effective_gbs=round(value * bytes_per_cell_step(layout, 1), 1))
    else:
        roofline = hbm_roofline(res, layout, kname_of(wl, layout),
                                {"copy_ceiling_gbs": copy_ceiling(B, dev), "alu": alu,
                                 "effective_gbs": round(value * bytes_per_cell_step(layout, 1),
                                                        1)})
    lt0 = wl.lattices[0]
    out = {
        "metric": "GCUPS (cell updates/s) + % HBM roofline; density-sweep time vs plain",
        "value": round(value, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.layout,
        "data": "synthetic (SplitMix64 iid lattices, seeded)",
        "config": {"workload": wl.name + ("-klein" if args.topology == "klein" else "")
                   + {1: "", 2: "-modelII", 3: "-modelIII"}[args.model],
                   "layout": args.layout, "topology": args.topology,
                   "update_rule": {1: "LR phase then TB phase",
                                   2: "Model II (one phase, coin seed %d)" % args.coin_seed,
                                   3: "Model III (one phase, a contested cell takes both "
                                      "cars)"}[args.model],
                   "lattices": [[lt.n, lt.cols or lt.n, lt.rho_lr if lt.rho_lr is not None
                                 else lt.rho / 2, lt.rho_tb if lt.rho_tb is not None
                                 else lt.rho / 2, lt.seed] for lt in wl.lattices],
                   "lattice_fields": ["rows", "cols", "rho_lr", "rho_tb", "seed"],
                   "steps_per_lattice": wl.steps,
                   "tuning": launch_shape(res),
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "step_ms_stats": {"median": round(statistics.median(res["step_ms"]), 3),
                          "mean": round(statistics.fmean(res["step_ms"]), 3),
                          "min": round(res["step_ms"][0], 3),
                          "max": round(res["step_ms"][-1], 3)},
    }

    if not args.no_variants and args.workload in ("large", "rect") and layout == 0 \
            and args.model == 1:
        # the unblocked kernel: one step per HBM pass (every cell read and
        # written once per step), one wave per block
        t2 = measure(B, dev, wl, 0, 1, 1, main_mode, load, configure, tuning=(0, 2, 1))
        out["t2"] = dict(hbm_roofline(t2, 0, kname_of(wl, 0)), gcups=round(t2["gcups"], 1))

    if not args.no_variants:
        other = 1 - layout
        r2 = measure(B, dev, wl, other, 1, 1, main_mode, load, configure)
        out["variants"] = {("bitplane" if other else "u8"): {
            "gcups": round(r2["gcups"], 2), **launch_shape(r2), "mode": r2["mode"],
            "alu": alu_roofline(other, r2["k"], r2["gcups"], args.model),
            "hbm": hbm_roofline(r2, other, kname_of(wl, other))}}
        if res["resident"]:
            # the streaming kernel on the same workload and layout
            r3 = measure(B, dev, wl, layout, 1, 1, main_mode, load, configure, resident=0)
            out["variants"][("u8" if layout == 0 else "bitplane") + "_streaming"] = {
                "gcups": round(r3["gcups"], 2), **launch_shape(r3), "mode": r3["mode"],
                "alu": alu_roofline(layout, r3["k"], r3["gcups"], args.model),
                "hbm": hbm_roofline(r3, layout, kname_of(wl, layout))}

    if not args.no_variants and args.workload == "large" and args.model == 1 \
            and args.topology == "torus" and not args.tuning:
        out["medium"] = medium_block(B, dev, workloads, load_for(args), configure)
        # the metric's second half: the 512-lattice density sweep, batched
        # in one captured graph against plain per-lattice runs of all 512
        # (about 5 s)
        out["density_sweep"] = sweep_measure(B, workloads, dev, 1, 1, None)
        st = sweep_measure(B, workloads, dev, 1, 1, 0, resident_max_n=0)
        out["density_sweep"]["streaming"] = {k: st[k] for k in ("kernel", "tuning", "gcups",
                                                                "batched_wall_s", "roofline")}
        out["early_exit"] = early_exit_block()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lt0, model=args.model, coin_seed=args.coin_seed)
    out["paper_context"] = paper_context()

    print(json.dumps(out), flush=True)
    return 0


def launch_shape(r: dict) -> dict:
    """The launch shape a measurement ran: the tile kernel's steps per
    launch, else the streaming kernel's strip rows, phases per pass and
    waves per block."""
    if r["resident"]:
        return {"resident_steps": r["resident"]}
    return {"tile_rows": r["tile_rows"], "t_phases": 2 * r["k"], "waves_per_block": r["wpb"]}


def medium_block(B, dev, workloads, load, configure) -> dict:
    """The four 4096 x 4096 lattices (rho .25/.35/.38/.45, seeds 1-4, 10000
    steps each) in joint launches, both layouts, plus the same lattices on
    separate streams and each alone.  Their 16 MiB (uint8) states stay in
    the Infinity Cache, so the roofline here is the ALU one."""
    wl = workloads.MEDIUM
    out = {"workload": wl.name}
    for lay in (0, 1):
        r = measure(B, dev, wl, lay, 1, 1, "joint", load, configure)
        name = "u8" if lay == 0 else "bitplane"
        out[name] = {"gcups": round(r["gcups"], 1), **launch_shape(r),
                     "avg_launch_us": round(r["avg_launch_s"] * 1e6, 2),
                     "roofline": alu_roofline(lay, r["k"], r["gcups"])}
    r3 = measure(B, dev, wl, 0, 1, 1, "streams", load, configure)
    out["u8_separate_streams_gcups"] = round(r3["gcups"], 1)
    single = {}
    for lay in (0, 1):
        lt = wl.lattices[0]
        one = workloads.Workload(wl.name + "-first", (lt,), wl.steps, "")
        r = measure(B, dev, one, lay, 1, 1, "single", load, configure)
        single["u8" if lay == 0 else "bitplane"] = round(r["gcups"], 1)
    out["single_lattice_gcups_rho0.25"] = single
    return out


def early_exit_block() -> dict:
    """The learned early exit on its full workload (9024 lattices of 512 x
    512, 20000-step labels, held-out seeds 51..63), with plain per-lattice
    runs timed on 8 held-out lattices and scaled."""
    from paper_1804_07981_amd import early_exit as ee
    ns, rhos, seeds, split = ee.c4_lattices()
    rep = ee.experiment(ns, rhos, seeds, split, plain_sample=8,
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    return {"workload": "bml-early-exit-512x512-141rho-64seeds-20000steps", **rep}


if __name__ == "__main__":
    sys.exit(main())
