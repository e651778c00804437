"""CPU checks of bench.py's measurement helpers: the algorithmic byte and
lane-op counts, the counter summary on a synthetic rocprofv3 output, the
source-hash gate on stored traffic figures, tuning lookup and the one-GPU
guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_cell_step():
    # the state is read and written once per pass of k steps
    assert bench.bytes_per_cell_step(0, 1) == 2.0
    assert bench.bytes_per_cell_step(0, 8) == 0.25
    assert bench.bytes_per_cell_step(1, 1) == 0.5
    assert bench.bytes_per_cell_step(1, 4) == 0.125


def test_alu_roofline_counts():
    r = bench.alu_roofline(1, 8, 1000.0)             # bitplane: 18 slots per word-step
    assert r["lane_ops_per_cell_step"] == pytest.approx(18 / 32, rel=1e-3)
    assert r["achieved"] == pytest.approx(1000e9 * 18 / 32 / 1e12, abs=0.01)
    u8 = bench.alu_roofline(0, 8, 1000.0)            # + 128 conversion slots per word and pass
    assert u8["lane_ops_per_cell_step"] == pytest.approx((18 + 16) / 32, rel=1e-3)
    assert bench.alu_roofline(1, 8, 1.0, model=2)["lane_ops_per_cell_step"] == \
        pytest.approx(75 / 32, rel=1e-3)
    assert bench.alu_roofline(1, 8, 1.0, model=3)["lane_ops_per_cell_step"] == \
        pytest.approx(18 / 32, rel=1e-3)
    # 256 CUs x 128 lanes per clock x 2.4 GHz: the fp32 vector rate
    # (157.3 TFLOP/s counting an FMA as two)
    assert bench.ALU_PEAK_LANE_OPS == pytest.approx(7.86432e13)
    assert 2 * bench.ALU_PEAK_LANE_OPS == pytest.approx(157.3e12, rel=1e-3)


def _write_pmc(dirpath, counter, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "pmc_counter_collection.csv"), "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, name, v in rows:
            # counters come per shader engine / XCD: split each value in two
            f.write(f'{d},"{name}",{counter},{v / 2}\n{d},"{name}",{counter},{v / 2}\n')


def test_pmc_summary_scales_by_the_copy(tmp_path):
    """A 1 GiB copy reading 524288 KiB (the counter sees half) and writing
    1048576 KiB calibrates the step kernel's counters: FETCH is doubled,
    WRITE kept."""
    probe = {"probe": "x", "layout": "u8", "steps": 16, "n": 1024, "lattices_per_launch": 1,
             "cells_per_launch": 1 << 20, "t_phases": 2, "tile_rows": 0, "waves_per_block": 1,
             "kernel_hash": "abc"}
    log = tmp_path / "probe.log"
    log.write_text("noise\n" + json.dumps(probe) + "\n")
    fetch, write = tmp_path / "f", tmp_path / "w"
    _write_pmc(fetch, "FETCH_SIZE", [(1, "copy_kernel", 524288.0),
                                     (2, "void bml::pass_kernel<0, 1, 0, 0, 1>", 512.0),
                                     (3, "void bml::pass_kernel<0, 1, 0, 0, 1>", 512.0)])
    _write_pmc(write, "WRITE_SIZE", [(1, "copy_kernel", 1048576.0),
                                     (2, "void bml::pass_kernel<0, 1, 0, 0, 1>", 1024.0),
                                     (3, "void bml::pass_kernel<0, 1, 0, 0, 1>", 1024.0)])
    out_dir = tmp_path / "profiles"
    out_dir.mkdir()
    assert bench.pmc_summary(str(log), str(fetch), str(write), profiles=str(out_dir)) == 0
    d = json.load(open(out_dir / "pass_u8_1024_t2.traffic.json"))
    assert d["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert d["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    assert d["hbm_bytes_per_launch"] == pytest.approx((512 * 2 + 1024) * 1024)
    assert d["algorithmic_bytes_per_launch"] == 2 * (1 << 20)     # 1 B read + 1 B written per cell
    assert d["ratio_to_algorithmic"] == pytest.approx(1.0)
    assert d["dispatches"] == 2


def test_traffic_needs_the_same_source_and_tuning(tmp_path):
    good = {"kernel_hash": bench.kernel_hash(), "hbm_bytes_per_launch": 123.0,
            "probe": {"tile_rows": 16, "t_phases": 16, "waves_per_block": 4}}
    (tmp_path / "pass_u8_4096_t16.traffic.json").write_text(json.dumps(good))
    assert bench.traffic_from_profile("pass_u8_4096", (16, 16, 4), 1.0, str(tmp_path)) == 123.0
    assert bench.traffic_from_profile("pass_u8_4096", (8, 16, 4), 1.0, str(tmp_path)) is None
    stale = dict(good, kernel_hash="0000000000000000")
    (tmp_path / "pass_u8_4096_t16.traffic.json").write_text(json.dumps(stale))
    assert bench.traffic_from_profile("pass_u8_4096", (16, 16, 4), 1.0, str(tmp_path)) is None
    assert bench.traffic_from_profile("pass_u8_32", (16, 16, 4), 1.0, str(tmp_path)) is None


def test_committed_traffic_summaries_are_well_formed():
    """Every stored counter summary names its kernel source hash and launch
    shape and carries the copy calibration it was scaled by; the benchmark
    uses it only while the hash matches the current source (otherwise its
    line reports traffic as null)."""
    names = [f for f in os.listdir(bench.PROFILES) if f.endswith(".traffic.json")]
    assert names
    for f in names:
        d = json.load(open(os.path.join(bench.PROFILES, f)))
        assert len(d["kernel_hash"]) == 16
        for key in ("tile_rows", "t_phases", "waves_per_block"):
            assert key in d["probe"]
        cal = d["copy_calibration"]
        assert cal["fetch_scale"] > 0 and cal["write_scale"] > 0
        assert d["hbm_bytes_per_launch"] == pytest.approx(
            (d["fetch_kib_per_dispatch"] * cal["fetch_scale"]
             + d["write_kib_per_dispatch"] * cal["write_scale"]) * 1024, rel=1e-9)
        assert d["ratio_to_algorithmic"] == pytest.approx(
            d["hbm_bytes_per_launch"] / d["algorithmic_bytes_per_launch"], rel=1e-9)


def test_tuning_lookup_and_model_fallback():
    t = bench.load_tuning(0, 4096, "medium4")
    assert t is not None and len(t) == 3
    m2 = bench.load_tuning(0, 4096, "medium4", model=2)
    assert m2 is not None
    # no Model III entry: the two-phase rule's tuning is used
    assert bench.load_tuning(0, 4096, "medium4", model=3) == t
    assert bench.size_key(type("L", (), {"n": 8192, "cols": 32768})()) == "8192x32768"
    assert bench.size_key(type("L", (), {"n": 4096, "cols": None})()) == 4096


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_paper_context_values():
    """GCUPS derived from the paper's times: N^2 * 1024 steps / seconds."""
    runs = {(r["machine"].split(" (")[0], r["n"]): r for r in bench.paper_context()["runs"]}
    gtx = runs[("GeForce GTX 1070", 4096)]
    assert gtx["gcups"] == pytest.approx(4096**2 * 1024 / 0.768 / 1e9, abs=0.01)
    assert gtx["gcups"] == pytest.approx(22.37, abs=0.01)
    assert runs[("Xeon E5-2603", 4096)]["gcups"] == pytest.approx(7.50, abs=0.01)
    assert runs[("Quadro K620", 4096)]["gcups"] == pytest.approx(2.88, abs=0.01)
