"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): bml_oracle.c is rebuilt with -fsanitize=address,undefined (every
report fatal) and the whole pin suite runs against it, so an out-of-bounds
neighbour index, a signed overflow or a misaligned access anywhere in the
oracle stops the run.  A planted heap overflow checks that the sanitizer is
really active in that run."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bml_oracle.c")
FLAGS = ["-O1", "-g", "-std=c11", "-fopenmp", "-shared", "-fPIC",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _build(src_text, out_dir):
    src = os.path.join(out_dir, "oracle_san.c")
    with open(src, "w") as f:
        f.write(src_text)
    so = os.path.join(out_dir, "liboracle_san.so")
    subprocess.run(["gcc", *FLAGS, "-o", so, src, "-lm"], check=True)
    return so


def _run_pins(so, log_dir):
    # reports go to files: the child's pytest captures its own stderr, and
    # a report written there is lost when the sanitizer ends the process
    log = os.path.join(log_dir, "san")
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=so,
               ASAN_OPTIONS=f"detect_leaks=0:log_path={log}",
               UBSAN_OPTIONS=f"print_stacktrace=1:log_path={log}",
               LD_PRELOAD=" ".join([_runtime("libasan.so"), _runtime("libubsan.so")]))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    reports = "".join(open(os.path.join(log_dir, f)).read()
                      for f in sorted(os.listdir(log_dir)) if f.startswith("san"))
    return r, reports


needs_runtime = pytest.mark.skipif(
    shutil.which("gcc") is None or _runtime("libasan.so") is None
    or _runtime("libubsan.so") is None, reason="gcc sanitizer runtimes not installed")


@pytest.mark.slow
@needs_runtime
def test_pins_pass_under_asan_and_ubsan(tmp_path):
    so = _build(open(SRC).read(), str(tmp_path))
    syms = subprocess.run(["nm", "-D", so], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "not instrumented"
    r, reports = _run_pins(so, str(tmp_path))
    assert r.returncode == 0 and not reports, r.stdout[-3000:] + reports[-3000:]
    assert "passed" in r.stdout


@pytest.mark.slow
@needs_runtime
def test_sanitizer_catches_a_planted_overflow(tmp_path):
    """run_many's per-lattice scratch one byte short: the oracle writes past
    it on the first step, and the sanitized pin run must stop there."""
    src = open(SRC).read()
    site = "uint8_t *tmp = (uint8_t *)malloc((size_t)(n * n));"
    assert site in src
    so = _build(src.replace(site, "uint8_t *tmp = (uint8_t *)malloc((size_t)(n * n - 1));"),
                str(tmp_path))
    r, reports = _run_pins(so, str(tmp_path))
    assert r.returncode != 0
    assert "heap-buffer-overflow" in reports
