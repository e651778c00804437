"""Builds libbml.so (the HIP kernels and the C ABI of include/bml.h) for
gfx950 with hipcc, in place next to this file."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbml.so")
# The step kernels: bml_pass_inst.hip compiled once per (layout, column
# mode / range of K, topology); see bml_pass.hpp.
PASS_RANGES = {"lo": (0, 1, 4), "hi": (0, 5, 4), "row1": (1, 1, 8), "row2": (2, 1, 8)}
# variant name -> (topology, model)
PASS_KINDS = {"torus": ("TOPO_TORUS", 1), "klein": ("TOPO_KLEIN", 1), "model2": ("TOPO_TORUS", 2),
              "model3": ("TOPO_TORUS", 3)}
PASS_VARIANTS = [
    (f"pass_table_{io}_{rng}_{kind}",
     [f"-DBML_INST_IO={'IO_U8' if io == 'u8' else 'IO_BP'}", f"-DBML_INST_ROW={row}",
      f"-DBML_INST_TOPO={topo}", f"-DBML_INST_MODEL={model}",
      f"-DBML_INST_KLO={klo}", f"-DBML_INST_KN={kn}",
      f"-DBML_INST_NAME=pass_table_{io}_{rng}_{kind}"])
    for kind, (topo, model) in PASS_KINDS.items() for io in ("u8", "bp")
    for rng, (row, klo, kn) in PASS_RANGES.items()]
SOURCES = ["bml_lattice.hip", "bml_batch.hip", "bml_batch_u8.hip", "bml_batch_bp.hip",
           "bml_resident_u8.hip", "bml_resident_bp.hip", "bml_block.hip", "bml_mlp.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    # Keep the compiler from forming packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(out: str | None = None, extra: list[str] | None = None,
          verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source (in parallel) and link one shared library.
    Always recompiles."""
    out = out or LIB
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(job) -> str:
        src, name, defines = job
        obj = os.path.join(objdir, name + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, *(extra or []), *defines, *inc, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n" + r.stdout + r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        jobs = [("bml_pass_inst.hip", name, defs) for name, defs in PASS_VARIANTS]
        jobs += [(src, os.path.splitext(src)[0], []) for src in SOURCES]
        objs = list(ex.map(compile_one, jobs))
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
