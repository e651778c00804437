"""Plants plausible mistakes in a copy of the oracle (on the CPU) and checks
that the pin tests catch every one of them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bml_oracle.c")

MUTATIONS = [
    ("right neighbour taken on the left", "return c + 1 < cols ? c + 1 : 0;",
     "return c > 0 ? c - 1 : cols - 1;"),
    ("TB cars move up instead of down",
     "if (r + 1 < rows)\n        return (r + 1) * cols + c;\n    return topology == 1 ? cols - 1 - c : c;",
     "if (r > 0)\n        return (r - 1) * cols + c;\n    return (rows - 1) * cols + (topology == 1 ? cols - 1 - c : c);"),
    ("TB enters any non-TB cell", "            if (cur[dest] == EMPTY) {\n                nxt[here] = EMPTY;",
     "            if (cur[dest] != TB) {\n                nxt[here] = EMPTY;"),
    ("LR leaves into any non-LR cell", "            if (row[dest] == EMPTY) {",
     "            if (row[dest] != LR) {"),
    ("LR moves decided on the partly updated row", "            if (row[dest] == EMPTY) {",
     "            if (out[dest] == EMPTY) {"),
    ("V phase decides on the lattice it is updating",
     "moved_tb += tb_moves(i, i + 1, rows, cols, tmp, cells, topology);",
     "moved_tb += tb_moves(i, i + 1, rows, cols, cells, cells, topology);"),
    ("V phase applied to the pre-H lattice (row copy dropped)",
     "            memcpy(cells + i * cols, tmp + i * cols, (size_t)cols);",
     "            (void)0;"),
    ("moved counts each LR move twice", "                out[dest] = LR;\n                cars_moved++;",
     "                out[dest] = LR;\n                cars_moved += 2;"),
    ("LR threshold off by a factor of two", "*thr_lr = (uint64_t)ldexp(rho * 0.5, 53);",
     "*thr_lr = (uint64_t)ldexp(rho * 0.5, 52);"),
    ("SplitMix64 shift constant", "z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;",
     "z = (z ^ (z >> 26)) * 0x94D049BB133111EBull;"),
    ("SplitMix64 stream offset by one", "uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;",
     "uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;"),
    ("bit order reversed in the TB plane", "if (c == TB)\n                    b |= 1u << bit;",
     "if (c == TB)\n                    b |= 1u << (31 - bit);"),
    ("stats fields swapped", "stats[4 * s + 1] = (uint32_t)moved_lr;",
     "stats[4 * s + 1] = (uint32_t)moved_tb;"),
    ("Klein seam glued without the reversal",
     "return topology == 1 ? cols - 1 - c : c;\n}",
     "return c;\n}"),
    ("Klein seam reversal off by one column",
     "return topology == 1 ? cols - 1 - c : c;\n}",
     "return topology == 1 ? (cols - c) % cols : c;\n}"),
    ("Model II: the TB car obeys the coin the wrong way round",
     "if (!contested || !model2_coin(coin_seed, step, f, down, j)) {",
     "if (!contested || model2_coin(coin_seed, step, f, down, j)) {"),
    ("Model II: the LR car reads the coin of its own cell",
     "if (!contested || model2_coin(coin_seed, step, f, i, right)) {",
     "if (!contested || model2_coin(coin_seed, step, f, i, j)) {"),
    ("Model III: an LR car enters a cell that holds only a TB car",
     "if (cur[i * cols + right] == EMPTY)\n                    (*moved_lr)++;",
     "if (!(cur[i * cols + right] & LR))\n                    (*moved_lr)++;"),
    ("Model III: a contested cell keeps only the LR car",
     "if (cur[up * cols + j] & TB)\n                    out |= TB;",
     "if ((cur[up * cols + j] & TB) && !(out & LR))\n                    out |= TB;"),
    ("Model III: cars arrive in a cell the other type holds",
     "if (c == EMPTY) {                 /* arrivals, possibly both */",
     "if (c != BOTH) {                  /* arrivals, possibly both */"),
    ("Model II window: the coin column ignores the window origin",
     "int64_t gi = (f->row0 + i) % f->rows_g, gj = (f->col0 + j) % f->cols_g;",
     "int64_t gi = (f->row0 + i) % f->rows_g, gj = j % f->cols_g;"),
    ("asymmetric TB threshold without the LR share", "*thr_tb = (uint64_t)ldexp(rho_lr + rho_tb, 53);",
     "*thr_tb = (uint64_t)ldexp(rho_tb, 53);"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,before,after", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, before, after):
    src = open(SRC).read()
    assert before in src, "mutation site not found"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(before, after, 1))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                    "-o", str(so), str(mut), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True)
    assert r.returncode != 0, f"pins did not catch: {name}"
