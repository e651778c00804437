/*
 * bml_oracle.c -- plain, slow, obviously correct CPU oracle for the
 * Biham-Middleton-Levine traffic automaton (Model I).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path.
 *
 * What it follows (Marzolla, "Parallel Implementations of Cellular Automata
 * for Traffic Models", arXiv:1804.07981):
 *   - Sec. 2 (the BML model): an N x N periodic lattice; each cell is EMPTY,
 *     LR (moves left-to-right) or TB (moves top-to-bottom); horizontal and
 *     vertical phases alternate; a car leaving one side re-enters on the
 *     opposite side.
 *   - Sec. 2, the two phase rules: a cell that is EMPTY receives the LR car
 *     on its left (horizontal phase) or the TB car above it (vertical
 *     phase); a car whose target cell is EMPTY leaves; nothing else changes.
 *     Written here car by car: every car that can advance does, all
 *     decisions taken on the lattice as it was before the phase.
 *   - Sec. 2, Fig. 1 caption text: one step = a horizontal then a vertical
 *     phase.
 *   - Sec. 3 (serial implementation): synchronous update through two grids
 *     (read one, write the other, swap); row-major cell index i*N + j; one
 *     byte per cell with EMPTY=0, LR=1, TB=2.
 *   - Sec. 4 (OpenMP): the row loop is split across threads.
 * Readings where the paper is silent (initial placement, stats) are the
 * project's own and are stated at each function.
 *
 * Lattices are rows x cols (the paper's case is rows = cols = N); the
 * oracle accepts any rows, cols >= 1.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { EMPTY = 0, LR = 1, TB = 2 };

/* ------------------------------------------------------------------------ */
/* Initial placement.  The paper only says vehicles are placed at random     */
/* (Sec. 2, text under Fig. 1).  Reading used here: every cell is drawn      */
/* independently, LR with probability rho/2, TB with probability rho/2,      */
/* else EMPTY, from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014; Vigna's    */
/* public-domain reference generator).                                       */
/* ------------------------------------------------------------------------ */

/* The k-th output (k = 0, 1, ...) of the SplitMix64 stream whose state
 * starts at `seed`: the state advances by the golden gamma before each
 * output, and the output is the state passed through the finaliser. */
uint64_t bmlo_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Integer thresholds on a 53-bit uniform u = output >> 11: a cell is LR if
 * u < thr_lr, TB if thr_lr <= u < thr_tb, EMPTY otherwise.  Both are
 * truncations of rho/2 * 2^53 and rho * 2^53 computed in IEEE double. */
void bmlo_thresholds(double rho, uint64_t *thr_lr, uint64_t *thr_tb)
{
    *thr_lr = (uint64_t)ldexp(rho * 0.5, 53);
    *thr_tb = (uint64_t)ldexp(rho, 53);
}

/* Cell k = i*cols + j takes the k-th SplitMix64 output of stream `seed`. */
void bmlo_init_cells(int64_t rows, int64_t cols, uint64_t seed, double rho,
                     uint8_t *cells)
{
    uint64_t thr_lr, thr_tb;
    bmlo_thresholds(rho, &thr_lr, &thr_tb);
    int64_t total = rows * cols;
    for (int64_t k = 0; k < total; k++) {
        uint64_t u = bmlo_splitmix64(seed, (uint64_t)k) >> 11;
        cells[k] = (u < thr_lr) ? LR : (u < thr_tb) ? TB : EMPTY;
    }
}

/* Asymmetric placement (Sec. 2 lists an unequal number of LR and TB cars
 * among the extensions of the model): LR w.p. rho_lr, TB w.p. rho_tb, from
 * the same uniform u as above: LR if u < floor(rho_lr 2^53), else TB if
 * u < floor((rho_lr + rho_tb) 2^53).  rho_lr = rho_tb = rho/2 gives exactly
 * the thresholds of bmlo_thresholds(rho). */
void bmlo_thresholds_asym(double rho_lr, double rho_tb, uint64_t *thr_lr, uint64_t *thr_tb)
{
    *thr_lr = (uint64_t)ldexp(rho_lr, 53);
    *thr_tb = (uint64_t)ldexp(rho_lr + rho_tb, 53);
}

void bmlo_init_cells_asym(int64_t rows, int64_t cols, uint64_t seed, double rho_lr,
                          double rho_tb, uint8_t *cells)
{
    uint64_t thr_lr, thr_tb;
    bmlo_thresholds_asym(rho_lr, rho_tb, &thr_lr, &thr_tb);
    int64_t total = rows * cols;
    for (int64_t k = 0; k < total; k++) {
        uint64_t u = bmlo_splitmix64(seed, (uint64_t)k) >> 11;
        cells[k] = (u < thr_lr) ? LR : (u < thr_tb) ? TB : EMPTY;
    }
}

/* ------------------------------------------------------------------------ */
/* The two phases, stated car by car (Sec. 2): in the horizontal phase every */
/* LR car whose cell to the right is EMPTY moves into it; in the vertical   */
/* phase every TB car whose cell below is EMPTY moves into it.  Every test  */
/* looks at `cur` only (the synchronous update of Sec. 3); the moves are    */
/* applied to `nxt`, which starts as a copy of `cur`.  An EMPTY cell has     */
/* exactly one cell to its left and one above it, so no two cars ever claim */
/* the same cell and the order of the moves is irrelevant.  The functions   */
/* return how many cars moved.                                              */
/* ------------------------------------------------------------------------ */

/* Column to the right of column c on a ring of `cols` columns. */
static int64_t right_of(int64_t c, int64_t cols)
{
    return c + 1 < cols ? c + 1 : 0;
}

/* Horizontal phase restricted to rows [first, end): LR cars never leave
 * their row, so each row is independent of the others. */
static int64_t lr_moves(int64_t first, int64_t end, int64_t cols, const uint8_t *cur,
                        uint8_t *nxt)
{
    int64_t cars_moved = 0;
    for (int64_t r = first; r < end; r++) {
        const uint8_t *row = cur + r * cols;
        uint8_t *out = nxt + r * cols;
        memcpy(out, row, (size_t)cols);
        for (int64_t c = 0; c < cols; c++) {
            if (row[c] != LR)
                continue;
            const int64_t dest = right_of(c, cols);
            if (row[dest] == EMPTY) {
                out[c] = EMPTY;
                out[dest] = LR;
                cars_moved++;
            }
        }
    }
    return cars_moved;
}

/* Cell below (r, c).  On the torus (topology 0) it is (r+1, c), the last
 * row wrapping to row 0.  On the Klein bottle (topology 1; the lattice of
 * Campora et al. cited in Sec. 2) the bottom edge is glued to the top one
 * with a reversal: below (rows-1, c) lies (0, cols-1-c).  Left and right
 * stay periodic either way. */
static int64_t index_below(int64_t r, int64_t c, int64_t rows, int64_t cols, int topology)
{
    if (r + 1 < rows)
        return (r + 1) * cols + c;
    return topology == 1 ? cols - 1 - c : c;
}

/* Vertical phase for the TB cars of rows [first, end).  `nxt` must already
 * hold a copy of `cur` (a car may move into the next row, which another
 * caller may own). */
static int64_t tb_moves(int64_t first, int64_t end, int64_t rows, int64_t cols,
                        const uint8_t *cur, uint8_t *nxt, int topology)
{
    int64_t cars_moved = 0;
    for (int64_t r = first; r < end; r++) {
        for (int64_t c = 0; c < cols; c++) {
            const int64_t here = r * cols + c;
            if (cur[here] != TB)
                continue;
            const int64_t dest = index_below(r, c, rows, cols, topology);
            if (cur[dest] == EMPTY) {
                nxt[here] = EMPTY;
                nxt[dest] = TB;
                cars_moved++;
            }
        }
    }
    return cars_moved;
}

static int64_t count_value(const uint8_t *cells, int64_t n, uint8_t v)
{
    int64_t c = 0;
    for (int64_t k = 0; k < n; k++)
        c += (cells[k] == v);
    return c;
}

/* One horizontal phase over the whole lattice (Sec. 2). */
int64_t bmlo_phase_h(int64_t rows, int64_t cols, const uint8_t *cur,
                     uint8_t *next)
{
    return lr_moves(0, rows, cols, cur, next);
}

/* One vertical phase over the whole lattice (Sec. 2; the paper leaves its
 * code out as the mirror of the horizontal one). */
int64_t bmlo_phase_v(int64_t rows, int64_t cols, const uint8_t *cur,
                     uint8_t *next)
{
    memcpy(next, cur, (size_t)(rows * cols));
    return tb_moves(0, rows, rows, cols, cur, next, 0);
}

/* Vertical phase on the torus (topology 0) or the Klein bottle (1). */
int64_t bmlo_phase_v_topo(int64_t rows, int64_t cols, const uint8_t *cur,
                          uint8_t *next, int32_t topology)
{
    memcpy(next, cur, (size_t)(rows * cols));
    return tb_moves(0, rows, rows, cols, cur, next, topology);
}

int64_t bmlo_count(const uint8_t *cells, int64_t n, int32_t value)
{
    return count_value(cells, n, (uint8_t)value);
}

/* ------------------------------------------------------------------------ */
/* Step loop.  One step = horizontal phase (cells -> tmp) then vertical     */
/* phase (tmp -> cells).  Per step it records four counts, the cars of     */
/* each type and how many of them moved in their phase:                     */
/*   stats[4s+0] n_lr     = LR cars in the lattice after the H phase        */
/*   stats[4s+1] moved_lr = LR cars that moved in the H phase               */
/*   stats[4s+2] n_tb     = TB cars in the lattice after the V phase        */
/*   stats[4s+3] moved_tb = TB cars that moved in the V phase               */
/* `stats` may be NULL.  `tmp` is caller scratch of rows*cols bytes.        */
/* n_threads > 0 splits the row loop over that many OpenMP threads (Sec. 4);*/
/* any thread count gives the same bytes and counts.                        */
/* ------------------------------------------------------------------------ */
static void run_topo(int64_t rows, int64_t cols, uint8_t *cells, uint8_t *tmp,
                     int64_t steps, uint32_t *stats, int32_t n_threads, int topology);

void bmlo_run(int64_t rows, int64_t cols, uint8_t *cells, uint8_t *tmp,
              int64_t steps, uint32_t *stats, int32_t n_threads)
{
    run_topo(rows, cols, cells, tmp, steps, stats, n_threads, 0);
}

/* As bmlo_run, on the torus (topology 0) or the Klein bottle (1). */
void bmlo_run_topo(int64_t rows, int64_t cols, uint8_t *cells, uint8_t *tmp,
                   int64_t steps, uint32_t *stats, int32_t n_threads, int32_t topology)
{
    run_topo(rows, cols, cells, tmp, steps, stats, n_threads, topology);
}

static void run_topo(int64_t rows, int64_t cols, uint8_t *cells, uint8_t *tmp,
                     int64_t steps, uint32_t *stats, int32_t n_threads, int topology)
{
    int nt = n_threads > 0 ? n_threads : 1;
    for (int64_t s = 0; s < steps; s++) {
        int64_t moved_lr = 0, moved_tb = 0, n_lr = 0, n_tb = 0;
        /* horizontal phase: cells -> tmp, one row per iteration */
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : moved_lr, n_lr)
#endif
        for (int64_t i = 0; i < rows; i++) {
            moved_lr += lr_moves(i, i + 1, cols, cells, tmp);
            n_lr += count_value(tmp + i * cols, cols, LR);
        }
        /* vertical phase: tmp -> cells; every row is copied before any TB
         * car moves, since a car lands in the next row */
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static)
#endif
        for (int64_t i = 0; i < rows; i++)
            memcpy(cells + i * cols, tmp + i * cols, (size_t)cols);
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : moved_tb)
#endif
        for (int64_t i = 0; i < rows; i++)
            moved_tb += tb_moves(i, i + 1, rows, cols, tmp, cells, topology);
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : n_tb)
#endif
        for (int64_t i = 0; i < rows; i++)
            n_tb += count_value(cells + i * cols, cols, TB);
        if (stats) {
            stats[4 * s + 0] = (uint32_t)n_lr;
            stats[4 * s + 1] = (uint32_t)moved_lr;
            stats[4 * s + 2] = (uint32_t)n_tb;
            stats[4 * s + 3] = (uint32_t)moved_tb;
        }
    }
    (void)nt; /* unused when built without OpenMP */
}

/* ------------------------------------------------------------------------ */
/* Model II (Sec. 2): every car advances in one phase per step.  A car moves */
/* when its target cell (right for LR, below for TB) is EMPTY before the    */
/* step; if an EMPTY cell is the target of both an LR car (its left         */
/* neighbour) and a TB car (its top neighbour), one of them is chosen at    */
/* random to move and the other stays.  The paper gives no distribution;    */
/* here it is a fair coin from a counter-based generator: at global step s, */
/* the coin of cell (i, j) is bit (j mod 32) of the low 32 bits of the      */
/* SplitMix64 output number s*(rows*W) + i*W + j/32 of stream `coin_seed`,  */
/* W = ceil(cols/32); 1 means the LR car moves.  Torus only.                */
/* stats per step: n_lr, moved_lr, n_tb, moved_tb after that one phase.     */
/* A window of a larger lattice (used to check a large run on small        */
/* windows) keeps the coins of its cells' positions in that lattice: cell   */
/* (i, j) of the window is cell ((row0 + i) mod rows_g, (col0 + j) mod      */
/* cols_g) of a rows_g x cols_g lattice, and i, j, rows, cols above are     */
/* those global ones.  A whole lattice is its own frame (0, 0, rows, cols). */
/* Parity unpinned against the paper: it gives no Model II values, and the  */
/* coin is this library's reading; the tests pin the code to that reading.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t row0, col0, rows_g, cols_g;
} coin_frame;

static int model2_coin(uint64_t coin_seed, int64_t step, const coin_frame *f, int64_t i,
                       int64_t j)
{
    int64_t gi = (f->row0 + i) % f->rows_g, gj = (f->col0 + j) % f->cols_g;
    int64_t words = (f->cols_g + 31) / 32;
    uint64_t k = (uint64_t)step * (uint64_t)(f->rows_g * words) + (uint64_t)(gi * words + gj / 32);
    uint32_t z = (uint32_t)bmlo_splitmix64(coin_seed, k);
    return (int)((z >> (gj % 32)) & 1u);
}

static void model2_rows(int64_t r0, int64_t r1, int64_t rows, int64_t cols,
                        const uint8_t *cur, uint8_t *next, uint64_t coin_seed, int64_t step,
                        const coin_frame *f, int64_t *moved_lr, int64_t *moved_tb)
{
    for (int64_t i = r0; i < r1; i++) {
        int64_t up = (i - 1 + rows) % rows, down = (i + 1) % rows;
        for (int64_t j = 0; j < cols; j++) {
            int64_t left = (j - 1 + cols) % cols, right = (j + 1) % cols;
            uint8_t c = cur[i * cols + j], out = c;
            if (c == EMPTY) {
                int from_left = cur[i * cols + left] == LR;
                int from_top = cur[up * cols + j] == TB;
                if (from_left && from_top)
                    out = model2_coin(coin_seed, step, f, i, j) ? LR : TB;
                else if (from_left)
                    out = LR;
                else if (from_top)
                    out = TB;
            } else if (c == LR && cur[i * cols + right] == EMPTY) {
                /* a TB car above the target competes for it */
                int contested = cur[up * cols + right] == TB;
                if (!contested || model2_coin(coin_seed, step, f, i, right)) {
                    out = EMPTY;
                    (*moved_lr)++;
                }
            } else if (c == TB && cur[down * cols + j] == EMPTY) {
                /* an LR car left of the target competes for it */
                int contested = cur[down * cols + left] == LR;
                if (!contested || !model2_coin(coin_seed, step, f, down, j)) {
                    out = EMPTY;
                    (*moved_tb)++;
                }
            }
            next[i * cols + j] = out;
        }
    }
}

/* `steps` Model II steps starting at global step `step0` (the coin index),  */
/* the lattice being the window (row0, col0) of a rows_g x cols_g one.       */
void bmlo_run_model2(int64_t rows, int64_t cols, uint8_t *cells, uint8_t *tmp, int64_t steps,
                     int64_t step0, uint64_t coin_seed, uint32_t *stats, int32_t n_threads,
                     int64_t row0, int64_t col0, int64_t rows_g, int64_t cols_g)
{
    int nt = n_threads > 0 ? n_threads : 1;
    const coin_frame frame = {row0, col0, rows_g, cols_g};
    for (int64_t s = 0; s < steps; s++) {
        int64_t moved_lr = 0, moved_tb = 0;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : moved_lr, moved_tb)
#endif
        for (int64_t i = 0; i < rows; i++) {
            int64_t ml = 0, mt = 0;
            model2_rows(i, i + 1, rows, cols, cells, tmp, coin_seed, step0 + s, &frame, &ml, &mt);
            moved_lr += ml;
            moved_tb += mt;
        }
        memcpy(cells, tmp, (size_t)(rows * cols));
        if (stats) {
            stats[4 * s + 0] = (uint32_t)count_value(cells, rows * cols, LR);
            stats[4 * s + 1] = (uint32_t)moved_lr;
            stats[4 * s + 2] = (uint32_t)count_value(cells, rows * cols, TB);
            stats[4 * s + 3] = (uint32_t)moved_tb;
        }
    }
    (void)nt;
}

/* ------------------------------------------------------------------------ */
/* Model III (Sec. 2): a cell may hold an LR and a TB car at once (value 3 = */
/* LR | TB).  The paper gives one sentence; the reading here keeps Model   */
/* II's one-phase update and changes only the conflict: every car may       */
/* advance in one phase per step, moving when its target cell (right for    */
/* LR, below for TB) holds no car before the step, and an EMPTY cell wanted */
/* by both an LR car (its left neighbour) and a TB car (its top neighbour)  */
/* takes both.  A doubly occupied cell blocks cars of either type, like any */
/* occupied cell, and each of its two cars leaves by its own rule.  Torus   */
/* only.  stats per step: n_lr, moved_lr, n_tb, moved_tb after that phase,  */
/* a doubly occupied cell counting once in n_lr and once in n_tb.           */
/* Parity unpinned against the paper, which states Model III in one         */
/* sentence; the tests pin the code to the reading above.                   */
/* ------------------------------------------------------------------------ */
#define BOTH (LR | TB)

static int64_t count_bit(const uint8_t *cells, int64_t n, uint8_t bit)
{
    int64_t c = 0;
    for (int64_t k = 0; k < n; k++)
        c += (cells[k] & bit) != 0;
    return c;
}

static void model3_rows(int64_t r0, int64_t r1, int64_t rows, int64_t cols,
                        const uint8_t *cur, uint8_t *next, int64_t *moved_lr,
                        int64_t *moved_tb)
{
    for (int64_t i = r0; i < r1; i++) {
        int64_t up = (i - 1 + rows) % rows, down = (i + 1) % rows;
        for (int64_t j = 0; j < cols; j++) {
            int64_t left = (j - 1 + cols) % cols, right = (j + 1) % cols;
            uint8_t c = cur[i * cols + j], out = EMPTY;
            if (c & LR) {
                if (cur[i * cols + right] == EMPTY)
                    (*moved_lr)++;            /* the LR car leaves */
                else
                    out |= LR;
            }
            if (c & TB) {
                if (cur[down * cols + j] == EMPTY)
                    (*moved_tb)++;            /* the TB car leaves */
                else
                    out |= TB;
            }
            if (c == EMPTY) {                 /* arrivals, possibly both */
                if (cur[i * cols + left] & LR)
                    out |= LR;
                if (cur[up * cols + j] & TB)
                    out |= TB;
            }
            next[i * cols + j] = out;
        }
    }
}

void bmlo_run_model3(int64_t rows, int64_t cols, uint8_t *cells, uint8_t *tmp, int64_t steps,
                     uint32_t *stats, int32_t n_threads)
{
    int nt = n_threads > 0 ? n_threads : 1;
    for (int64_t s = 0; s < steps; s++) {
        int64_t moved_lr = 0, moved_tb = 0;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : moved_lr, moved_tb)
#endif
        for (int64_t i = 0; i < rows; i++) {
            int64_t ml = 0, mt = 0;
            model3_rows(i, i + 1, rows, cols, cells, tmp, &ml, &mt);
            moved_lr += ml;
            moved_tb += mt;
        }
        memcpy(cells, tmp, (size_t)(rows * cols));
        if (stats) {
            stats[4 * s + 0] = (uint32_t)count_bit(cells, rows * cols, LR);
            stats[4 * s + 1] = (uint32_t)moved_lr;
            stats[4 * s + 2] = (uint32_t)count_bit(cells, rows * cols, TB);
            stats[4 * s + 3] = (uint32_t)moved_tb;
        }
    }
    (void)nt;
}

/* Many independent square lattices, one lattice per thread at a time
 * (dynamic schedule): lattice b has sizes[b] x sizes[b] cells starting at
 * cells + offsets[b]; its per-step counts (4 per step, as in bmlo_run) go to
 * stats + stats_offsets[b] when stats is not NULL.  Returns 0, or -1 if
 * scratch could not be allocated. */
int32_t bmlo_run_many(int64_t count, const int64_t *sizes,
                      const int64_t *offsets, uint8_t *cells,
                      const int64_t *stats_offsets, uint32_t *stats,
                      int64_t steps, int32_t n_threads)
{
    int nt = n_threads > 0 ? n_threads : 1;
    int32_t status = 0;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
#endif
    for (int64_t b = 0; b < count; b++) {
        int64_t n = sizes[b];
        uint8_t *tmp = (uint8_t *)malloc((size_t)(n * n));
        if (!tmp) {
            status = -1;
            continue;
        }
        bmlo_run(n, n, cells + offsets[b], tmp, steps,
                 stats ? stats + stats_offsets[b] : NULL, 1);
        free(tmp);
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* 2-bitplane packed form.  The paper notes that two bits per cell would    */
/* suffice (Sec. 3).  Layout used by the project: two planes of             */
/* rows x (cols/32) 32-bit words, row-major; bit b of word w in row i is    */
/* cell (i, 32w + b), least significant bit = leftmost cell.  Plane `lr`    */
/* has a 1 where the cell is LR, plane `tb` where it is TB.  cols must be a */
/* multiple of 32.                                                           */
/* ------------------------------------------------------------------------ */
void bmlo_pack(int64_t rows, int64_t cols, const uint8_t *cells,
               uint32_t *lr, uint32_t *tb)
{
    int64_t words = cols / 32;
    for (int64_t i = 0; i < rows; i++) {
        for (int64_t w = 0; w < words; w++) {
            uint32_t a = 0, b = 0;
            for (int bit = 0; bit < 32; bit++) {
                uint8_t c = cells[i * cols + 32 * w + bit];
                if (c == LR)
                    a |= 1u << bit;
                if (c == TB)
                    b |= 1u << bit;
            }
            lr[i * words + w] = a;
            tb[i * words + w] = b;
        }
    }
}

/* Inverse of bmlo_pack.  A position set in both planes is not a valid
 * state; it is written as 3 so that a caller can detect it. */
void bmlo_unpack(int64_t rows, int64_t cols, const uint32_t *lr,
                 const uint32_t *tb, uint8_t *cells)
{
    int64_t words = cols / 32;
    for (int64_t i = 0; i < rows; i++) {
        for (int64_t j = 0; j < cols; j++) {
            uint32_t a = (lr[i * words + j / 32] >> (j % 32)) & 1u;
            uint32_t b = (tb[i * words + j / 32] >> (j % 32)) & 1u;
            cells[i * cols + j] = (uint8_t)(a * LR + b * TB);
        }
    }
}
