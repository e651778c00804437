/*
 * bml.h -- C ABI of libbml: the Biham-Middleton-Levine (BML) Model I traffic
 * automaton on AMD Instinct MI355X (gfx950).
 *
 * Model (M. Marzolla, "Parallel Implementations of Cellular Automata for
 * Traffic Models", arXiv:1804.07981, Sec. 2): an N x N lattice with periodic
 * boundaries; every cell is EMPTY (0), LR (1, moves left to right) or TB
 * (2, moves top to bottom).  One step is a horizontal phase -- every LR car
 * whose right neighbour (i, j+1 mod N) is EMPTY moves there -- followed by a
 * vertical phase -- every TB car whose lower neighbour (i+1 mod N, j) is
 * EMPTY moves there.  Both phases are synchronous: every decision is taken
 * on the lattice as it was before the phase (Sec. 3).  Cells are stored
 * row-major, cell (i, j) at index i*N + j (Sec. 3).
 *
 * Conventions for every function below:
 *   - Return value: BML_OK (0) or a negative BML_E* code.  Nothing aborts or
 *     throws; bml_last_error() gives a message for the calling thread.
 *   - Device pointers are caller-owned device memory (hipMalloc or a torch
 *     tensor) that must stay alive until bml_free / bml_batch_free.  Host
 *     pointers are only read or written during the call.
 *   - `hip_stream` is a caller-owned hipStream_t (NULL = the null stream).
 *     Work is enqueued on it asynchronously unless a function says it
 *     synchronises.
 *   - One handle is used by one host thread at a time.
 *   - Lattice size: 32 <= N <= 65504 and N a multiple of 32 (so a row is a
 *     whole number of 32-cell words and every count fits in 32 bits).
 */
#ifndef BML_H
#define BML_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BML_OK = 0,
    BML_EINVAL = -1,    /* bad argument: NULL, size, layout, rho, cell value, alignment */
    BML_EDEVICE = -2,   /* a HIP runtime call failed (message names it) */
    BML_ERANGE = -3,    /* requested steps outside the retained stats window */
    BML_ESTATE = -4,    /* NULL or already freed handle */
    BML_ECORRUPT = -5   /* a car count differs from the initial one: state corrupted */
};

/* Storage of the lattice state in device memory.
 *   BML_LAYOUT_U8:       N*N bytes, cell (i,j) at byte i*N + j, values 0/1/2
 *                        (the paper's one-byte cell, Sec. 3).
 *   BML_LAYOUT_BITPLANE: two planes of N rows x N/32 uint32 words each, the LR
 *                        plane first then the TB plane; bit b of word w in
 *                        row i is cell (i, 32w + b), least significant bit =
 *                        leftmost cell (two bits per cell suffice, Sec. 3). */
enum { BML_LAYOUT_U8 = 0, BML_LAYOUT_BITPLANE = 1 };

/* Counts of one step (the project's reading of per-phase car counts and
 * moved counts): n_lr = LR cars after the horizontal phase, moved_lr = LR
 * cars that moved in it, n_tb = TB cars after the vertical phase, moved_tb =
 * TB cars that moved in it. */
typedef struct {
    uint32_t n_lr, moved_lr, n_tb, moved_tb;
} bml_step_stats;

typedef struct bml_lattice bml_lattice;   /* opaque, library-owned */

/* Bytes one state buffer needs for an N x N lattice in `layout`
 * (N*N for U8, N*N/4 for BITPLANE).  EINVAL on a bad N or layout. */
int bml_state_bytes(int32_t n, int32_t layout, size_t *bytes);

/* Create a lattice handle and write the initial state into d_state_a.
 *   n, layout    lattice size and storage layout (see above).
 *   seed, rho    used when cells_host is NULL: cell k = i*N + j takes the
 *                k-th output z of the SplitMix64 stream started at state
 *                `seed`; with u = z >> 11 (53 bits) the cell is LR if
 *                u < floor(rho/2 * 2^53), else TB if u < floor(rho * 2^53),
 *                else EMPTY.  The paper only says cars are placed at random
 *                (Sec. 2); this iid draw is the library's reading.  rho must
 *                be in [0, 1].
 *   cells_host   NULL, or N*N host bytes (row-major, values 0..2) to start
 *                from instead (also how a saved state is resumed).
 *   d_state_a/b  two caller-owned device buffers of bml_state_bytes() each,
 *                256-byte aligned, not overlapping; the library ping-pongs
 *                between them (synchronous update via two grids, Sec. 3).
 *   d_stats      caller-owned device ring of stats_cap bml_step_stats; the
 *                counts of global step s land in d_stats[s % stats_cap].
 *   hip_stream   stream every later call of this handle enqueues on.
 * Synchronises the stream once (to read the initial car counts).
 * EINVAL on bad arguments, EDEVICE on a HIP failure. */
int bml_init(bml_lattice **out, int32_t n, int32_t layout, uint64_t seed,
             double rho, const uint8_t *cells_host, void *d_state_a,
             void *d_state_b, bml_step_stats *d_stats, int64_t stats_cap,
             void *hip_stream);

/* Advance the lattice by n_steps steps (n_steps >= 0), asynchronously on the
 * handle's stream.  Each kernel pass advances every tile by up to
 * t_phases/2 steps (see bml_set_tuning).  Only the counts of the last
 * min(n_steps, stats_cap) steps of this call are kept in the ring. */
int bml_step(bml_lattice *L, int64_t n_steps);

/* Copy the counts of steps first_step .. first_step+count-1 (global step
 * numbers, 0 = the first step after bml_init) to out_host.  The steps must
 * have been run and still be in the ring: first_step >= steps_done -
 * stats_cap, else ERANGE.  Synchronises the stream.  Returns ECORRUPT (after
 * filling out_host) if any n_lr or n_tb differs from the initial counts. */
int bml_stats(bml_lattice *L, int64_t first_step, int64_t count,
              bml_step_stats *out_host);

/* Copy the current lattice to out_host as N*N row-major bytes (values 0..2),
 * whatever the layout (a bitplane lattice is unpacked on the device first).
 * Synchronises the stream. */
int bml_get_cells(bml_lattice *L, uint8_t *out_host);

/* Initial car counts computed at bml_init. */
int bml_initial_counts(const bml_lattice *L, uint64_t *n_lr, uint64_t *n_tb);

/* Launch shape of the step kernels: tile_rows = lattice rows one wavefront
 * writes per tile (32 or 64; 64 is used only when it divides N, else 32),
 * t_phases = phases per HBM pass (even, 2..16; each pass advances every
 * tile t_phases/2 steps), waves_per_block = 1, 2 or 4.  0 keeps the current
 * value.  Results do not depend on the tuning; only speed does.  EINVAL on
 * any other value. */
int bml_set_tuning(bml_lattice *L, int32_t tile_rows, int32_t t_phases,
                   int32_t waves_per_block);
int bml_get_tuning(const bml_lattice *L, int32_t *tile_rows, int32_t *t_phases,
                   int32_t *waves_per_block);

/* Steps run since bml_init (-1 for a NULL handle). */
int64_t bml_step_count(const bml_lattice *L);

/* The caller buffer (d_state_a or d_state_b) that holds the current state
 * (NULL for a NULL handle). */
const void *bml_current_state(const bml_lattice *L);

/* Release the handle (and the library's own small scratch).  Synchronises
 * the stream first.  Never frees caller memory.  NULL is ignored. */
void bml_free(bml_lattice *L);

/* Message describing the last error on the calling thread ("" if none). */
const char *bml_last_error(void);

/* ---------------- device-buffer helpers (no handle) ---------------------- */

/* Pack N*N bytes (values 0..2) at d_cells into the two planes at d_planes
 * (layout as BML_LAYOUT_BITPLANE), and the inverse.  Asynchronous. */
int bml_pack(int32_t n, const uint8_t *d_cells, uint32_t *d_planes,
             void *hip_stream);
int bml_unpack(int32_t n, const uint32_t *d_planes, uint8_t *d_cells,
               void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* BML_H */
