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

/* Lattice topologies.  TORUS: both directions periodic (the model of
 * Sec. 2).  KLEIN: left and right edges periodic, top and bottom edges
 * glued with a reversal (the Klein-bottle lattice Sec. 2 cites): a TB car
 * leaving the bottom row in column j enters the top row in column
 * cols-1-j.  LR cars never cross that edge. */
enum { BML_TOPO_TORUS = 0, BML_TOPO_KLEIN = 1 };

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
 *                from instead (also how a saved state is resumed); value 3
 *                (an LR and a TB car in one cell) is accepted too, but such
 *                a lattice steps only under Model III (bml_set_model).
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

/* Rectangular and asymmetric lattices (Sec. 2 lists an unequal number of LR
 * and TB cars among the model's extensions; the rules of Sec. 2 apply
 * unchanged to `rows` x `cols` cells with both directions periodic).
 *   rows         32..65504 (any count); cols: a multiple of 32 in
 *                [32, 65504].  Cells are row-major, cell k = i*cols + j; a
 *                bitplane row is cols/32 words, each plane rows*cols/32 words.
 *   rho_lr, rho_tb  when cells_host is NULL: cell k is LR if
 *                u < floor(rho_lr * 2^53), else TB if
 *                u < floor((rho_lr + rho_tb) * 2^53) (the sum rounded as an
 *                IEEE double), else EMPTY, with u as for bml_init; both >= 0
 *                and their sum <= 1.  bml_init(n, rho) is exactly
 *                bml_init_rect(n, n, rho/2, rho/2).
 * Everything else (buffers, ring, stream, errors, later calls) is as for
 * bml_init; bml_get_cells returns rows*cols bytes; bml_step_group needs
 * equal rows, cols, topology and model. */
int bml_state_bytes_rect(int32_t rows, int32_t cols, int32_t layout, size_t *bytes);
int bml_init_rect(bml_lattice **out, int32_t rows, int32_t cols, int32_t layout,
                  uint64_t seed, double rho_lr, double rho_tb, const uint8_t *cells_host,
                  void *d_state_a, void *d_state_b, bml_step_stats *d_stats,
                  int64_t stats_cap, void *hip_stream);

/* Advance the lattice by n_steps steps (n_steps >= 0), asynchronously on the
 * handle's stream.  Each kernel pass advances every tile by up to
 * t_phases/2 steps (see bml_set_tuning).  Only the counts of the last
 * min(n_steps, stats_cap) steps of this call are kept in the ring.  The
 * step count, the current buffer of the ping-pong pair and the ring slots
 * are kept on the host, so a call captured into a graph would replay with
 * stale ones: to replay step sequences, use the batch API
 * (bml_batch_capture), whose kernels read that state from device memory. */
int bml_step(bml_lattice *L, int64_t n_steps);

/* Device-to-device copy of `bytes` (a multiple of 16) from d_src to d_dst
 * (256-byte aligned, not overlapping), asynchronously on hip_stream, with a
 * plain streaming kernel.  Not part of the automaton: it is the bandwidth
 * reference that benchmarks report next to the step kernels (a kernel that
 * reads and writes every byte once).  EINVAL on bad arguments, EDEVICE on a
 * HIP failure. */
int bml_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream);

/* Advance `count` lattices (1..8) by n_steps each in joint launches: every
 * kernel pass advances all of them, their strips spread over the device as
 * one grid (several small lattices fill the GPU better together than one
 * after another or on separate streams).  The handles must be distinct and
 * share N, layout, tuning (bml_set_tuning), device and stream; their step
 * counts and stats rings may differ, and each lattice's ring and counts
 * behave exactly as if bml_step had been called on it alone.  Results are
 * identical to stepping each lattice alone.  EINVAL on a bad count, a
 * repeated handle or a mismatch, ESTATE on an invalid handle. */
int bml_step_group(bml_lattice *const *handles, int32_t count, int64_t n_steps);

/* Allocation-free stepping, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the launches of bml_step_group on caller buffers, with no
 * handle and no library-allocated memory.  The per-launch stats-reduction
 * scratch lives in a static device array of the library, sized for
 * BML_STATIC_MAX_LATTICES lattices (about 1 KiB each); each device that
 * calls this holds its own copy until the process ends.
 *   count        lattices, 1..BML_STATIC_MAX_LATTICES (EINVAL beyond)
 *   rows, cols, layout  as for bml_init_rect; the same for every lattice
 *   d_state_a/b  count device buffers each (host arrays of device
 *                pointers): lattice i's state at step first_step is in
 *                d_state_a[i]; the buffers ping-pong as for bml_init
 *   d_stats      count device rings of stats_cap bml_step_stats: the counts
 *                of global step s land in slot s % stats_cap; only the last
 *                min(n_steps, stats_cap) steps of the call are kept
 *   first_step   global number of the first step (for the ring slots)
 *   t_phases     phases per kernel pass (even, 2..16), as bml_set_tuning;
 *                strip height automatic, 4 waves per block
 *   result_in_b  out: 1 if the states after the call are in d_state_b,
 *                0 if in d_state_a
 * Model of Sec. 2 on the torus.  Asynchronous on hip_stream.  The counts
 * are written but not checked: compare n_lr / n_tb with the initial car
 * counts to detect corruption.  Every call on one device shares that
 * device's scratch array, so calls that overlap in time on one device (two
 * host threads, or two streams running at once) race: serialise them.
 * EINVAL on bad arguments, EDEVICE on a HIP failure. */
#define BML_STATIC_MAX_LATTICES 8
int bml_step_group_static(int32_t count, int32_t rows, int32_t cols, int32_t layout,
                          void *const *d_state_a, void *const *d_state_b,
                          bml_step_stats *const *d_stats, int64_t stats_cap,
                          int64_t first_step, int64_t n_steps, int32_t t_phases,
                          void *hip_stream, int32_t *result_in_b);

/* Copy the counts of steps first_step .. first_step+count-1 (global step
 * numbers, 0 = the first step after bml_init) to out_host.  The steps must
 * have been run and still be in the ring: first_step >= steps_done -
 * stats_cap, else ERANGE.  Synchronises the stream.  Returns ECORRUPT (after
 * filling out_host) if any n_lr or n_tb differs from the initial counts. */
int bml_stats(bml_lattice *L, int64_t first_step, int64_t count,
              bml_step_stats *out_host);

/* Copy the current lattice to out_host as N*N (rows*cols) row-major bytes (values 0..2,
 * and 3 for a cell holding both cars under Model III), whatever the layout (a
 * bitplane lattice is unpacked on the device first).
 * Synchronises the stream. */
int bml_get_cells(bml_lattice *L, uint8_t *out_host);

/* Initial car counts computed at bml_init. */
int bml_initial_counts(const bml_lattice *L, uint64_t *n_lr, uint64_t *n_tb);

/* Topology of the lattice for the steps that follow (BML_TOPO_TORUS after
 * init).  The state layout does not change.  EINVAL on an unknown value,
 * ESTATE on an invalid handle.  bml_get_topology returns it (or ESTATE). */
int bml_set_topology(bml_lattice *L, int32_t topology);
int bml_get_topology(const bml_lattice *L);

/* Update rule for the steps that follow.  model 1 (after init): the model
 * of Sec. 2, a horizontal then a vertical phase per step.  model 2: Model II
 * (Sec. 2): every car advances in one phase per step when its target cell
 * (right for LR, below for TB) is EMPTY before the step; an EMPTY cell that
 * is the target of both an LR car and a TB car goes to one of them by a fair
 * coin.  The paper gives no distribution; here, at global step s (the
 * handle's step count), the coin of cell (i, j) is bit (j mod 32) of the low
 * 32 bits of the SplitMix64 output number s*rows*W + i*W + j/32 of the stream
 * started at `coin_seed` (W = cols/32), 1 meaning the LR car moves.  The
 * counts of a Model II step are taken after its one phase, and a kernel
 * pass still advances t_phases/2 steps (bml_set_tuning).  model 3: Model III
 * (Sec. 2: a cell may hold an LR and a TB car).  The paper gives one
 * sentence; here it is the one-phase step of Model II in which an EMPTY
 * cell wanted by both an LR and a TB car takes both (cell value 3, LR and
 * TB bits both set; coin_seed unused).  A car still moves only into a cell
 * that held no car before the step, so a doubly occupied cell blocks both
 * types, and each of its cars leaves by its own rule; counts are taken
 * after the phase, a doubly occupied cell counting once in n_lr and once in
 * n_tb.  A lattice that has run Model III steps, or was initialised with a
 * value-3 cell, stays on Model III: selecting model 1 or 2 for it is EINVAL,
 * and so is stepping it (bml_step, bml_step_group) under model 1 before
 * Model III is selected.  Models II and III run on the torus only: EINVAL
 * with the Klein topology, or for another model value; ESTATE on an
 * invalid handle. */
int bml_set_model(bml_lattice *L, int32_t model, uint64_t coin_seed);
/* The update rule in force (1, 2 or 3), or ESTATE on an invalid handle. */
int bml_get_model(const bml_lattice *L);

/* Launch shape of the step kernels.  Each wavefront streams down a strip of
 * the lattice `tile_rows` output rows tall (plus t_phases/2 halo rows above
 * and below), advancing every row t_phases/2 steps per pass (t_phases even,
 * 2..16).  A strip is 62 words (1984 cells) wide, or, for N = 2048 and 4096,
 * the whole row (one wavefront holds a row, so x needs no halo).
 * tile_rows = 0 picks the strip height from the occupancy of the device;
 * otherwise 1 <= tile_rows <= 65504.  waves_per_block = 1, 2 or 4.  A
 * negative tile_rows, or a t_phases / waves_per_block <= 0, keeps the
 * current value.  Results do not depend on the tuning; only speed does.
 * EINVAL on any other value. */
int bml_set_tuning(bml_lattice *L, int32_t tile_rows, int32_t t_phases,
                   int32_t waves_per_block);
int bml_get_tuning(const bml_lattice *L, int32_t *tile_rows, int32_t *t_phases,
                   int32_t *waves_per_block);

/* Register-resident tile kernel.  steps = 0 (the default): the streaming
 * kernel above.  steps = K (even, 2..32): each launch advances the lattice
 * K steps with the state held in registers: a workgroup loads a tile of
 * 1024 columns (512 or 256 when the lattice, or the group of lattices
 * stepped together, is too small to give every compute unit two such
 * tiles) by up to 512 - 2K rows together with one 32-cell halo word
 * on each side and K halo rows above and below, advances it K steps
 * (both phases of Sec. 2 per step, synchronous as in Sec. 3, or Model III's
 * one phase) and stores the tile's own cells, which are exact because what
 * the held block does not know moves at most one cell and one row per step.
 * The state is read and written once per K steps.  Needs the model of
 * Sec. 2 (on the torus or on the Klein bottle above, where a tile of the
 * first or last slab holds the rows across the glued edge mirrored) or
 * Model III on the torus (bml_set_model; Model II is refused
 * here and, once the tile kernel is on, by bml_set_model), rows a multiple
 * of 32 and columns a multiple of 256 (EINVAL otherwise; the
 * library then keeps the streaming kernel), and allocates a small count
 * buffer with the handle (EDEVICE if that fails).  Synchronises the stream.
 * bml_get_resident returns K (0 = streaming), < 0 on error.  Results do not
 * depend on the kernel; only speed does. */
int bml_set_resident(bml_lattice *L, int32_t steps);
int bml_get_resident(const bml_lattice *L);

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

/* ---------------- batched sweeps -------------------------------------------
 * Many independent lattices of (possibly) different N advanced together: one
 * kernel launch per pass covers every active lattice, and a run of passes
 * can be captured once in a hipGraph and replayed.  Each lattice starts from
 * SplitMix64 stream seed[b] at density rho[b] as in bml_init.  Per step and
 * lattice the number of LR and TB cars that moved is written to a trace:
 * trace[(b * trace_steps + s) * 2 + 0] = LR moved, ... + 1] = TB moved, for
 * global step s < trace_steps (s counts every step the batch ran; a lattice
 * that was inactive during a step has 0 there).  Car counts are conserved;
 * bml_batch_check verifies that.  Batches run the two-phase rule of Sec. 2
 * on square tori (the single-lattice API covers the other rules, shapes
 * and topologies). */
typedef struct bml_batch bml_batch;

/* Bytes of the caller-owned device arena that holds two state buffers per
 * lattice (each rounded up to 256 bytes). */
int bml_batch_arena_bytes(int32_t count, const int32_t *n, int32_t layout, size_t *bytes);

/* n, rho, seed: host arrays of `count` entries.  d_arena: caller device
 * memory of bml_batch_arena_bytes(), 256-byte aligned.  d_trace: caller
 * device memory of count * trace_steps * 2 uint32, 256-byte aligned.
 * Synchronises the stream (initial car counts).  Every lattice is active. */
int bml_batch_init(bml_batch **out, int32_t count, const int32_t *n, const double *rho,
                   const uint64_t *seed, int32_t layout, void *d_arena, size_t arena_bytes,
                   uint32_t *d_trace, int64_t trace_steps, void *hip_stream);

/* strip_rows: target strip height (the largest divisor of each N not above
 * it is used), t_phases: even, 2..16, waves_per_block: 1, 2 or 4; values
 * <= 0 keep the current setting.  Drops a captured graph.  Synchronises. */
int bml_batch_set_tuning(bml_batch *B, int32_t strip_rows, int32_t t_phases,
                         int32_t waves_per_block);

/* Register-resident runs.  When every lattice of the batch has N <= max_n
 * (max_n in [0, 1024]; 0 = never; the default is 1024), runs use a kernel
 * in which the lattices live in the registers of workgroups for many
 * steps: two rows per lane, the horizontal phase inside the lane, the
 * vertical phase through the lane's two rows, neighbouring lanes and,
 * across wavefronts, LDS, one barrier per step.  A workgroup holds up to
 * 512 rows; a taller lattice is cut into the fewest slabs of rows that
 * fit one, each held with K halo rows above and below in a workgroup of its
 * own, and a launch then runs at most K steps (the halo rows are
 * recomputed and absorb what the slab's edges cannot know for K steps).
 * split_steps sets K (a multiple of 16, at most 240; 0 = 64); a batch with
 * no lattice taller than 512 runs a whole run in one launch.  The state is
 * read once at the start of a launch and written once at the end.
 * Otherwise the streaming kernel runs, one launch per pass of t_phases/2
 * steps (bml_batch_set_tuning).  Results are identical either way.  Drops
 * a captured graph.  Synchronises.  bml_batch_get_resident: 1 if runs are
 * register-resident, 0 if streaming, < 0 on error. */
int bml_batch_set_resident(bml_batch *B, int32_t max_n, int32_t split_steps);
int bml_batch_get_resident(const bml_batch *B);

/* active_host: `count` bytes, non-zero = the lattice advances in later runs
 * (NULL = all).  Inactive lattices keep their state.  Synchronises. */
int bml_batch_set_active(bml_batch *B, const uint8_t *active_host);

/* Enqueue n_steps steps of every active lattice (asynchronous). */
int bml_batch_run(bml_batch *B, int64_t n_steps);

/* Capture bml_batch_run(B, n_steps) into a hipGraph (nothing runs), and
 * replay it with bml_batch_replay (asynchronous).  The graph reads the step
 * counter, the parities and the active list from device memory, so replays
 * continue where the batch stands.  Needs a non-null stream. */
int bml_batch_capture(bml_batch *B, int64_t n_steps);
int bml_batch_replay(bml_batch *B);

/* Global steps run (-1 for a bad handle); steps run by lattice idx. */
int64_t bml_batch_step_count(const bml_batch *B);
int bml_batch_lattice_steps(const bml_batch *B, int32_t idx, int64_t *steps);

/* Initial car counts of lattice idx. */
int bml_batch_initial_counts(const bml_batch *B, int32_t idx, uint64_t *n_lr, uint64_t *n_tb);

/* Copy lattice idx to out_host (N*N bytes, values 0..2).  Synchronises. */
int bml_batch_get_cells(bml_batch *B, int32_t idx, uint8_t *out_host);

/* Recount every lattice: ECORRUPT if any car count changed.  Synchronises. */
int bml_batch_check(bml_batch *B);

/* Release the handle and the library's scratch (synchronises first). */
void bml_batch_free(bml_batch *B);

/* ---------------- learned early exit ------------------------------------------
 * Below a critical density a BML lattice settles into free flow, above it
 * into a global jam, with both possible near the critical point (Sec. 2).
 * A small MLP reads a lattice's early mobile-fraction trajectory and its
 * density and predicts which: 65 inputs -> 64 (ReLU) -> 64 (ReLU) -> 1 logit
 * (p = sigmoid(logit) = probability of a jam).  Its BML_MLP_PARAMS fp32
 * parameters are one array, row-major (out x in):
 *   W1[64][65] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
 * All pointers below are device pointers; all calls are asynchronous. */
#define BML_MLP_INPUTS 65
#define BML_MLP_HIDDEN 64
#define BML_MLP_PARAMS 8449
#define BML_MLP_MAX_BATCH 256

/* out[b][m] (m < 64) = (sum over steps window*m .. window*m+window-1 of
 * trace LR moved + TB moved) / (window * cars[b]), computed in double and
 * rounded to float (1 for a lattice without cars); out[b][64] = rho[b].
 * trace as in bml_batch_init ([count][trace_steps][2] uint32); 64 windows
 * must fit in trace_steps. */
int bml_features(const uint32_t *d_trace, int64_t trace_steps, int32_t count,
                 const uint64_t *d_cars, const double *d_rho, int32_t window,
                 float *d_out, void *hip_stream);

/* frozen[b] = 1 if some global step in [first_step, end_step) of lattice b
 * moved no car (such a lattice is a fixed point from then on: the exact
 * stop rule), else 0. */
int bml_trace_frozen(const uint32_t *d_trace, int64_t trace_steps, int32_t count,
                     int64_t first_step, int64_t end_step, uint8_t *d_frozen, void *hip_stream);

/* mean[b] = mean over steps [first_step, end_step) of the mobile fraction
 * (LR moved + TB moved) / cars[b], in double (1 without cars). */
int bml_trace_mobility(const uint32_t *d_trace, int64_t trace_steps, int32_t count,
                       const uint64_t *d_cars, int64_t first_step, int64_t end_step,
                       double *d_mean, void *hip_stream);

/* Column means and standard deviations (population) of x[n][65], and the
 * in-place standardisation x = (x - mean) / std in float. */
int bml_feature_stats(const float *d_x, int32_t n, float *d_mean, float *d_std,
                      void *hip_stream);
int bml_standardize(float *d_x, int32_t n, const float *d_mean, const float *d_std,
                    void *hip_stream);

/* Device scratch bml_mlp_grad / bml_mlp_train_step need. */
size_t bml_mlp_scratch_bytes(void);

/* Gradient (fp32) of the mean binary cross-entropy with logits of samples
 * x[0..n), labels y (1 = jammed), 1 <= n <= 256, into grad[8449]; the loss
 * into *loss. */
int bml_mlp_grad(const float *d_params, const float *d_x, const float *d_y, int32_t n,
                 void *d_scratch, float *d_grad, float *d_loss, void *hip_stream);

/* One Adam step (t = 1, 2, ...) on the minibatch x[idx[0..n)] (n <= 256):
 * the gradient as above, then m, v and params updated in place. */
int bml_mlp_train_step(float *d_params, float *d_m, float *d_v, float *d_grad, int64_t t,
                       const float *d_x, const float *d_y, const int32_t *d_idx, int32_t n,
                       float lr, float beta1, float beta2, float eps, void *d_scratch,
                       float *d_loss, void *hip_stream);

/* Logits of n samples: fp32, and BF16 (weights and every layer's input
 * rounded to bfloat16, nearest-even; biases and accumulation in fp32). */
int bml_mlp_forward(const float *d_params, const float *d_x, int32_t n, float *d_logits,
                    void *hip_stream);
int bml_mlp_infer_bf16(const float *d_params, const float *d_x, int32_t n, float *d_logits,
                       void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* BML_H */
