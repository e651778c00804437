// bml_pass.hpp -- the temporally blocked BML step kernel (gfx950).
//
// One launch advances the lattice K steps (2K phases) with one read and one
// write of the state (temporal blocking).  The lattice is cut into strips
// of H output rows; a wavefront streams its strip top to bottom through a
// pipeline of K levels held in VGPRs, level k turning rows after k steps
// into rows after k + 1 steps (bml_tile.hpp).  The strip is read with K
// halo rows above and below, addressed modulo N, so no ghost cells are ever
// stored (the ghost cells of Marzolla, arXiv:1804.07981, Sec. 3, become
// modular addressing of the halo); each step invalidates one more halo row
// at each end, so exactly the H strip rows leave the last level exact.
//
// Columns: in tile mode a wavefront covers 62 words (lanes 1..62) plus a
// halo word on each side (lanes 0 and 63), whose edge bits go stale one cell
// per step, far from the exact words for K <= 8.  In row mode (rows of 2048 or
// 4096) the wavefront holds a whole row, one or two words per lane, and the
// lane moves wrap around the wavefront, so x is periodic with no halo lanes
// and no tile of a row is left partly used.
//
// Memory access: buffer loads/stores with the per-lane word offset in a VGPR
// and the row offset in an SGPR; rows are prefetched D rows ahead of the
// pipeline into a register ring.  Byte lattices are converted to bitplanes
// in registers after loading and back before storing.
//
// Grids are persistent: every wavefront walks a strided list of strips.
// Blocks are dispatched round-robin over the 8 XCDs, so block b is mapped to
// the (b % 8)-th eighth of every round of strips: each XCD works on a band
// of vertically adjacent strips, which share halo rows in that XCD's L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "bml_tile.hpp"

namespace bml {

enum { IO_U8 = 0, IO_BP = 1 };
enum { TOPO_TORUS = 0, TOPO_KLEIN = 1 };
constexpr int MAX_K = 8;        // steps per pass
constexpr int TILE_WORDS = 62;  // output words per wavefront tile (lanes 1..62)

constexpr int ACC_STRIPES = 8;  // one stats accumulator stripe per XCD

// Library-owned scratch of the stats reduction; all zero between launches.
struct PassScratch {
    uint32_t acc[ACC_STRIPES][MAX_K][4];
    uint32_t ticket;
};

constexpr int MAX_GROUP = 8;    // lattices advanced by one launch

// One lattice of a launch.
struct PassLattice {
    const void *src;
    void *dst;
    uint32_t *stats;         // caller's ring, 4 u32 per slot
    PassScratch *scratch;    // its stats reduction scratch
    uint32_t rec_mask;       // bit k set: record the counts of step k of this pass
    int32_t slot[MAX_K];     // ring slot of step k
    int32_t pad;
    uint64_t step0;          // Model II: global index of the pass's first step
    uint64_t coin_seed;      // Model II: stream of the conflict coins
};

// A launch advances n_lat lattices of the same size and layout by K steps;
// their work items (strips) are numbered lattice-major in one list, so one
// grid spreads the strips of all of them evenly over the device.
struct PassArgs {
    PassLattice lat[MAX_GROUP];
    int32_t n_lat;
    int32_t rows;            // lattice rows
    int32_t words;           // 32-cell words per row (columns / 32)
    int32_t tiles_x;         // column blocks across a row (62 words each)
    int32_t n_tiles;         // tiles_x * ceil(n / strip_rows) work items per lattice
    int32_t strip_rows;      // output rows per strip
    int32_t xcd_split;       // 1: gridDim.x % 8 == 0, give each XCD a band of tiles
    uint32_t any_rec;        // OR of the lattices' rec_mask
};

using PassFn = void (*)(PassArgs);

// Buffer resource of a state buffer of `bytes` bytes: raw (untyped)
// addressing, no stride.  The hardware checks every access against `bytes`:
// a load beyond it returns 0 and a store beyond it is dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes,
                                             0x00020000);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Rows prefetched ahead of the pipeline (register ring depth) for byte and
// bitplane rows, one or two words per lane.  Deeper rings hide more memory
// latency but cost VGPRs; these keep every variant within 256 VGPRs (no
// accumulation-register spills) and at two or more waves per SIMD.
constexpr int U8_RING = 4, BP_RING = 8;     // one word per lane
constexpr int U8_RING2 = 1, BP_RING2 = 2;   // two words per lane

// ROW = 0: tile mode, any row length; a wavefront covers 62 words plus a
// halo lane on each side.  ROW = m > 0: row mode for rows of 2048 m cells;
// the wavefront holds a whole row, m words per lane, and the lane moves wrap
// around it (periodic in x without halo lanes, every lane exact).
// TOPO = TOPO_TORUS: both directions periodic.  TOPO = TOPO_KLEIN: the top
// and bottom edges are glued with a reversal (a Klein bottle).  A strip then
// holds the halo rows that lie across that edge mirrored, in the strip's own
// frame: a lane loads the mirror word (columns counted from the other side)
// and reverses its bits, and the horizontal phase of those rows runs towards
// lower bit indices.  In that frame the vertical neighbours of every row are
// simply the rows before and after it.  Output rows never lie across the
// edge, so stores and counts are unchanged.
// MODEL = 1: the model of Sec. 2 (horizontal then vertical phase).
// MODEL = 2: Model II (both car types in one phase, a coin on conflicts;
// level_push_model2), torus only.
// MODEL = 3: Model III (one phase; a contested cell takes both cars;
// level_push_model3), torus only.
template <int IO, int K, int ROW, int TOPO, int MODEL>
__global__ __launch_bounds__(256) void pass_kernel(PassArgs a)
{
    static_assert(K >= 1 && K <= MAX_K, "bad steps per pass");
    static_assert(MODEL == 1 || ((MODEL == 2 || MODEL == 3) && TOPO == TOPO_TORUS),
                  "Models II and III on the torus");
    static_assert(ROW >= 0 && ROW <= 2, "row mode holds at most 2 words per lane");
    constexpr int WL = ROW ? ROW : 1;        // words per lane
    constexpr bool WRAP = ROW > 0;
    constexpr int D = IO == IO_U8 ? (WL > 1 ? U8_RING2 : U8_RING)
                                  : (WL > 1 ? BP_RING2 : BP_RING);
    constexpr int NW = (IO == IO_U8 ? 8 : 2) * WL;   // dwords one lane loads per row
    const int lane = threadIdx.x & 63;
    // Wave-uniform values must be visibly uniform so that strip and row
    // offsets live in SGPRs (buffer soffset) rather than per-lane VGPRs.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int total_waves = gridDim.x * wpb;
    int first;
    if (a.xcd_split) {
        const int per_xcd = gridDim.x >> 3;
        first = ((blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3)) * wpb + wave;
    } else {
        first = blockIdx.x * wpb + wave;
    }
    const uint32_t row_bytes = (uint32_t)a.words * (IO == IO_U8 ? 32u : 4u);
    const uint32_t plane_bytes = row_bytes * (uint32_t)a.rows;   // lattice bytes (one plane)
    const uint32_t state_bytes = IO == IO_U8 ? plane_bytes : 2u * plane_bytes;
    const int H = a.strip_rows;

    // Counts: wave totals (uniform) of the lattice being worked on, moved
    // to the block's LDS slot of that lattice when the wave changes lattice
    // and at the end.
    __shared__ uint32_t red[MAX_GROUP][MAX_K * 4];
    __shared__ uint32_t is_last;
    for (int i = threadIdx.x; i < MAX_GROUP * MAX_K * 4; i += blockDim.x)
        (&red[0][0])[i] = 0;
    __syncthreads();
    uint32_t wtot[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
        wtot[k][0] = wtot[k][1] = wtot[k][2] = wtot[k][3] = 0;
    int cur = -1;   // lattice of wtot
    auto flush = [&]() {
        if (cur >= 0 && lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (wtot[k][q])
                        atomicAdd(&red[cur][k * 4 + q], wtot[k][q]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            wtot[k][0] = wtot[k][1] = wtot[k][2] = wtot[k][3] = 0;
    };

    const int all_items = a.n_lat * a.n_tiles;
    for (int item = first; item < all_items; item += total_waves) {
        const int li = item / a.n_tiles;               // lattice of this item
        const int local = item - li * a.n_tiles;
        if (li != cur) {
            flush();
            cur = li;
        }
        const __amdgpu_buffer_rsrc_t src = make_rsrc(a.lat[li].src, state_bytes);
        const __amdgpu_buffer_rsrc_t dst = make_rsrc(a.lat[li].dst, state_bytes);
        const int sy = local / a.tiles_x;
        const int tx = local - sy * a.tiles_x;
        const int row_a = sy * H;                       // first output row
        const int h = min(H, a.rows - row_a);           // output rows of this strip
        const int total_in = h + 2 * K;                 // input rows streamed
        const int total_it = h + 3 * K - 1;             // pipeline iterations
        uint32_t word;   // first word of this lane
        bool lane_ok;    // lane holds exact output words
        if constexpr (ROW > 0) {
            word = (uint32_t)(lane * WL);
            lane_ok = true;
        } else {
            const int w0 = tx * TILE_WORDS;
            const int vwords = min(TILE_WORDS, a.words - w0);
            word = (uint32_t)((w0 + lane - 1 + a.words) % a.words);
            lane_ok = lane >= 1 && lane <= vwords;
        }
        const uint32_t voff = IO == IO_U8 ? word * 32u : word * 4u;
        // Model II: the lane's share of each coin counter (word * gamma).
        uint64_t coin_lane[WL];
#pragma unroll
        for (int i = 0; i < WL; ++i)
            coin_lane[i] = MODEL == 2 ? (uint64_t)(word + i) * SPLITMIX64_GAMMA : 0;
        // Klein bottle: offset of the lane's words in a mirrored row (the
        // WL words ending at column words-1-word, loaded in natural order).
        const uint32_t word_m = (uint32_t)(a.words - WL) - word;
        const uint32_t voff_m = IO == IO_U8 ? word_m * 32u : word_m * 4u;
        // Input row s of the strip lies across the glued top/bottom edge.
        const int lattice_rows = a.rows;
        const bool edge_strip = row_a < K || row_a + h + K > lattice_rows;
        auto mirrored = [row_a, lattice_rows](int s) {
            if constexpr (TOPO == TOPO_KLEIN) {
                const int g = row_a - K + s;
                return g < 0 || g >= lattice_rows;
            } else {
                return false;
            }
        };

        // Byte offset of input row t (lattice row row_a - K + t, periodic).
        // `ld_off` runs D rows ahead of the pipeline; `st_off` is the next
        // output row.  Each advance moves one row: one conditional wrap.
        uint32_t ld_off = (uint32_t)((row_a - K + a.rows) % a.rows) * row_bytes;
        uint32_t st_off = (uint32_t)row_a * row_bytes;
        // The offsets are wave-uniform; readfirstlane keeps them visibly so
        // (the compiler may otherwise compute the wrap with vector min/sub
        // and then wrap every buffer load in a loop over distinct offsets).
        auto advance = [&](uint32_t o) {
            const uint32_t x = o + row_bytes;
            return (uint32_t)__builtin_amdgcn_readfirstlane(
                (int)(x >= plane_bytes ? x - plane_bytes : x));
        };
        uint32_t ring[D][NW];
        // Row layout in the ring: u8: 8 dwords (32 cells) per word; bp: the
        // WL LR words, then the WL TB words.
        // Captures by value: a select between captured references would be
        // lowered to an indexed private (scratch) array.
        auto issue = [src, voff, voff_m, plane_bytes](uint32_t (&dstw)[NW], uint32_t off_,
                                                     bool mir) {
            const uint32_t off = (uint32_t)__builtin_amdgcn_readfirstlane((int)off_);
            const uint32_t vo = (TOPO == TOPO_KLEIN && mir) ? voff_m : voff;
            if constexpr (IO == IO_U8) {
#pragma unroll
                for (int j = 0; j < 2 * WL; ++j) {
                    const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(src, vo + 16 * j,
                                                                          off, 0);
                    dstw[4 * j + 0] = u.x; dstw[4 * j + 1] = u.y;
                    dstw[4 * j + 2] = u.z; dstw[4 * j + 3] = u.w;
                }
            } else if constexpr (WL == 1) {
                dstw[0] = __builtin_amdgcn_raw_buffer_load_b32(src, vo, off, 0);
                dstw[1] = __builtin_amdgcn_raw_buffer_load_b32(src, vo, off + plane_bytes,
                                                               0);
            } else {
                const u32x2 l = __builtin_amdgcn_raw_buffer_load_b64(src, vo, off, 0);
                const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(src, vo, off + plane_bytes,
                                                                     0);
                dstw[0] = l.x; dstw[1] = l.y; dstw[2] = t.x; dstw[3] = t.y;
            }
        };
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (d < total_in) {
                issue(ring[d], ld_off, mirrored(d));
                ld_off = advance(ld_off);
            }
        }

        // Skewed pipeline: in iteration t, level k works on the row level
        // k-1 produced in iteration t-1 (lattice row row_a - K + t - 2k after
        // k steps) and emits it one row higher after k+1 steps.  Levels are
        // visited from K-1 down to 0 so each reads its input before level
        // k-1 overwrites it; within one iteration the levels are independent.
        Level<WL> lv[K];
        uint32_t bl[K][WL], bt[K][WL];   // bl/bt[k]: last output of level k
        uint32_t acc[K][4];
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = 0; i < WL; ++i)
                lv[k].L[i] = lv[k].T[i] = lv[k].mvp[i] = bl[k][i] = bt[k][i] = 0;
            acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0;
        }

        // EDGE: this strip's halo may cross the Klein edge (only the first
        // and last strips of a Klein lattice); every other strip runs the
        // torus code (one-word rows; see below).
        auto body = [&](int t0, auto full_tag, auto edge_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            constexpr bool EDGE = TOPO == TOPO_KLEIN && decltype(edge_tag)::value;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int t = t0 + d;
                if (!FULL && t >= total_it)
                    break;
                uint32_t L0[WL], T0[WL];
#pragma unroll
                for (int i = 0; i < WL; ++i)
                    L0[i] = T0[i] = 0;
                if (FULL || t < total_in) {
#pragma unroll
                    for (int i = 0; i < WL; ++i) {
                        if constexpr (IO == IO_U8) {
                            bytes_to_planes(&ring[d][8 * i], L0[i], T0[i]);
                            asm("" : "+v"(L0[i]), "+v"(T0[i]));
                        } else {
                            L0[i] = ring[d][i];
                            T0[i] = ring[d][WL + i];
                        }
                    }
                    // A row across the Klein edge was loaded from the mirror
                    // columns: reverse its words (and their order) into the
                    // strip's frame.  Never in the FULL body, whose input
                    // rows all lie inside the lattice's own rows.
                    if (EDGE && !FULL && mirrored(t)) {
                        uint32_t l[WL], tt[WL];
#pragma unroll
                        for (int i = 0; i < WL; ++i) {
                            l[i] = __builtin_bitreverse32(L0[WL - 1 - i]);
                            tt[i] = __builtin_bitreverse32(T0[WL - 1 - i]);
                        }
#pragma unroll
                        for (int i = 0; i < WL; ++i) {
                            L0[i] = l[i];
                            T0[i] = tt[i];
                        }
                    }
                    if (FULL || t + D < total_in) {
                        issue(ring[d], ld_off, EDGE && (FULL || edge_strip) && mirrored(t + D));
                        ld_off = advance(ld_off);
                    }
                }
#pragma unroll
                for (int k = K - 1; k >= 0; --k) {
                    // Level k only matters for 3k <= t <= h + 2K - 1 + k:
                    // it first needs two rows of state before emitting
                    // its first exact row (k + 1 after k + 1 steps), and
                    // its last exact row is h + 2K - 2 - k.  Outside that
                    // window (prologue and drain only) the uniform branch
                    // skips it; its stale outputs are never read because
                    // level k + 1 is then idle too.
                    if (!FULL && (t < 3 * k || t > h + 2 * K - 1 + k))
                        continue;
                    // The row this level takes in is input row t - 2k; in the
                    // FULL body it never lies across the Klein edge.
                    LevelOut<WL> o;
                    if constexpr (MODEL == 2) {
                        // coins of input row t - 2k at global step step0 + k
                        const int g0 = row_a - K + (t - 2 * k);
                        const int g = g0 < 0 ? g0 + a.rows : g0 >= a.rows ? g0 - a.rows : g0;
                        const uint64_t base =
                            (a.lat[li].step0 + (uint64_t)k) * (uint64_t)a.rows * (uint64_t)a.words +
                            (uint64_t)g * (uint64_t)a.words;
                        const uint64_t row_z =
                            a.lat[li].coin_seed + (base + 1ull) * SPLITMIX64_GAMMA;
                        uint32_t coin[WL];
#pragma unroll
                        for (int i = 0; i < WL; ++i)
                            coin[i] = splitmix64_mix_lo(row_z + coin_lane[i]);
                        o = level_push_model2<WL, WRAP>(lv[k], k ? bl[k - 1] : L0,
                                                         k ? bt[k - 1] : T0, coin);
                    } else if constexpr (MODEL == 3) {
                        o = level_push_model3<WL, WRAP>(lv[k], k ? bl[k - 1] : L0,
                                                         k ? bt[k - 1] : T0);
                    } else {
                        const bool mir = EDGE && !FULL && mirrored(t - 2 * k);
                        o = level_push<WL, WRAP>(lv[k], k ? bl[k - 1] : L0, k ? bt[k - 1] : T0,
                                                 mir);
                    }
                    const int rh = t - 2 * k - K;   // H row relative to row_a
#pragma unroll
                    for (int i = 0; i < WL; ++i) {
                        if (FULL || (rh >= 0 && rh < h)) {
                            acc[k][0] += __builtin_popcount(o.l_h[i]);
                            acc[k][1] += __builtin_popcount(o.mv_h[i]);
                        }
                        if (FULL || (rh >= 1 && rh <= h)) {
                            acc[k][2] += __builtin_popcount(o.T[i]);
                            acc[k][3] += __builtin_popcount(o.mv_v[i]);
                        }
                    }
                    // Opaque after each row: stops the adds from being
                    // reassociated into one tree per macro-iteration, which
                    // would keep every popcount of it live.
                    asm("" : "+v"(acc[k][0]), "+v"(acc[k][1]), "+v"(acc[k][2]),
                        "+v"(acc[k][3]));
#pragma unroll
                    for (int i = 0; i < WL; ++i) {
                        bl[k][i] = o.L[i];
                        bt[k][i] = o.T[i];
                    }
                }
                if (FULL || (t >= 3 * K - 1 && t < 3 * K - 1 + h)) {
                    const uint32_t so = (uint32_t)__builtin_amdgcn_readfirstlane((int)st_off);
                    if (lane_ok) {
                        if constexpr (IO == IO_U8) {
#pragma unroll
                            for (int i = 0; i < WL; ++i) {
                                uint32_t b[8];
                                planes_to_bytes(bl[K - 1][i], bt[K - 1][i], b);
                                __builtin_amdgcn_raw_buffer_store_b128(
                                    (u32x4){b[0], b[1], b[2], b[3]}, dst, voff + 32 * i, so,
                                    0);
                                __builtin_amdgcn_raw_buffer_store_b128(
                                    (u32x4){b[4], b[5], b[6], b[7]}, dst, voff + 32 * i + 16,
                                    so, 0);
                            }
                        } else if constexpr (WL == 1) {
                            __builtin_amdgcn_raw_buffer_store_b32(bl[K - 1][0], dst, voff, so,
                                                                  0);
                            __builtin_amdgcn_raw_buffer_store_b32(bt[K - 1][0], dst, voff,
                                                                  so + plane_bytes,
                                                                  0);
                        } else {
                            __builtin_amdgcn_raw_buffer_store_b64(
                                (u32x2){bl[K - 1][0], bl[K - 1][1]}, dst, voff, so,
                                0);
                            __builtin_amdgcn_raw_buffer_store_b64(
                                (u32x2){bt[K - 1][0], bt[K - 1][1]}, dst, voff,
                                so + plane_bytes, 0);
                        }
                    }
                    st_off += row_bytes;
                }
                // Keep each iteration's work together: bounds register use
                // (iterations would otherwise be interleaved) without losing
                // the parallelism between the levels of one iteration.
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        for (int t0 = 0; t0 < total_it; t0 += D) {
            // Full: every level counts, every iteration stores and the
            // prefetch stays inside the strip for all D iterations.
            if (t0 >= 3 * K - 1 && t0 + D <= h + K && t0 + 2 * D <= total_in)
                // (its only edge work is choosing the mirror offset of a
                // prefetched bottom halo row: one select per load)
                body(t0, std::true_type{}, std::bool_constant<TOPO == TOPO_KLEIN>{});
            else
            // (two-word rows keep one body: a second copy would push them
            // past 256 VGPRs)
            if (TOPO == TOPO_KLEIN && (WL > 1 || edge_strip))
                body(t0, std::false_type{}, std::true_type{});
            else
                body(t0, std::false_type{}, std::false_type{});
        }

        // Fold this item's counts into the wave totals (halo and duplicate
        // lanes contribute nothing).
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                wtot[k][q] += wave_total(lane_ok ? acc[k][q] : 0u);
    }

    // Counts: wave -> block (LDS, per lattice) -> one of 8 device-wide
    // stripes of each lattice (block b adds to stripe b % 8) -> the last
    // block to finish sums the stripes, writes the ring slots and clears the
    // scratch for the next launch.  The launch's ticket lives in the first
    // lattice's scratch.
    if (a.any_rec == 0)
        return;
    flush();
    __syncthreads();
    const int n_counts = a.n_lat * K * 4;
    for (int i = threadIdx.x; i < n_counts; i += blockDim.x) {
        const int l = i / (K * 4), j = i - l * (K * 4);
        if (red[l][j])
            __hip_atomic_fetch_add(&a.lat[l].scratch->acc[blockIdx.x % ACC_STRIPES][0][0] + j,
                                   red[l][j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // Every thread's stripe additions must be complete before the ticket
    // says this block is done; the last block reads the stripes only with
    // atomics, issued after it has seen the final ticket.
    wait_vector_memory();
    __syncthreads();
    PassScratch *const ticket_owner = a.lat[0].scratch;
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(&ticket_owner->ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        is_last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!is_last)
        return;
    for (int i = threadIdx.x; i < n_counts; i += blockDim.x) {
        const int l = i / (K * 4), j = i - l * (K * 4);
        const int k = j >> 2, q = j & 3;
        uint32_t sum = 0;
#pragma unroll
        for (int st = 0; st < ACC_STRIPES; ++st)
            sum += __hip_atomic_exchange(&a.lat[l].scratch->acc[st][0][0] + j, 0u,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((a.lat[l].rec_mask >> k) & 1u)
            a.lat[l].stats[(size_t)a.lat[l].slot[k] * 4 + q] = sum;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(&ticket_owner->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fills tab[k] (k = KLO..KHI) with pass_kernel<IO, k, ROW, TOPO, MODEL>.
template <int IO, int ROW, int TOPO, int MODEL, int KLO, int... Ks>
inline void fill_pass_table(PassFn *tab, std::integer_sequence<int, Ks...>)
{
    ((tab[KLO + Ks] = pass_kernel<IO, KLO + Ks, ROW, TOPO, MODEL>), ...);
}

// Each table function fills tab[k] for its range of K; tab has MAX_K + 1
// entries.  One translation unit per (layout, column mode / K range,
// topology): bml_pass_inst.hip compiled once per variant, so the variants
// build in parallel.  Ranges: lo = tile mode K 1..4, hi = tile mode K 5..8,
// row1 / row2 = row mode with one / two words per lane, K 1..8.
#define BML_PASS_TABLE_DECL(io, range, topo) void pass_table_##io##_##range##_##topo(PassFn *tab);
#define BML_PASS_TABLES(X, topo)                                                        \
    X(u8, lo, topo) X(u8, hi, topo) X(u8, row1, topo) X(u8, row2, topo) X(bp, lo, topo) \
    X(bp, hi, topo) X(bp, row1, topo) X(bp, row2, topo)
BML_PASS_TABLES(BML_PASS_TABLE_DECL, torus)
BML_PASS_TABLES(BML_PASS_TABLE_DECL, klein)
BML_PASS_TABLES(BML_PASS_TABLE_DECL, model2)   // Model II, torus
BML_PASS_TABLES(BML_PASS_TABLE_DECL, model3)   // Model III, torus

} // namespace bml
