// bml_block.hpp -- register-resident tile kernel for single lattices
// (gfx950): up to 32 steps per HBM pass.
//
// The lattice is cut into tiles of 32 words (1024 cells; 16 or 8 words for
// lattices too small to give every CU work) by up to 512 - 2K rows.  A
// 4-wave workgroup holds one tile with one halo word on each side and K
// halo rows above and below, two rows per lane (34 LR and 34 TB words per
// row for the widest tiles), loads it once, advances it K steps in
// registers and stores the tile's own words and rows.  Three such
// workgroups fit a CU (at most 168 VGPRs per lane, 41 KB of LDS each), so
// each SIMD interleaves three waves.  The rule of Marzolla,
// arXiv:1804.07981, Sec. 2 decides every move from the cell's neighbour in the direction of
// travel, so what the held block does not know (the cells beyond its halo)
// travels at most one cell right and one row down per step, and its error
// reaches at most K cells into the 32-cell halo words and K rows into the
// halo rows: after K <= 32 steps the tile's own cells are exact.  The
// horizontal phase runs inside the lane over the 34 words with open ends (a
// car on the last held cell does not move, none arrives into the first);
// the vertical phase passes TB cars from a lane's upper row to its lower
// row in registers, between lanes by DPP wave shifts and between the wave
// fronts through LDS with one barrier per step, as in bml_resident.hpp.
// Both phases read only the state before the phase (synchronous update,
// Sec. 3).  Counts of the tile's own cells (LR cars after the horizontal
// phase, LR movers, TB cars after the vertical phase, TB movers) are summed
// per step and written per tile; block_sum_kernel adds the tiles of each
// lattice and records the steps the caller keeps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "bml_pass.hpp"
#include "bml_resident.hpp"
#include "bml_tile.hpp"

namespace bml {

constexpr int BLK_WORDS = 32;                 // own words per row of the widest tiles
constexpr int BLK_WAVES = 4;                  // one wave per SIMD, three workgroups per CU
constexpr int BLK_ROWS = BLK_WAVES * 128;     // rows a workgroup holds (two per lane)
constexpr int BLK_MAX_K = 32;                 // steps per launch (the halo word's 32 cells)

struct BlockLattice {
    const void *src;
    void *dst;
    uint32_t *partial;       // [tile][step of the launch][4] counts of the tile's cells
};

// A launch advances n_lat lattices of the same size and layout by n_steps
// <= halo steps; workgroup b works on tile b % tiles of lattice b / tiles,
// tiles numbered slab-major (slab = b / tiles_x, column block = b % tiles_x).
struct BlockArgs {
    BlockLattice lat[MAX_GROUP];
    int32_t n_lat;
    int32_t rows;            // lattice rows (a multiple of 32)
    int32_t words;           // 32-cell words per row (a multiple of 32)
    int32_t tiles_x;         // words / 32
    int32_t slabs;           // row slabs
    int32_t halo;            // halo rows (>= n_steps, even)
    int32_t n_steps;
};

// Loads and stores go through a per-wave staging area so that each memory
// instruction covers whole 128-byte lines of a few rows (lanes along a row)
// while the step loop keeps two rows per lane: the tile's 32 own words are
// moved in four chunks of 8 words x 128 rows.  A staged row is 9 words
// (8 + 1 pad) and a lane's upper and lower rows sit in separate halves, so
// a lane reading its own rows hits bank 9 * lane + j: no conflicts.
constexpr int BLK_CHUNK = 8;                  // words per staged chunk
constexpr int BLK_BATCH = 8;                  // staged rows whose loads are in flight per lane
constexpr int BLK_SROW = BLK_CHUNK + 1;       // padded staged row

// Exchange rows padded to 36 words: read and written 4 words (16 bytes) at a
// time.
constexpr int BLK_XW = 36;
constexpr int BLK_G = 4;                      // words per scheduling group of the step

struct BlockShared {
    uint32_t x[2][BLK_WAVES][2][BLK_XW];     // as ResidentShared::x (16-byte aligned: first member)
    uint32_t none[BLK_XW];                    // zero: no neighbour beyond the halo rows
    // Per wave and step: LR cars that entered the tile's own cells minus
    // those that left them, LR movers, the same difference for TB cars, TB
    // movers.
    uint32_t cnt[BLK_MAX_K][BLK_WAVES][4];
    uint32_t cars[2][BLK_WAVES][2];           // [after load, after the steps][wave][LR, TB]
    uint32_t stage[BLK_WAVES][2][2 * 64 * BLK_SROW];   // [wave][plane][row half][lane, word]
};

__device__ __forceinline__ int stage_index(int r, int j)
{
    return (r & 1) * 64 * BLK_SROW + (r >> 1) * BLK_SROW + j;
}

// 16 byte cells (d.x = cells 0..3, byte k of a dword = cell 4q + k) to one
// word holding their LR bits in bits 0..15 and TB bits in bits 16..31.  The
// gather leaves the LR bit of cell 4q + k at 8k + q and its TB bit at
// 8k + 4 + q; index_rotl2 moves position [k t q] to [t q k].
__device__ __forceinline__ uint32_t bytes16_to_halves(u32x4 d)
{
    uint32_t x = (d.x & 0x01010101u) | ((d.x & 0x02020202u) << 3);
    x |= ((d.y & 0x01010101u) << 1) | ((d.y & 0x02020202u) << 4);
    x |= ((d.z & 0x01010101u) << 2) | ((d.z & 0x02020202u) << 5);
    x |= ((d.w & 0x01010101u) << 3) | ((d.w & 0x02020202u) << 6);
    return index_rotl2(x);
}

// The inverse: the delta swaps of index_rotl2 in reverse order (each is its
// own inverse), then the bits back to bytes.
__device__ __forceinline__ u32x4 halves_to_bytes16(uint32_t x)
{
    x = delta_swap(x, 14, 0x0000ccccu);
    x = delta_swap(x, 7, 0x00aa00aau);
    x = delta_swap(x, 2, 0x0c0c0c0cu);
    x = delta_swap(x, 1, 0x22222222u);
    return (u32x4){(x & 0x01010101u) | ((x >> 3) & 0x02020202u),
                   ((x >> 1) & 0x01010101u) | ((x >> 4) & 0x02020202u),
                   ((x >> 2) & 0x01010101u) | ((x >> 5) & 0x02020202u),
                   ((x >> 3) & 0x01010101u) | ((x >> 6) & 0x02020202u)};
}

// Every lane's LDS accesses before this point are complete and visible to
// the wave's other lanes after it.
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// MODEL 1: the two-phase rule of Sec. 2 (horizontal phase, then the
// vertical phase on the state it leaves).  MODEL 3: Model III, one phase in
// which every car looks at the state before the step (a car moves when its
// target cell held no car; an empty cell wanted by an LR and a TB car takes
// both).
// TW: own words per tile row (32, 16 or 8); narrower tiles make more
// workgroups for lattices too small to fill the GPU with 1024-column tiles.
// KLEIN: the Klein bottle (top and bottom edges glued with a reversal;
// the model of Sec. 2 only): a held row beyond the lattice's first or last
// row is the row across the glued edge, held mirrored (tile column j holds
// the lattice cell vertically next to it, cols - 1 - j), so its LR cars move
// towards lower tile columns.  Only tiles of the first and last slab hold
// such rows, and only they run the mirrored horizontal phase.
template <int IO, int MODEL, int TW, bool KLEIN>
__global__ __launch_bounds__(64 * BLK_WAVES, 3) void block_kernel(BlockArgs a)
{
    static_assert(!KLEIN || MODEL == 1, "Klein bottle: the model of Sec. 2 only");
    static_assert(TW % BLK_CHUNK == 0 && TW <= BLK_WORDS, "tile width");
    constexpr int W = TW + 2;                    // words held per row
    constexpr int XW = (W + 3) / 4 * 4;          // exchange words, whole 16-byte groups
    __shared__ BlockShared sh;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tiles = a.tiles_x * a.slabs;
    // Workgroups go to the eight XCDs in turn (workgroup b to XCD b % 8);
    // each XCD takes a contiguous run of tiles, so that the neighbours whose
    // boundary lines a tile reads as halo (the tiles left and right, the
    // slabs above and below) mostly run on the same XCD and share its L2.
    const int nb = (int)gridDim.x, xcd = (int)blockIdx.x & 7;
    int j = (int)blockIdx.x >> 3;
    // Klein bottle: the tiles of the first and last slab do more work per
    // step; the last XCD takes its run backwards, so that they start in the
    // first round instead of finishing the launch.
    if constexpr (KLEIN)
        if (xcd == 7)
            j = (nb >> 3) - 1 - j;   // XCD 7 runs exactly nb / 8 workgroups
    const int t = xcd * (nb >> 3) + min(xcd, nb & 7) + j;
    const int li = t / tiles;
    const int local = t - li * tiles;
    const int slab = local / a.tiles_x;
    const int tx = local - slab * a.tiles_x;
    // Slabs cut at even rows, as equal as possible (at most
    // BLK_ROWS - 2 * halo rows each).
    const int pairs = a.rows / 2;
    const int r0 = pairs * slab / a.slabs * 2;
    const int R = pairs * (slab + 1) / a.slabs * 2 - r0;
    const int H = a.halo;
    const int held = R + 2 * H;
    const int waves = (held + 127) / 128;
    const bool wave_on = wave < waves;
    const int row = wave * 128 + 2 * lane;           // the lane's upper row in the held block
    const bool row_ok = wave_on && row < held;
    const bool counted = row_ok && row >= H && row < H + R;   // H, R even: both rows or none
    const int lanes = wave_on ? min(64, (held - wave * 128) / 2) : 64;
    const int last_lane = lanes - 1;
    const int wdown = wave + 1 < waves ? wave + 1 : -1;
    const int wup = wave > 0 ? wave - 1 : -1;
    const int n_steps = a.n_steps;
    const int N = a.rows;
    const int words = a.words;
    const uint32_t row_bytes = IO == IO_U8 ? (uint32_t)words * 32u : (uint32_t)words * 4u;
    const uint32_t plane_bytes = row_bytes * (uint32_t)N;
    const uint32_t state_bytes = IO == IO_U8 ? plane_bytes : 2u * plane_bytes;
    const __amdgpu_buffer_rsrc_t src = make_rsrc(a.lat[li].src, state_bytes);
    const __amdgpu_buffer_rsrc_t dst = make_rsrc(a.lat[li].dst, state_bytes);

    // Lattice rows of the lane (periodic).
    const int g0 = row_ok ? (r0 - H + row + 2 * N) % N : 0;
    const int g1 = g0 + 1 == N ? 0 : g0 + 1;
    const int w0 = tx * TW;
    const int wrow0 = wave * 128;                           // the wave's first held row
    const int wrows = wave_on ? min(128, held - wrow0) : 0; // rows the wave holds
    // Lattice row of held row wrow0 + q (0 <= q < 8): the staged loops step
    // it by 4 or 8 rows (N >= 32).
    const int gbase = __builtin_amdgcn_readfirstlane((r0 - H + wrow0 + 2 * N) % N);
    // Klein bottle: the block holds rows across the glued edge (edge), and
    // which of the lane's two rows are such rows (held mirrored).
    const int ubase = r0 - H + wrow0;            // unwrapped lattice row of held row wrow0
    const bool edge = KLEIN && (r0 - H < 0 || r0 + R + H > N);
    // the wave holds mirrored rows (uniform across the wave)
    const bool wave_mir = edge && wave_on && (ubase < 0 || ubase + wrows > N);
    const bool mir0 = edge && (r0 - H + row < 0 || r0 - H + row >= N);
    const bool mir1 = edge && (r0 - H + row + 1 < 0 || r0 - H + row + 1 >= N);
    uint32_t *stL = sh.stage[wave][0];
    uint32_t *stT = sh.stage[wave][1];
    uint32_t L0[W], T0[W], L1[W], T1[W];

    // Halo word h of a row (h = 0: held word 0, lattice word w0 - 1; h = 1:
    // held word W - 1, lattice word w0 + 32; periodic), each lane its own
    // rows.
    auto load_halo = [&](int h, int g, bool mir, uint32_t (&Lr)[W], uint32_t (&Tr)[W]) {
        const uint32_t ro = (uint32_t)g * row_bytes;
        const int i = h ? W - 1 : 0;
        int w = h ? (w0 + TW == words ? 0 : w0 + TW) : (w0 == 0 ? words - 1 : w0 - 1);
        if (KLEIN && mir)
            w = words - 1 - w;                   // the mirror word, bits reversed below
        uint32_t l, t;
        if constexpr (IO == IO_U8) {
            const u32x4 u0 = __builtin_amdgcn_raw_buffer_load_b128(src, ro + (uint32_t)w * 32u,
                                                                   0, 0);
            const u32x4 u1 = __builtin_amdgcn_raw_buffer_load_b128(
                src, ro + (uint32_t)w * 32u + 16u, 0, 0);
            const uint32_t dw[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
            bytes_to_planes(dw, l, t);
        } else {
            l = __builtin_amdgcn_raw_buffer_load_b32(src, ro + (uint32_t)w * 4u, 0, 0);
            t = __builtin_amdgcn_raw_buffer_load_b32(src, ro + plane_bytes + (uint32_t)w * 4u, 0,
                                                     0);
        }
        if (KLEIN && mir) {
            l = __builtin_bitreverse32(l);
            t = __builtin_bitreverse32(t);
        }
        Lr[i] = l;
        Tr[i] = t;
    };

    // Chunk c of the tile's own words (held words 1 + 8c .. 8 + 8c) of the
    // wave's rows into the staging area: uint8, 16 lanes per row (16 cells,
    // half a word, each), four rows per load; bitplanes, 8 lanes per row and
    // plane, eight rows per load.  Rows beyond the held block stage zeros.
    auto stage_in = [&](int c) {
        if constexpr (IO == IO_U8) {
            uint16_t *sL = reinterpret_cast<uint16_t *>(stL);
            uint16_t *sT = reinterpret_cast<uint16_t *>(stT);
            const int q = lane >> 4, w = (lane & 15) >> 1, hf = lane & 1;
            const uint32_t co = (uint32_t)(w0 + BLK_CHUNK * c + w) * 32u + (uint32_t)hf * 16u;
            // a mirrored row: the other half of the mirror word, cells reversed
            const uint32_t co_m =
                (uint32_t)(words - 1 - (w0 + BLK_CHUNK * c + w)) * 32u + (uint32_t)(1 - hf) * 16u;
            int g = gbase + q;
            g = g >= N ? g - N : g;
            // Batches of BLK_BATCH loads, all issued before the first is
            // used: a batch's registers fit beside the state of the chunks
            // already held (without explicit batches the compiler waited for
            // each load of the last chunks before issuing the next).
#pragma unroll 1
            for (int it0 = 0; it0 < 32; it0 += BLK_BATCH) {
                u32x4 v[BLK_BATCH];
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    const int r = 4 * (it0 + k) + q;
                    const bool mir = edge && (ubase + r < 0 || ubase + r >= N);
                    // Unconditional loads: g is always a lattice row.
                    v[k] = __builtin_amdgcn_raw_buffer_load_b128(
                        src, (uint32_t)g * row_bytes + (KLEIN && mir ? co_m : co), 0, 0);
                    g += 4;
                    g = g >= N ? g - N : g;
                }
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    const int r = 4 * (it0 + k) + q;
                    const bool mir = edge && (ubase + r < 0 || ubase + r >= N);
                    uint32_t x = bytes16_to_halves(v[k]);
                    if (KLEIN && mir) {              // both halves' cells reversed
                        x = __builtin_bitreverse32(x);
                        x = __builtin_amdgcn_alignbit(x, x, 16);
                    }
                    x = r < wrows ? x : 0u;
                    const int si = 2 * stage_index(r, w) + hf;
                    sL[si] = (uint16_t)x;
                    sT[si] = (uint16_t)(x >> 16);
                }
            }
        } else {
            const int q = lane >> 3, w = lane & 7;
            const uint32_t co = (uint32_t)(w0 + BLK_CHUNK * c + w) * 4u;
            const uint32_t co_m = (uint32_t)(words - 1 - (w0 + BLK_CHUNK * c + w)) * 4u;
            int g = gbase + q;
            g = g >= N ? g - N : g;
#pragma unroll 1
            for (int it0 = 0; it0 < 16; it0 += BLK_BATCH) {
                uint32_t l[BLK_BATCH], t[BLK_BATCH];
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    const int r = 8 * (it0 + k) + q;
                    const bool mir = edge && (ubase + r < 0 || ubase + r >= N);
                    const uint32_t o = (uint32_t)g * row_bytes + (KLEIN && mir ? co_m : co);
                    l[k] = __builtin_amdgcn_raw_buffer_load_b32(src, o, 0, 0);
                    t[k] = __builtin_amdgcn_raw_buffer_load_b32(src, o + plane_bytes, 0, 0);
                    g += 8;
                    g = g >= N ? g - N : g;
                }
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    const int r = 8 * (it0 + k) + q;
                    const bool mir = edge && (ubase + r < 0 || ubase + r >= N);
                    if (KLEIN && mir) {
                        l[k] = __builtin_bitreverse32(l[k]);
                        t[k] = __builtin_bitreverse32(t[k]);
                    }
                    stL[stage_index(r, w)] = r < wrows ? l[k] : 0u;
                    stT[stage_index(r, w)] = r < wrows ? t[k] : 0u;
                }
            }
        }
    };
    // The reverse for the counted rows: each lane stages its own rows' words
    // of chunk c, then the wave stores them along the rows.
    auto stage_out = [&](int c) {
        if constexpr (IO == IO_U8) {
            const uint16_t *sL = reinterpret_cast<const uint16_t *>(stL);
            const uint16_t *sT = reinterpret_cast<const uint16_t *>(stT);
            const int q = lane >> 4, w = (lane & 15) >> 1, hf = lane & 1;
            const uint32_t co = (uint32_t)(w0 + BLK_CHUNK * c + w) * 32u + (uint32_t)hf * 16u;
            int g = gbase + q;
            g = g >= N ? g - N : g;
            // Batches: the staged halves of BLK_BATCH rows are read before
            // the first is converted, so that one LDS latency covers them.
#pragma unroll 1
            for (int it0 = 0; it0 < 32; it0 += BLK_BATCH) {
                uint32_t x[BLK_BATCH];
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    const int si = 2 * stage_index(4 * (it0 + k) + q, w) + hf;
                    x[k] = (uint32_t)sL[si] | ((uint32_t)sT[si] << 16);
                }
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    const int hr = wrow0 + 4 * (it0 + k) + q;
                    if (hr >= H && hr < H + R)
                        __builtin_amdgcn_raw_buffer_store_b128(halves_to_bytes16(x[k]), dst,
                                                               (uint32_t)g * row_bytes + co, 0, 0);
                    g += 4;
                    g = g >= N ? g - N : g;
                }
            }
        } else {
            const int q = lane >> 3, w = lane & 7;
            const uint32_t co = (uint32_t)(w0 + BLK_CHUNK * c + w) * 4u;
            int g = gbase + q;
            g = g >= N ? g - N : g;
#pragma unroll 1
            for (int it0 = 0; it0 < 16; it0 += BLK_BATCH) {
                uint32_t l[BLK_BATCH], t[BLK_BATCH];
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    l[k] = stL[stage_index(8 * (it0 + k) + q, w)];
                    t[k] = stT[stage_index(8 * (it0 + k) + q, w)];
                }
#pragma unroll
                for (int k = 0; k < BLK_BATCH; ++k) {
                    const int hr = wrow0 + 8 * (it0 + k) + q;
                    if (hr >= H && hr < H + R) {
                        const uint32_t o = (uint32_t)g * row_bytes + co;
                        __builtin_amdgcn_raw_buffer_store_b32(l[k], dst, o, 0, 0);
                        __builtin_amdgcn_raw_buffer_store_b32(t[k], dst, o + plane_bytes, 0, 0);
                    }
                    g += 8;
                    g = g >= N ? g - N : g;
                }
            }
        }
    };

#pragma unroll
    for (int i = 0; i < W; ++i)
        L0[i] = T0[i] = L1[i] = T1[i] = 0;
    // The right halo word is the first word the tile to the right loads,
    // the left one the last word the tile to the left loads: loaded at the
    // same times, their lines are mostly still in the XCD's L2.
    if (row_ok) {
        load_halo(1, g0, mir0, L0, T0);
        load_halo(1, g1, mir1, L1, T1);
    }
    if (wave_on) {
#pragma unroll
        for (int c = 0; c < TW / BLK_CHUNK; ++c) {
            stage_in(c);
            wave_sync_lds();
#pragma unroll
            for (int j = 0; j < BLK_CHUNK; ++j) {
                const int i = 1 + BLK_CHUNK * c + j;
                L0[i] = stL[stage_index(2 * lane, j)];
                T0[i] = stT[stage_index(2 * lane, j)];
                L1[i] = stL[stage_index(2 * lane + 1, j)];
                T1[i] = stT[stage_index(2 * lane + 1, j)];
            }
            wave_sync_lds();
        }
    }
    if (row_ok) {
        load_halo(0, g0, mir0, L0, T0);
        load_halo(0, g1, mir1, L1, T1);
    }
    // Cars on the tile's own cells, per wave: counted directly after the
    // load and after the last step; the per-step counts in between follow
    // from what crosses the tile's edges, and must end at the second count.
    auto count_cars = [&](int when) {
        uint32_t nl = 0, nt = 0;
#pragma unroll
        for (int i = 1; i < W - 1; ++i) {
            nl = __builtin_popcount(L0[i]) + nl;
            nl = __builtin_popcount(L1[i]) + nl;
            nt = __builtin_popcount(T0[i]) + nt;
            nt = __builtin_popcount(T1[i]) + nt;
        }
        const uint32_t cl = wave_total(counted ? nl : 0u);
        const uint32_t ct = wave_total(counted ? nt : 0u);
        if (lane == 0) {
            sh.cars[when][wave][0] = cl;
            sh.cars[when][wave][1] = ct;
        }
    };
    count_cars(0);
    // The lanes whose lower row is the last held row above the tile's own
    // rows (its TB movers enter them) and the tile's last own row (its TB
    // movers leave them).
    const int in_row = H - 2, out_row = H + R - 2;
    const int w_in = in_row >> 7, l_in = (in_row & 127) >> 1;
    const int w_out = out_row >> 7, l_out = (out_row & 127) >> 1;
    if (threadIdx.x < BLK_XW)
        sh.none[threadIdx.x] = 0;

    // Horizontal phase of both rows with open ends: the cell beyond the last
    // held one counts as occupied, nothing arrives into the first.  Every
    // mover is decided before any word changes.  The words go in groups of
    // BLK_G, each stage of the rule applied to the group's words of both
    // rows before the next stage, so that a lone wave finds independent
    // instructions to issue back to back.  Returns the LR movers of the
    // tile's own words.  The emptiness the vertical phase needs is
    // recomputed there from the planes (no array of it stays live).
    // Klein bottle: a mirrored row reversed in place (word order and bit
    // order), so that its LR cars move towards higher columns; the
    // horizontal phase then runs unchanged on it (its open ends swap with
    // the row), and a second reversal restores the tile frame.  Lanes whose
    // rows are not mirrored keep them.
    auto reverse_mirrored = [&]() {
#pragma unroll
        for (int i = 0; i < W / 2; ++i) {
            const int k = W - 1 - i;
            uint32_t a, b;
            a = L0[i]; b = L0[k];
            L0[i] = mir0 ? __builtin_bitreverse32(b) : a;
            L0[k] = mir0 ? __builtin_bitreverse32(a) : b;
            a = T0[i]; b = T0[k];
            T0[i] = mir0 ? __builtin_bitreverse32(b) : a;
            T0[k] = mir0 ? __builtin_bitreverse32(a) : b;
            a = L1[i]; b = L1[k];
            L1[i] = mir1 ? __builtin_bitreverse32(b) : a;
            L1[k] = mir1 ? __builtin_bitreverse32(a) : b;
            a = T1[i]; b = T1[k];
            T1[i] = mir1 ? __builtin_bitreverse32(b) : a;
            T1[k] = mir1 ? __builtin_bitreverse32(a) : b;
        }
    };

    auto hphase = [&](uint32_t &flux) {
        // one accumulator per popcount stream: each popcount adds into its
        // own (v_bcnt_u32_b32 with an addend), no separate adds
        uint32_t c0 = 0, c1 = 0;
        uint32_t p0 = 0, p1 = 0, o0 = L0[0] | T0[0], o1 = L1[0] | T1[0];
#pragma unroll
        for (int g = 0; g < W; g += BLK_G) {
            uint32_t on0[BLK_G], on1[BLK_G], m0[BLK_G], m1[BLK_G];
#pragma unroll
            for (int j = 0; j < BLK_G; ++j) {       // occupancy of the next word
                const int i = g + j;
                if (i < W) {
                    on0[j] = i + 1 < W ? (L0[i + 1] | T0[i + 1]) : 0xffffffffu;
                    on1[j] = i + 1 < W ? (L1[i + 1] | T1[i + 1]) : 0xffffffffu;
                }
            }
#pragma unroll
            for (int j = 0; j < BLK_G; ++j) {       // movers: the next cell is empty
                const int i = g + j;
                if (i < W) {
                    m0[j] = L0[i] & ~__builtin_amdgcn_alignbit(on0[j], j ? on0[j - 1] : o0, 1);
                    m1[j] = L1[i] & ~__builtin_amdgcn_alignbit(on1[j], j ? on1[j - 1] : o1, 1);
                }
            }
#pragma unroll
            for (int j = 0; j < BLK_G; ++j) {       // movers leave, arrivals land (disjoint)
                const int i = g + j;
                if (i < W) {
                    L0[i] = xor3(L0[i], m0[j],
                                 __builtin_amdgcn_alignbit(m0[j], j ? m0[j - 1] : p0, 31));
                    L1[i] = xor3(L1[i], m1[j],
                                 __builtin_amdgcn_alignbit(m1[j], j ? m1[j - 1] : p1, 31));
                }
            }
#pragma unroll
            for (int j = 0; j < BLK_G; ++j) {
                const int i = g + j;
                if (i >= 1 && i < W - 1) {
                    c0 = __builtin_popcount(m0[j]) + c0;
                    c1 = __builtin_popcount(m1[j]) + c1;
                    asm("" : "+v"(c0), "+v"(c1));
                }
                // cars entering the own words from the left halo word, and
                // leaving the last own word for the right one
                if (i == 0)
                    flux = (m0[j] >> 31) + (m1[j] >> 31);
                if (i == W - 2)
                    flux -= (m0[j] >> 31) + (m1[j] >> 31);
            }
            const int last = (W - g < BLK_G ? W - g : BLK_G) - 1;
            o0 = on0[last];
            o1 = on1[last];
            p0 = m0[last];
            p1 = m1[last];
            // Opaque new values (and counts): updated in place here, not
            // carried as pieces to the end of the step.
#pragma unroll
            for (int j = 0; j < BLK_G; ++j) {
                const int i = g + j;
                if (i < W)
                    asm("" : "+v"(L0[i]), "+v"(L1[i]));
            }
            asm("" : "+v"(c0), "+v"(c1), "+v"(flux));
            __builtin_amdgcn_sched_barrier(0);
        }
        return c0 + c1;
    };

    for (int s = 0; s < n_steps; ++s) {
        const int p = s & 1;
        uint32_t f_lr = 0, c_lr = 0, c_tb = 0, c_tb1 = 0;
        if (wave_on) {
            // Model III reads every neighbour before the step: the rows
            // exchanged below are then the state before the step, and its
            // LR moves are made in the vertical loop.
            if constexpr (MODEL == 1) {
                if constexpr (KLEIN) {
                    if (wave_mir)
                        reverse_mirrored();
                }
                c_lr = hphase(f_lr);
                if constexpr (KLEIN) {
                    if (wave_mir)
                        reverse_mirrored();
                }
            }
            if (lane == 0) {
#pragma unroll
                for (int i = 0; i < XW; i += 4)
                    *reinterpret_cast<u32x4 *>(&sh.x[p][wave][0][i]) =
                        (u32x4){~(L0[i] | T0[i]), i + 1 < W ? ~(L0[i + 1] | T0[i + 1]) : 0u,
                                i + 2 < W ? ~(L0[i + 2] | T0[i + 2]) : 0u,
                                i + 3 < W ? ~(L0[i + 3] | T0[i + 3]) : 0u};
            }
            if (lane == last_lane) {
#pragma unroll
                for (int i = 0; i < XW; i += 4)
                    *reinterpret_cast<u32x4 *>(&sh.x[p][wave][1][i]) =
                        (u32x4){T1[i], i + 1 < W ? T1[i + 1] : 0u, i + 2 < W ? T1[i + 2] : 0u,
                                i + 3 < W ? T1[i + 3] : 0u};
            }
        }
        __syncthreads();
        if (wave_on) {
            const uint32_t *xb = wdown >= 0 ? sh.x[p][wdown][0] : sh.none;
            const uint32_t *xa = wup >= 0 ? sh.x[p][wup][1] : sh.none;
            // The neighbour rows four words at a time, one group ahead of
            // their use, so that LDS latency hides behind the previous group.
            // Words per group: Model III keeps more values live per word
            // (its LR movers too), so its groups are half as wide.
            constexpr int VG = MODEL == 3 ? 2 : 4;
            typedef uint32_t xvec __attribute__((ext_vector_type(VG)));
            xvec nb = *reinterpret_cast<const xvec *>(xb);
            xvec na = *reinterpret_cast<const xvec *>(xa);
            // Model III: occupancy of the current word and LR movers of the
            // previous one, carried from group to group
            uint32_t o0 = L0[0] | T0[0], o1 = L1[0] | T1[0], q0 = 0, q1 = 0, c_l1 = 0;
#pragma unroll
            for (int g = 0; g < XW; g += VG) {
                const xvec cb = nb, ca = na;
                if (g + VG < XW) {
                    nb = *reinterpret_cast<const xvec *>(xb + g + VG);
                    na = *reinterpret_cast<const xvec *>(xa + g + VG);
                }
                uint32_t e0[VG], e1[VG], eb[VG], mv0[VG], mv1[VG], ar[VG], m0[VG], m1[VG];
                if constexpr (MODEL == 3) {
                    // LR movers from the state before the step: the next
                    // cell held no car (open right end: the cell beyond the
                    // last held word counts as occupied)
#pragma unroll
                    for (int j = 0; j < VG; ++j) {
                        const int i = g + j;
                        if (i < W) {
                            const uint32_t on0 = i + 1 < W ? (L0[i + 1] | T0[i + 1]) : 0xffffffffu;
                            const uint32_t on1 = i + 1 < W ? (L1[i + 1] | T1[i + 1]) : 0xffffffffu;
                            m0[j] = L0[i] & ~__builtin_amdgcn_alignbit(on0, o0, 1);
                            m1[j] = L1[i] & ~__builtin_amdgcn_alignbit(on1, o1, 1);
                            o0 = on0;
                            o1 = on1;
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < VG; ++j) {
                    const int i = g + j;
                    if (i < W) {
                        e0[j] = ~(L0[i] | T0[i]);
                        e1[j] = ~(L1[i] | T1[i]);
                    }
                }
#pragma unroll
                for (int j = 0; j < VG; ++j) {
                    const int i = g + j;
                    if (i < W) {
                        // The lane below; lane 63 keeps the first row of
                        // the wave below (or none).  In a short last wave
                        // the last held row sees an unused lane instead of
                        // none: that row is a halo row of the open lower
                        // end, whose error reaches the own rows only after
                        // more than H >= K steps, so it needs no select.
                        eb[j] = from_below_or(cb[j], e0[j]);
                        // The lane shift runs with every lane on (see
                        // bml_resident.hpp).
                        asm volatile("" : "+v"(eb[j]));
                    }
                }
#pragma unroll
                for (int j = 0; j < VG; ++j) {
                    const int i = g + j;
                    if (i < W) {
                        mv0[j] = T0[i] & e1[j];
                        mv1[j] = T1[i] & eb[j];
                    }
                }
#pragma unroll
                for (int j = 0; j < VG; ++j) {
                    const int i = g + j;
                    if (i < W)
                        ar[j] = from_above_or(ca[j] & e0[j], mv1[j]);
                }
#pragma unroll
                for (int j = 0; j < VG; ++j) {
                    const int i = g + j;
                    if (i < W) {
                        T0[i] = xor3(T0[i], mv0[j], ar[j]);
                        T1[i] = xor3(T1[i], mv1[j], mv0[j]);
                    }
                }
                if constexpr (MODEL == 3) {
#pragma unroll
                    for (int j = 0; j < VG; ++j) {
                        const int i = g + j;
                        if (i < W) {
                            L0[i] = xor3(L0[i], m0[j],
                                         __builtin_amdgcn_alignbit(m0[j], j ? m0[j - 1] : q0, 31));
                            L1[i] = xor3(L1[i], m1[j],
                                         __builtin_amdgcn_alignbit(m1[j], j ? m1[j - 1] : q1, 31));
                            if (i >= 1 && i < W - 1) {
                                c_lr = __builtin_popcount(m0[j]) + c_lr;
                                c_l1 = __builtin_popcount(m1[j]) + c_l1;
                                asm("" : "+v"(c_lr), "+v"(c_l1));
                            }
                            if (i == 0)
                                f_lr = (m0[j] >> 31) + (m1[j] >> 31);
                            if (i == W - 2)
                                f_lr -= (m0[j] >> 31) + (m1[j] >> 31);
                            asm("" : "+v"(L0[i]), "+v"(L1[i]));
                        }
                    }
                    const int last = (W - g < VG ? W - g : VG) - 1;
                    q0 = m0[last];
                    q1 = m1[last];
                }
#pragma unroll
                for (int j = 0; j < VG; ++j) {
                    const int i = g + j;
                    if (i >= 1 && i < W - 1) {
                        c_tb = __builtin_popcount(mv0[j]) + c_tb;
                        c_tb1 = __builtin_popcount(mv1[j]) + c_tb1;
                        asm("" : "+v"(c_tb), "+v"(c_tb1));
                    }
                }
#pragma unroll
                for (int j = 0; j < VG; ++j) {
                    const int i = g + j;
                    if (i < W)
                        asm("" : "+v"(T0[i]), "+v"(T1[i]));
                }
                asm("" : "+v"(c_tb), "+v"(c_tb1));
                __builtin_amdgcn_sched_barrier(0);
            }
            c_lr += c_l1;
            // TB cars entering the own rows from the row above them, minus
            // those leaving the last own row (lower-row movers of two lanes)
            uint32_t t2 = 0;
            if (wave == w_in)
                t2 += (uint32_t)__builtin_amdgcn_readlane((int)c_tb1, l_in);
            if (wave == w_out)
                t2 -= (uint32_t)__builtin_amdgcn_readlane((int)c_tb1, l_out);
            c_tb += c_tb1;
            const uint32_t t0 = wave_total(counted ? f_lr : 0u);
            const uint32_t t1 = wave_total(counted ? c_lr : 0u);
            const uint32_t t3 = wave_total(counted ? c_tb : 0u);
            if (lane == 0) {
                sh.cnt[s][wave][0] = t0;
                sh.cnt[s][wave][1] = t1;
                sh.cnt[s][wave][2] = t2;
                sh.cnt[s][wave][3] = t3;
            }
        } else if (lane == 0) {
            sh.cnt[s][wave][0] = sh.cnt[s][wave][1] = sh.cnt[s][wave][2] =
                sh.cnt[s][wave][3] = 0;
        }
    }
    count_cars(1);
    __syncthreads();
    // The tile's counts of every step of the launch: movers as summed; cars
    // as the count after the load plus what crossed the edges up to each
    // step.  If that does not end at the count after the last step, the
    // tile's car counts are written as all ones, so that the lattice's sums
    // fail the conservation check.
    uint32_t *part = a.lat[li].partial + (size_t)local * BLK_MAX_K * 4;
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        uint32_t v = 0, end = 0;
        if (!(q & 1)) {
#pragma unroll
            for (int w = 0; w < BLK_WAVES; ++w) {
                v += sh.cars[0][w][q >> 1];
                end += sh.cars[1][w][q >> 1];
            }
        }
        uint32_t total = v;
        for (int st = 0; st < n_steps; ++st)
#pragma unroll
            for (int w = 0; w < BLK_WAVES; ++w)
                total += sh.cnt[st][w][q];
        const bool bad = !(q & 1) && total != end;
        for (int st = 0; st < n_steps; ++st) {
            uint32_t d = 0;
#pragma unroll
            for (int w = 0; w < BLK_WAVES; ++w)
                d += sh.cnt[st][w][q];
            v = (q & 1) ? d : v + d;
            part[st * 4 + q] = bad ? 0xffffffffu : v;
        }
    }
    if (wave_on) {
#pragma unroll
        for (int c = 0; c < TW / BLK_CHUNK; ++c) {
#pragma unroll
            for (int j = 0; j < BLK_CHUNK; ++j) {
                const int i = 1 + BLK_CHUNK * c + j;
                stL[stage_index(2 * lane, j)] = L0[i];
                stT[stage_index(2 * lane, j)] = T0[i];
                stL[stage_index(2 * lane + 1, j)] = L1[i];
                stT[stage_index(2 * lane + 1, j)] = T1[i];
            }
            wave_sync_lds();
            stage_out(c);
            wave_sync_lds();
        }
    }
}

using BlockFn = void (*)(BlockArgs);
// [layout][0: the two-phase rule, 1: Model III, 2: the two-phase rule on
// the Klein bottle][tile width 32, 16, 8 words]
void block_kernels(BlockFn (*fn)[3][3]);

} // namespace bml
