// bml_block.hpp -- register-resident tile kernel for single lattices
// (gfx950): up to 32 steps per HBM pass.
//
// The lattice is cut into tiles of 32 words (1024 cells) by up to 512 - 2K
// rows.  A 4-wave workgroup holds one tile with one halo word on each side
// and K halo rows above and below, two rows per lane (34 LR and 34 TB words
// per row), loads it once, advances it K steps in registers and stores the
// tile's own words and rows.  The rule of Marzolla, arXiv:1804.07981,
// Sec. 2 decides every move from the cell's neighbour in the direction of
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

#include "bml_pass.hpp"
#include "bml_resident.hpp"
#include "bml_tile.hpp"

namespace bml {

constexpr int BLK_WORDS = 32;                 // tile words (columns / 32)
constexpr int BLK_W = BLK_WORDS + 2;          // words held per row: a halo word each side
constexpr int BLK_WAVES = 4;                  // one wave per SIMD, two workgroups per CU
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

struct BlockShared {
    uint32_t x[2][BLK_WAVES][2][BLK_W];      // as ResidentShared::x
    uint32_t none[BLK_W];                     // zero: no neighbour beyond the halo rows
    uint32_t cnt[BLK_MAX_K][BLK_WAVES][4];    // per-wave counts of each step
};

template <int IO>
__global__ __launch_bounds__(64 * BLK_WAVES, 2) void block_kernel(BlockArgs a)
{
    constexpr int W = BLK_W;
    __shared__ BlockShared sh;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tiles = a.tiles_x * a.slabs;
    const int li = blockIdx.x / tiles;
    const int local = blockIdx.x - li * tiles;
    const int slab = local / a.tiles_x;
    const int tx = local - slab * a.tiles_x;
    const int blocks32 = a.rows / 32;
    const int r0 = blocks32 * slab / a.slabs * 32;
    const int R = blocks32 * (slab + 1) / a.slabs * 32 - r0;
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

    // Lattice rows of the lane (periodic) and word w0 - 1 + i (periodic).
    const int g0 = row_ok ? (r0 - H + row + 2 * N) % N : 0;
    const int g1 = g0 + 1 == N ? 0 : g0 + 1;
    const int w0 = tx * BLK_WORDS;
    uint32_t L0[W], T0[W], L1[W], T1[W];
    auto load_row = [&](int g, uint32_t (&Lr)[W], uint32_t (&Tr)[W]) {
        const uint32_t ro = (uint32_t)g * row_bytes;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const int w = i == 0 ? (w0 == 0 ? words - 1 : w0 - 1)
                                 : (w0 + i - 1 == words ? 0 : w0 + i - 1);
            if constexpr (IO == IO_U8) {
                const u32x4 u0 = __builtin_amdgcn_raw_buffer_load_b128(
                    src, ro + (uint32_t)w * 32u, 0, 0);
                const u32x4 u1 = __builtin_amdgcn_raw_buffer_load_b128(
                    src, ro + (uint32_t)w * 32u + 16u, 0, 0);
                const uint32_t dw[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
                bytes_to_planes(dw, Lr[i], Tr[i]);
            } else {
                Lr[i] = __builtin_amdgcn_raw_buffer_load_b32(src, ro + (uint32_t)w * 4u, 0, 0);
                Tr[i] = __builtin_amdgcn_raw_buffer_load_b32(
                    src, ro + plane_bytes + (uint32_t)w * 4u, 0, 0);
            }
        }
    };
    auto store_row = [&](int g, const uint32_t (&Lr)[W], const uint32_t (&Tr)[W]) {
        const uint32_t ro = (uint32_t)g * row_bytes;
#pragma unroll
        for (int i = 1; i < W - 1; ++i) {
            const uint32_t w = (uint32_t)(w0 + i - 1);
            if constexpr (IO == IO_U8) {
                uint32_t b[8];
                planes_to_bytes(Lr[i], Tr[i], b);
                __builtin_amdgcn_raw_buffer_store_b128((u32x4){b[0], b[1], b[2], b[3]}, dst,
                                                       ro + w * 32u, 0, 0);
                __builtin_amdgcn_raw_buffer_store_b128((u32x4){b[4], b[5], b[6], b[7]}, dst,
                                                       ro + w * 32u + 16u, 0, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b32(Lr[i], dst, ro + w * 4u, 0, 0);
                __builtin_amdgcn_raw_buffer_store_b32(Tr[i], dst, ro + plane_bytes + w * 4u, 0,
                                                      0);
            }
        }
    };
#pragma unroll
    for (int i = 0; i < W; ++i)
        L0[i] = T0[i] = L1[i] = T1[i] = 0;
    if (row_ok) {
        load_row(g0, L0, T0);
        load_row(g1, L1, T1);
    }
    if (threadIdx.x < W)
        sh.none[threadIdx.x] = 0;

    // Horizontal phase of one row with open ends: the cell beyond the last
    // held one counts as occupied, nothing arrives into the first.  Every
    // mover is decided before any word changes.  Returns the LR movers of
    // the tile's own words; E receives the row's emptiness after the phase.
    auto hphase = [&](uint32_t (&Lr)[W], const uint32_t (&Tr)[W], uint32_t (&E)[W],
                      uint32_t &n_lr) {
        uint32_t c = 0;
        uint32_t mv_prev = 0, o = Lr[0] | Tr[0];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const uint32_t on = i + 1 < W ? (Lr[i + 1] | Tr[i + 1]) : 0xffffffffu;
            const uint32_t mv = Lr[i] & ~__builtin_amdgcn_alignbit(on, o, 1);
            o = on;
            const uint32_t arrive = __builtin_amdgcn_alignbit(mv, mv_prev, 31);
            Lr[i] = Lr[i] ^ mv ^ arrive;    // movers leave, arrivals land (disjoint)
            E[i] = ~(Lr[i] | Tr[i]);
            if (i >= 1 && i < W - 1) {
                c += __builtin_popcount(mv);
                n_lr += __builtin_popcount(Lr[i]);
            }
            // Opaque new values (and counts): updated in place here, not
            // carried as pieces to the end of the step.
            asm("" : "+v"(Lr[i]), "+v"(E[i]), "+v"(c), "+v"(n_lr));
            mv_prev = mv;
            if ((i + 1) % RES_GROUP == 0)
                __builtin_amdgcn_sched_barrier(0);
        }
        return c;
    };

    for (int s = 0; s < n_steps; ++s) {
        const int p = s & 1;
        uint32_t E0[W], E1[W];
        uint32_t n_lr = 0, c_lr = 0, n_tb = 0, c_tb = 0;
        if (wave_on) {
            c_lr = hphase(L0, T0, E0, n_lr);
            c_lr += hphase(L1, T1, E1, n_lr);
            if (lane == 0) {
#pragma unroll
                for (int i = 0; i < W; ++i)
                    sh.x[p][wave][0][i] = E0[i];
            }
            if (lane == last_lane) {
#pragma unroll
                for (int i = 0; i < W; ++i)
                    sh.x[p][wave][1][i] = T1[i];
            }
        }
        __syncthreads();
        if (wave_on) {
            const uint32_t *xb = wdown >= 0 ? sh.x[p][wdown][0] : sh.none;
            const uint32_t *xa = wup >= 0 ? sh.x[p][wup][1] : sh.none;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const uint32_t e_x = xb[i];
                const uint32_t t_x = xa[i];
                uint32_t e_below = from_below_or(e_x, E0[i]);
                // The lane shift runs with every lane on (see bml_resident.hpp).
                asm volatile("" : "+v"(e_below));
                e_below = lane == last_lane ? e_x : e_below;
                const uint32_t mv0 = T0[i] & E1[i];
                const uint32_t mv1 = T1[i] & e_below;
                const uint32_t arrive = from_above_or(t_x & E0[i], mv1);
                T0[i] = T0[i] ^ mv0 ^ arrive;
                T1[i] = T1[i] ^ mv1 ^ mv0;
                if (i >= 1 && i < W - 1) {
                    c_tb += __builtin_popcount(mv0) + __builtin_popcount(mv1);
                    n_tb += __builtin_popcount(T0[i]) + __builtin_popcount(T1[i]);
                }
                asm("" : "+v"(T0[i]), "+v"(T1[i]), "+v"(c_tb), "+v"(n_tb));
                if ((i + 1) % RES_GROUP == 0)
                    __builtin_amdgcn_sched_barrier(0);
            }
            const uint32_t t0 = wave_total(counted ? n_lr : 0u);
            const uint32_t t1 = wave_total(counted ? c_lr : 0u);
            const uint32_t t2 = wave_total(counted ? n_tb : 0u);
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
    __syncthreads();
    // The tile's counts of every step of the launch.
    uint32_t *part = a.lat[li].partial + (size_t)local * BLK_MAX_K * 4;
    for (int j = threadIdx.x; j < n_steps * 4; j += blockDim.x) {
        const int st = j >> 2, q = j & 3;
        uint32_t v = 0;
#pragma unroll
        for (int w = 0; w < BLK_WAVES; ++w)
            v += sh.cnt[st][w][q];
        part[j] = v;
    }
    if (counted) {
        store_row(g0, L0, T0);
        store_row(g1, L1, T1);
    }
}

using BlockFn = void (*)(BlockArgs);
void block_kernels(BlockFn *u8, BlockFn *bp);

} // namespace bml
