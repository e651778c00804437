// bml_tile.hpp -- device building blocks of the BML step kernels (gfx950).
//
// A wavefront holds a tile of the lattice in VGPRs as two bitplanes: lane l
// owns one 32-cell word column (bit b = cell 32w+b, least significant bit =
// leftmost cell), register index r one row.  The horizontal phase needs the
// words of the lanes on either side (DPP wave_shl/wave_shr by one lane, then
// a funnel shift); the vertical phase only needs the rows above and below,
// which are in the same lane.  Phase rules: Marzolla, arXiv:1804.07981,
// Sec. 2 case tables; synchronous update as in Sec. 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bml {

// ---- cross-lane moves (one 64-lane wavefront) -----------------------------

// Lane l receives the value of lane l+1 (lane 63 receives 0: bound_ctrl
// writes zero where the source lane is out of range, so the destination
// needs no initialisation).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}

// Lane l receives the value of lane l-1 (lane 0 receives 0).
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}

// ---- the two phases on a register tile ------------------------------------
//
// L[r], T[r]: LR and TB planes of tile row r.  Rows [lo, hi) are updated; the
// rows outside that range are stale halo.  Counting covers rows
// [cnt_lo, cnt_hi) only.  All bounds are compile-time constants.

// Horizontal phase of one row.  A car moves when the cell to its right is
// EMPTY: mv = L & (E shifted one cell left); the new LR plane drops the
// movers and sets their destinations (mv shifted one cell right).
__device__ __forceinline__ uint32_t h_row(uint32_t &L, uint32_t T)
{
    const uint32_t E = ~(L | T);
    const uint32_t e_right = __builtin_amdgcn_alignbit(from_next_lane(E), E, 1);
    const uint32_t mv = L & e_right;
    const uint32_t arrive = __builtin_amdgcn_alignbit(mv, from_prev_lane(mv), 31);
    L = (L & ~mv) | arrive;
    // Opaque new state: stops the compiler from carrying pieces of this
    // expression (e.g. L & ~mv) into the vertical phase as extra live values.
    asm("" : "+v"(L));
    return mv;
}

template <int R, int lo, int hi, int cnt_lo, int cnt_hi>
__device__ __forceinline__ void h_phase(uint32_t (&L)[R], const uint32_t (&T)[R],
                                        uint32_t &moved, uint32_t &cars)
{
#pragma unroll
    for (int r = lo; r < hi; ++r) {
        const uint32_t mv = h_row(L[r], T[r]);
        if (r >= cnt_lo && r < cnt_hi) {
            moved += __builtin_popcount(mv);
            cars += __builtin_popcount(L[r]);
            // Count now: keeps the compiler from sinking the popcounts to
            // their single use, which would hold every row's mask live.
            asm volatile("" : "+v"(moved), "+v"(cars));
        }
    }
}

// Vertical phase.  A TB car at row r moves when row r+1 is EMPTY there:
// mv[r] = T[r] & ~(L[r+1] | T[r+1]); the new T[r] drops mv[r] and gains the
// arrivals mv[r-1].  Rows are visited top-down so that T[r+1] is still the
// pre-phase value when mv[r] is formed.  Row lo keeps its movers out but
// receives nothing (its upper neighbour is stale), so it becomes stale too;
// the caller shrinks [lo, hi) by one row per phase.
template <int R, int lo, int hi, int cnt_lo, int cnt_hi>
__device__ __forceinline__ void v_phase(const uint32_t (&L)[R], uint32_t (&T)[R],
                                        uint32_t &moved, uint32_t &cars)
{
    uint32_t prev = 0;
#pragma unroll
    for (int r = lo; r < hi - 1; ++r) {
        const uint32_t mv = T[r] & ~(L[r + 1] | T[r + 1]);
        const uint32_t nt = (T[r] & ~mv) | prev;
        T[r] = nt;
        asm("" : "+v"(T[r]));
        prev = mv;
        if (r >= cnt_lo && r < cnt_hi) {
            moved += __builtin_popcount(mv);
            cars += __builtin_popcount(nt);
            asm volatile("" : "+v"(moved), "+v"(cars));
        }
    }
}

// ---- streaming pipeline level ----------------------------------------------
//
// A wavefront sweeping down a strip keeps one Level per step of the pass.
// Level s receives rows of the lattice after s steps, one row at a time, top
// to bottom.  On receiving row r it applies the horizontal phase to r (row
// local), then completes the vertical phase of the row above, r-1, which
// needs the post-H rows r-2 (through its movers, kept as mvp), r-1 (kept)
// and r; it hands row r-1 after s+1 steps to the next level.
struct Level {
    uint32_t L, T;   // pending row r-1 after the horizontal phase
    uint32_t mvp;    // TB movers of row r-2 (they arrive in row r-1)
};

struct LevelOut {
    uint32_t L, T;       // row r-1 after the step
    uint32_t mv_h, l_h;  // LR movers and new LR plane of row r (H phase)
    uint32_t mv_v;       // TB movers of row r-1 (V phase)
};

__device__ __forceinline__ LevelOut level_push(Level &lv, uint32_t L_in, uint32_t T_in)
{
    LevelOut o;
    uint32_t L = L_in;
    o.mv_h = h_row(L, T_in);
    o.l_h = L;
    const uint32_t mv = lv.T & ~(L | T_in);
    uint32_t t_new = (lv.T & ~mv) | lv.mvp;
    asm("" : "+v"(t_new));
    o.L = lv.L;
    o.T = t_new;
    o.mv_v = mv;
    lv.L = L;
    lv.T = T_in;
    lv.mvp = mv;
    return o;
}

// ---- byte cells <-> bitplane words -----------------------------------------
//
// Byte j of a 32-byte chunk (cells 32w .. 32w+31) holds 0, 1 or 2; bit 0 of
// the byte says LR, bit 1 says TB.

// Moves the bit at position p = 8k + q (k = p >> 3, q = p & 7) to position
// 4q + k, i.e. rotates the 5-bit position index left by two, using four
// delta swaps (each exchanges two index bits).
__host__ __device__ __forceinline__ uint32_t delta_swap(uint32_t x, int s, uint32_t m)
{
    const uint32_t t = ((x >> s) ^ x) & m;
    return x ^ t ^ (t << s);
}

__host__ __device__ __forceinline__ uint32_t index_rotl2(uint32_t x)
{
    x = delta_swap(x, 1, 0x22222222u);
    x = delta_swap(x, 2, 0x0c0c0c0cu);
    x = delta_swap(x, 7, 0x00aa00aau);
    x = delta_swap(x, 14, 0x0000ccccu);
    return x;
}

// Inverse of index_rotl2: position 4q + k goes back to 8k + q.
__host__ __device__ __forceinline__ uint32_t index_rotl3(uint32_t x)
{
    x = delta_swap(x, 1, 0x22222222u);
    x = delta_swap(x, 3, 0x0a0a0a0au);
    x = delta_swap(x, 6, 0x00cc00ccu);
    x = delta_swap(x, 12, 0x0000f0f0u);
    return x;
}

// d[q] holds cells 4q .. 4q+3 (byte k = cell 4q + k).
__host__ __device__ __forceinline__ void bytes_to_planes(const uint32_t (&d)[8],
                                                         uint32_t &lr, uint32_t &tb)
{
    uint32_t a = 0, b = (d[0] >> 1) & 0x01010101u;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        a |= (d[q] & 0x01010101u) << q;
#pragma unroll
    for (int q = 1; q < 8; ++q)
        b |= (d[q] & 0x02020202u) << (q - 1);
    lr = index_rotl2(a);
    tb = index_rotl2(b);
}

__host__ __device__ __forceinline__ void planes_to_bytes(uint32_t lr, uint32_t tb,
                                                         uint32_t (&d)[8])
{
    const uint32_t a = index_rotl3(lr);
    const uint32_t b = index_rotl3(tb);
    d[0] = (a & 0x01010101u) | ((b << 1) & 0x02020202u);
#pragma unroll
    for (int q = 1; q < 8; ++q)
        d[q] = ((a >> q) & 0x01010101u) | ((b >> (q - 1)) & 0x02020202u);
}

} // namespace bml
