// bml_tile.hpp -- device building blocks of the BML step kernels (gfx950).
//
// A wavefront streams lattice rows through VGPRs as two bitplanes: lane l
// owns WL consecutive 32-cell words of a row (bit b of word w = cell 32w+b,
// least significant bit = leftmost cell).  The horizontal phase needs the
// words of the lanes on either side (DPP moves by one lane, then a funnel
// shift); the vertical phase only needs the rows above and below, which pass
// through the same lane.  Phase rules: Marzolla, arXiv:1804.07981, Sec. 2
// case tables; synchronous update as in Sec. 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bml {

// ---- cross-lane moves (one 64-lane wavefront) -----------------------------
//
// WRAP = false: lane l receives lane l+1 (or l-1), and the lane past the end
// receives 0 (bound_ctrl writes zero where the source lane is out of range,
// so the destination needs no initialisation).  WRAP = true: the wavefront is
// a ring (wave_rol / wave_ror), for rows that exactly fill it.

template <bool WRAP>
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, WRAP ? 0x134 /* wave_rol:1 */
                                                           : 0x130 /* wave_shl:1 */,
                                              0xF, 0xF, true);
}

template <bool WRAP>
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, WRAP ? 0x13C /* wave_ror:1 */
                                                           : 0x138 /* wave_shr:1 */,
                                              0xF, 0xF, true);
}

// Waits until every vector memory operation this wavefront has issued,
// atomics included, has completed.  The last-block detection of the step
// kernels communicates only through device-scope atomics (performed at the
// device's coherence point), so it needs this completion order but no
// cache-wide write-back or invalidation, which an acquire/release fence at
// device scope would add on every block (each XCD has its own L2).
__device__ __forceinline__ void wait_vector_memory()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Sum of v over the 64 lanes of the wavefront, as a wave-uniform value.
// DPP adds inside each 16-lane row (swap pairs, swap halves of quads, then
// rotate the row by 4 and by 8 lanes) leave every lane with its row's sum;
// the four row sums are then read from lanes 0, 16, 32 and 48.  No LDS
// round trips, so many such sums can be in flight together.
__device__ __forceinline__ uint32_t wave_total(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1 /* quad_perm 1,0,3,2 */, 0xF, 0xF,
                                            false);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E /* quad_perm 2,3,0,1 */, 0xF, 0xF,
                                            false);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124 /* row_ror:4 */, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128 /* row_ror:8 */, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// Horizontal phase of one row (WL words per lane).  A car moves when the
// cell to its right is EMPTY: mv = L & (E shifted one cell left); the new LR
// plane drops the movers and sets their destinations (mv shifted one cell
// right).  Word i's right neighbour is word i+1 of the same lane, or word 0
// of the next lane; its left neighbour is word i-1, or the last word of the
// previous lane.
template <int WL, bool WRAP>
__device__ __forceinline__ void h_row(uint32_t (&L)[WL], const uint32_t (&T)[WL],
                                      uint32_t (&mv)[WL])
{
    uint32_t E[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i)
        E[i] = ~(L[i] | T[i]);
    const uint32_t e_next = from_next_lane<WRAP>(E[0]);
#pragma unroll
    for (int i = 0; i < WL; ++i)
        mv[i] = L[i] & __builtin_amdgcn_alignbit(i + 1 < WL ? E[i + 1] : e_next, E[i], 1);
    const uint32_t mv_prev = from_prev_lane<WRAP>(mv[WL - 1]);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        const uint32_t arrive = __builtin_amdgcn_alignbit(mv[i], i ? mv[i - 1] : mv_prev, 31);
        L[i] = (L[i] & ~mv[i]) | arrive;
        // Opaque new state: stops the compiler from carrying pieces of this
        // expression (e.g. L & ~mv) into the vertical phase as extra live
        // values.
        asm("" : "+v"(L[i]));
    }
}

// The horizontal phase of a row held mirrored (cell order reversed), as the
// Klein-bottle kernels hold the rows that lie across the glued top/bottom
// edge: LR cars then move towards lower bit indices.  A car moves when the
// cell on its lower side is EMPTY (word i-1, or the previous lane's last
// word, supplies bit 31 of that neighbour), and lands one cell lower.
template <int WL, bool WRAP>
__device__ __forceinline__ void h_row_mirrored(uint32_t (&L)[WL], const uint32_t (&T)[WL],
                                               uint32_t (&mv)[WL])
{
    uint32_t E[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i)
        E[i] = ~(L[i] | T[i]);
    const uint32_t e_prev = from_prev_lane<WRAP>(E[WL - 1]);
#pragma unroll
    for (int i = 0; i < WL; ++i)
        mv[i] = L[i] & __builtin_amdgcn_alignbit(E[i], i ? E[i - 1] : e_prev, 31);
    const uint32_t mv_next = from_next_lane<WRAP>(mv[0]);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        const uint32_t arrive = __builtin_amdgcn_alignbit(i + 1 < WL ? mv[i + 1] : mv_next,
                                                          mv[i], 1);
        L[i] = (L[i] & ~mv[i]) | arrive;
        asm("" : "+v"(L[i]));
    }
}

// ---- streaming pipeline level ----------------------------------------------
//
// A wavefront sweeping down a strip keeps one Level per step of the pass.
// Level s receives rows of the lattice after s steps, one row at a time, top
// to bottom.  On receiving row r it applies the horizontal phase to r (row
// local), then completes the vertical phase of the row above, r-1, which
// needs the post-H rows r-2 (through its movers, kept as mvp), r-1 (kept)
// and r; it hands row r-1 after s+1 steps to the next level.  A TB car of
// row r-1 moves when row r is EMPTY there after the horizontal phase.
template <int WL>
struct Level {
    uint32_t L[WL], T[WL];   // pending row r-1 after the horizontal phase
    uint32_t mvp[WL];        // TB movers of row r-2 (they arrive in row r-1)
};

template <int WL>
struct LevelOut {
    uint32_t L[WL], T[WL];       // row r-1 after the step
    uint32_t mv_h[WL], l_h[WL];  // LR movers and new LR plane of row r (H phase)
    uint32_t mv_v[WL];           // TB movers of row r-1 (V phase)
};

// `mirrored` (wave-uniform; only Klein-bottle kernels pass true) says the
// incoming row is held with its cell order reversed.
template <int WL, bool WRAP>
__device__ __forceinline__ LevelOut<WL> level_push(Level<WL> &lv, const uint32_t (&L_in)[WL],
                                                   const uint32_t (&T_in)[WL],
                                                   bool mirrored = false)
{
    LevelOut<WL> o;
    uint32_t L[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i)
        L[i] = L_in[i];
    if (mirrored)
        h_row_mirrored<WL, WRAP>(L, T_in, o.mv_h);
    else
        h_row<WL, WRAP>(L, T_in, o.mv_h);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        o.l_h[i] = L[i];
        const uint32_t mv = lv.T[i] & ~(L[i] | T_in[i]);
        uint32_t t_new = (lv.T[i] & ~mv) | lv.mvp[i];
        asm("" : "+v"(t_new));
        o.L[i] = lv.L[i];
        o.T[i] = t_new;
        o.mv_v[i] = mv;
        lv.L[i] = L[i];
        lv.T[i] = T_in[i];
        lv.mvp[i] = mv;
    }
    return o;
}

// ---- Model II level ----------------------------------------------------------
//
// Model II (Sec. 2): every car advances in one phase per step; an EMPTY
// cell claimed by both an LR car (on its left) and a TB car (above it)
// goes to one of them by a coin (coin bit 1: the LR car moves).  With the
// same skew as level_push: on receiving row r (before this step) the level
// finishes row r itself for the LR cars (their claims need row r-1's TB
// cars, already held) and finishes row r-1 for the TB cars (their targets
// and claims are in row r).  In the bit words, cell j+1 of a word is bit
// j+1, continued into the next word / lane.
template <int WL, bool WRAP>
__device__ __forceinline__ LevelOut<WL> level_push_model2(Level<WL> &lv,
                                                          const uint32_t (&L_in)[WL],
                                                          const uint32_t (&T_in)[WL],
                                                          const uint32_t (&coin)[WL])
{
    LevelOut<WL> o;
    uint32_t E[WL], from_left[WL], claimed[WL], lr_loses[WL], mv[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i)
        E[i] = ~(L_in[i] | T_in[i]);
    // LR car on the left of each cell (bit j <- bit j-1, previous lane's
    // last word supplies bit 0).
    const uint32_t l_prev = from_prev_lane<WRAP>(L_in[WL - 1]);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        from_left[i] = __builtin_amdgcn_alignbit(L_in[i], i ? L_in[i - 1] : l_prev, 31);
        claimed[i] = E[i] & from_left[i] & lv.T[i];   // TB car above, too
        lr_loses[i] = claimed[i] & ~coin[i];
    }
    // An LR car moves when the cell on its right is EMPTY and not lost to
    // the TB car above that cell (bit j <- bit j+1 of E and of lr_loses).
    const uint32_t e_next = from_next_lane<WRAP>(E[0]);
    const uint32_t loss_next = from_next_lane<WRAP>(lr_loses[0]);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        const uint32_t e_right =
            __builtin_amdgcn_alignbit(i + 1 < WL ? E[i + 1] : e_next, E[i], 1);
        const uint32_t loss_right = __builtin_amdgcn_alignbit(
            i + 1 < WL ? lr_loses[i + 1] : loss_next, lr_loses[i], 1);
        mv[i] = L_in[i] & e_right & ~loss_right;
    }
    const uint32_t mv_prev = from_prev_lane<WRAP>(mv[WL - 1]);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        const uint32_t arrive = __builtin_amdgcn_alignbit(mv[i], i ? mv[i - 1] : mv_prev, 31);
        uint32_t l_new = (L_in[i] & ~mv[i]) | arrive;
        asm("" : "+v"(l_new));
        o.mv_h[i] = mv[i];
        o.l_h[i] = l_new;
        // TB cars of row r-1 move into EMPTY cells of row r unless the LR
        // car won the cell.
        const uint32_t mvt = lv.T[i] & E[i] & ~(claimed[i] & coin[i]);
        uint32_t t_new = (lv.T[i] & ~mvt) | lv.mvp[i];
        asm("" : "+v"(t_new));
        o.L[i] = lv.L[i];
        o.T[i] = t_new;
        o.mv_v[i] = mvt;
        lv.L[i] = l_new;
        lv.T[i] = T_in[i];
        lv.mvp[i] = mvt;
    }
    return o;
}

// Model III level (Sec. 2: a cell may hold an LR and a TB car): the phase of
// level_push_model2 without the coin.  A car moves when its target held no
// car before the step, and an EMPTY cell wanted by both an LR car (left) and
// a TB car (above) takes both, so no move is ever lost; a cell with both
// bits set blocks cars of either type, and each of its cars leaves by its
// own rule.
template <int WL, bool WRAP>
__device__ __forceinline__ LevelOut<WL> level_push_model3(Level<WL> &lv,
                                                          const uint32_t (&L_in)[WL],
                                                          const uint32_t (&T_in)[WL])
{
    LevelOut<WL> o;
    uint32_t E[WL], mv[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i)
        E[i] = ~(L_in[i] | T_in[i]);
    const uint32_t e_next = from_next_lane<WRAP>(E[0]);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        const uint32_t e_right =
            __builtin_amdgcn_alignbit(i + 1 < WL ? E[i + 1] : e_next, E[i], 1);
        mv[i] = L_in[i] & e_right;
    }
    const uint32_t mv_prev = from_prev_lane<WRAP>(mv[WL - 1]);
#pragma unroll
    for (int i = 0; i < WL; ++i) {
        const uint32_t arrive = __builtin_amdgcn_alignbit(mv[i], i ? mv[i - 1] : mv_prev, 31);
        uint32_t l_new = (L_in[i] & ~mv[i]) | arrive;
        asm("" : "+v"(l_new));
        o.mv_h[i] = mv[i];
        o.l_h[i] = l_new;
        // TB cars of row r-1 move into the cells of row r that held no car.
        const uint32_t mvt = lv.T[i] & E[i];
        uint32_t t_new = (lv.T[i] & ~mvt) | lv.mvp[i];
        asm("" : "+v"(t_new));
        o.L[i] = lv.L[i];
        o.T[i] = t_new;
        o.mv_v[i] = mvt;
        lv.L[i] = l_new;
        lv.T[i] = T_in[i];
        lv.mvp[i] = mvt;
    }
    return o;
}

// Model II coin word: the low 32 bits of SplitMix64 output number k of the
// stream started at `seed` (Steele, Lea and Flood; Vigna's constants);
// k = step * rows * words + row * words + word, bit b = the coin of cell
// 32 word + b.  Output k mixes seed + (k + 1) * gamma; the kernels split the
// product as seed + (row_base + 1) * gamma (uniform per row) plus
// word * gamma (fixed per lane), so a word costs one 64-bit add and the mix.
constexpr uint64_t SPLITMIX64_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint32_t splitmix64_mix_lo(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (uint32_t)(z ^ (z >> 31));
}

__device__ __forceinline__ uint32_t model2_coin_word(uint64_t seed, uint64_t k)
{
    return splitmix64_mix_lo(seed + (k + 1ull) * SPLITMIX64_GAMMA);
}

// ---- byte cells <-> bitplane words -----------------------------------------
//
// Byte j of a 32-byte chunk (cells 32w .. 32w+31) holds 0, 1 or 2; bit 0 of
// the byte says LR, bit 1 says TB.  d[q] holds cells 4q .. 4q+3 (byte j of
// the dword is cell 4q + j) and bit c of a plane word is cell 32w + c.

// Gathering bit 0 (or bit 1) of every byte with shifts leaves the bit of
// cell 4q + k at position 8k + q; index_rotl2 moves it to 4q + k, i.e. it
// rotates the 5-bit position index left by two with four delta swaps (each
// exchanges two index bits).  Plain shifts and masks only: the conversion
// stays on the ordinary 32-bit VALU instructions.
__device__ __forceinline__ uint32_t delta_swap(uint32_t x, int s, uint32_t m)
{
    const uint32_t t = ((x >> s) ^ x) & m;
    return x ^ t ^ (t << s);
}

__device__ __forceinline__ uint32_t index_rotl2(uint32_t x)
{
    x = delta_swap(x, 1, 0x22222222u);
    x = delta_swap(x, 2, 0x0c0c0c0cu);
    x = delta_swap(x, 7, 0x00aa00aau);
    x = delta_swap(x, 14, 0x0000ccccu);
    return x;
}

__device__ __forceinline__ void bytes_to_planes(const uint32_t *d, uint32_t &lr, uint32_t &tb)
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

// The inverse spreads a nibble over the four bytes of a dword: n * 0x204081
// is n + (n << 7) + (n << 14) + (n << 21), four copies that cannot overlap,
// so bit i of n lands on bit 8i (and, with 0x408102, on bit 8i + 1); the
// masks drop the other copies' bits.
__device__ __forceinline__ void planes_to_bytes(uint32_t lr, uint32_t tb, uint32_t *d)
{
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t nl = (lr >> (4 * q)) & 15u;
        const uint32_t nt = (tb >> (4 * q)) & 15u;
        d[q] = ((nl * 0x00204081u) & 0x01010101u) | ((nt * 0x00408102u) & 0x02020202u);
    }
}

} // namespace bml
