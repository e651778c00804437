// bml_resident.hpp -- register-resident batched BML kernel (gfx950): the
// lattices of a batch with N <= 1024 stay in VGPRs for many steps per
// launch.
//
// Layout: two rows per lane.  A lane holds two consecutive rows, each as
// W = N / 32 LR words and W TB words (bit b of word i = cell 32 i + b), so
// the horizontal phase (Marzolla, arXiv:1804.07981, Sec. 2 case table for
// LR cars) is entirely inside the lane: a ring of W words, periodic in x
// with no halo.  The vertical phase passes cars from a lane's upper row to
// its lower row in registers, and from its lower row to the next lane's
// upper row by DPP wave shifts; rows across a wavefront boundary come from
// the neighbouring wavefront through LDS.  One barrier per step separates
// the exchange writes (after the horizontal phase) from the reads; the
// exchange slots alternate between two buffers by step parity, so a wave
// can never overwrite a slot a slower wave has yet to read.  Both phases
// read only the state before the phase (the synchronous rule of Sec. 3):
// the horizontal phase decides every move from the words before any of
// them changes, and the vertical phase from the post-horizontal occupancy.
// Two rows per lane halve the wave shifts per row and the per-wave work
// that does not depend on W.  A workgroup is 4 wavefronts (one per SIMD);
// at most 168 VGPRs per lane let three workgroups share a CU, so each SIMD
// interleaves three waves.
//
// Work items.  An item is either a whole lattice (halo 0: its last row's
// lower neighbour is its first row, the periodic edge of Sec. 2) or a slab
// of R rows of a lattice held with H halo rows above and below (rows
// r0 - H .. r0 + R + H - 1, periodic in the lattice).  A slab's outermost
// rows have no neighbour beyond them; what they miss travels at most one
// row per step, so after at most H steps the R rows of the slab are still
// exact (the halo absorbs the error) and only they are stored and counted.
// Slabs let one lattice spread over several workgroups (CUs) for the K <= H
// steps of a launch, at the price of recomputing the halo rows.
//
// A workgroup (4 wavefronts) runs a bin of items of one row width W:
// ceil(rows held / 128) wavefronts each.  Per step and item the moved counts
// of the two phases are summed (wave total, then LDS) and added to the
// lattice's trace entry.  The state is read once at the start of a launch
// and written once at the end: the step loop touches only VGPRs and LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bml_batch.hpp"
#include "bml_tile.hpp"

namespace bml {

constexpr int RES_MAX_WORDS = 32;   // N <= 1024
constexpr int RES_WAVES = 4;        // waves per block (one per SIMD; three blocks per CU)
constexpr int RES_WAVE_ROWS = 128;  // rows per wave: two per lane
constexpr int RES_MAX_ITEMS = RES_WAVES;   // items per block (each starts a wave)
constexpr int RES_GROUP = 4;        // words per scheduling group of the step loop
constexpr int RES_CHUNK = 32;       // steps whose counts are gathered in LDS before a flush

// One lattice, or one slab of one.
struct ResidentItem {
    int32_t lattice;                // batch index
    int32_t r0;                     // first row stored (0 for a whole lattice)
    int32_t rows;                   // rows stored: N for a whole lattice
    int32_t halo;                   // halo rows above and below (0: whole, periodic)
    int32_t slab;                   // the slab's index in its lattice (-1: whole lattice)
};

// Items of one row width run by one block.
struct ResidentBin {
    int32_t words;                  // W = N / 32 of every item in the bin
    int32_t n_items;
    ResidentItem item[RES_MAX_ITEMS];
};

struct ResidentArgs {
    const BatchLattice *lat;
    const ResidentBin *bins;
    BatchCounters *ctr;
    uint32_t *trace;                // [lattice][trace_steps][2]: LR moved, TB moved
    int32_t trace_steps;
    int32_t n_steps;                // steps of this launch (<= every slab's halo)
};

// Lane l receives v of lane l+1 (the row below); lane 63 keeps `old`.
__device__ __forceinline__ uint32_t from_below_or(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x130 /* wave_shl:1 */, 0xF,
                                                 0xF, false);
}

// Lane l receives v of lane l-1 (the row above); lane 0 keeps `old`.
__device__ __forceinline__ uint32_t from_above_or(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x138 /* wave_shr:1 */, 0xF,
                                                 0xF, false);
}

// Exchange slots: [step parity][wave][0: emptiness of the wave's first row
// after the horizontal phase, 1: TB plane of its last row][word]; `none`
// stands for the missing neighbour beyond a slab's outermost rows (no car
// above, no empty cell below).
struct ResidentShared {
    alignas(16) uint32_t x[2][RES_WAVES][2][RES_MAX_WORDS];   // read 16 bytes at a time
    uint32_t none[RES_MAX_WORDS];
    // Moved counts [chunk parity][step in chunk][item][LR, TB], gathered
    // over RES_CHUNK steps and then added to the trace in one burst: a
    // global write inside the step loop would hold the barrier until it
    // completes, every step.
    uint32_t cnt[2][RES_CHUNK][RES_MAX_ITEMS][2];
};

// a ^ b ^ c as one three-input bit operation
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// SLAB: the bin is one slab of a taller lattice (open ends with halo rows)
// rather than whole lattices (periodic).
template <int IO, int W, bool SLAB>
__device__ __forceinline__ void resident_body(const ResidentArgs &a, const ResidentBin &bin,
                                              ResidentShared &sh)
{
    constexpr int N = 32 * W;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_items = __builtin_amdgcn_readfirstlane(bin.n_items);
    // This wave's item: items take consecutive waves, ceil(held rows / 128)
    // each.
    int slot = -1, first = 0, waves = 0;
    for (int it = 0, w0 = 0; it < n_items; ++it) {
        const int held = __builtin_amdgcn_readfirstlane(bin.item[it].rows) +
                         2 * __builtin_amdgcn_readfirstlane(bin.item[it].halo);
        const int nw = (held + RES_WAVE_ROWS - 1) / RES_WAVE_ROWS;
        if (wave >= w0 && wave < w0 + nw) {
            slot = it;
            first = w0;
            waves = nw;
        }
        w0 += nw;
    }
    const bool wave_on = slot >= 0;
    int li = 0, r0 = 0, R = 0, H = 0;
    if (wave_on) {
        li = __builtin_amdgcn_readfirstlane(bin.item[slot].lattice);
        r0 = __builtin_amdgcn_readfirstlane(bin.item[slot].r0);
        R = __builtin_amdgcn_readfirstlane(bin.item[slot].rows);
        H = __builtin_amdgcn_readfirstlane(bin.item[slot].halo);
    }
    const int held = R + 2 * H;
    const int wl = wave - first;                 // wave within its item
    const int row = wl * RES_WAVE_ROWS + 2 * lane;   // the lane's upper row within the item
    const bool row_ok = wave_on && row < held;
    // H and R are even, so a lane's two rows are both counted or neither.
    const bool counted = row_ok && row >= H && row < H + R;
    // Lanes of the item's last wave: held rows are a multiple of 32, so 16,
    // 32, 48 or 64.
    const int lanes = wave_on ? min(64, (held - wl * RES_WAVE_ROWS) / 2) : 64;
    const int last_lane = lanes - 1;
    // Neighbouring waves (exchange slots); across the item's ends: the
    // other end for a whole lattice (periodic), none (-1) for a slab.
    const bool open = H > 0;
    const int wdown = wl + 1 < waves ? wave + 1 : open ? -1 : first;
    const int wup = wl > 0 ? wave - 1 : open ? -1 : first + waves - 1;
    const uint32_t step0 = __builtin_amdgcn_readfirstlane(a.ctr->step);
    const uint32_t pass = __builtin_amdgcn_readfirstlane(a.ctr->pass);
    const int n_steps = a.n_steps;

    uint8_t *dst = nullptr;
    // Upper row (L0, T0) and lower row (L1, T1) of the lane.
    uint32_t L0[W], T0[W], L1[W], T1[W];
#pragma unroll
    for (int i = 0; i < W; ++i)
        L0[i] = T0[i] = L1[i] = T1[i] = 0;
    // Lattice rows held by this lane.
    const int g0 = row_ok ? (r0 - H + row + 2 * N) % N : 0;
    const int g1 = g0 + 1 == N ? 0 : g0 + 1;
    auto load_row = [&](const uint8_t *src, int g, uint32_t (&Lr)[W], uint32_t (&Tr)[W]) {
        if constexpr (IO == IO_U8) {
            const uint4 *p = (const uint4 *)(src + (size_t)g * N);
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const uint4 u0 = p[2 * i], u1 = p[2 * i + 1];
                const uint32_t dw[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
                bytes_to_planes(dw, Lr[i], Tr[i]);
            }
        } else {
            const uint32_t *pl = (const uint32_t *)src + (size_t)g * W;
            const uint32_t *pt = pl + (size_t)N * W;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                Lr[i] = pl[i];
                Tr[i] = pt[i];
            }
        }
    };
    auto store_row = [&](int g, const uint32_t (&Lr)[W], const uint32_t (&Tr)[W]) {
        if constexpr (IO == IO_U8) {
            uint4 *q = (uint4 *)(dst + (size_t)g * N);
#pragma unroll
            for (int i = 0; i < W; ++i) {
                uint32_t b[8];
                planes_to_bytes(Lr[i], Tr[i], b);
                q[2 * i] = make_uint4(b[0], b[1], b[2], b[3]);
                q[2 * i + 1] = make_uint4(b[4], b[5], b[6], b[7]);
            }
        } else {
            uint32_t *pl = (uint32_t *)dst + (size_t)g * W;
            uint32_t *pt = pl + (size_t)N * W;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                pl[i] = Lr[i];
                pt[i] = Tr[i];
            }
        }
    };
    if (wave_on) {
        const BatchLattice &d = a.lat[li];
        const int par = (__builtin_amdgcn_readfirstlane(d.parity_base) +
                         (int)(pass - (uint32_t)__builtin_amdgcn_readfirstlane(d.pass_base))) & 1;
        const uint8_t *src = (const uint8_t *)d.buf[par];
        dst = (uint8_t *)d.buf[par ^ 1];
        if (row_ok) {
            load_row(src, g0, L0, T0);
            load_row(src, g1, L1, T1);
        }
    }

    // The count slots and the missing-neighbour row are first used after
    // the first step's barrier.
    for (int i = threadIdx.x; i < 2 * RES_CHUNK * RES_MAX_ITEMS * 2; i += blockDim.x)
        (&sh.cnt[0][0][0][0])[i] = 0;
    if (threadIdx.x < RES_MAX_WORDS)
        sh.none[threadIdx.x] = 0;
    // Writes the gathered counts of steps [c0, c1) (one chunk) to the trace
    // and clears their slots; run by the first wave of each item.  A whole
    // lattice stores its trace entries; the slabs of a lattice add theirs
    // into the lattice's entries, which the run zeroed before its first
    // launch (at most a few slabs add to one entry, once per chunk).
    const bool is_slab = wave_on && __builtin_amdgcn_readfirstlane(bin.item[slot].slab) >= 0;
    auto flush = [&](int c0, int c1) {
        const int kb = (c0 / RES_CHUNK) & 1;
        for (int j = lane; j < 2 * (c1 - c0); j += 64) {
            const int st = c0 + (j >> 1), q = j & 1;
            uint32_t &slotv = sh.cnt[kb][st - c0][slot][q];
            const uint32_t v = slotv;
            slotv = 0;
            const uint32_t gs = step0 + (uint32_t)st;
            if (gs < (uint32_t)a.trace_steps) {
                uint32_t *t = &a.trace[((size_t)li * a.trace_steps + gs) * 2 + q];
                if (is_slab)
                    __hip_atomic_fetch_add(t, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else
                    *t = v;
            }
        }
    };

    // Horizontal phase of both rows: an LR car moves when the next cell
    // (bit j + 1, continued into the next word, word W-1 wrapping to word
    // 0) is EMPTY; it lands one cell further.  Every mover is decided before
    // any word changes.  Words go in groups of RES_GROUP, each stage of the
    // rule applied to the group's words of both rows before the next stage,
    // so that consecutive instructions rarely depend on each other, with
    // scheduling barriers between groups so that only a group's temporaries
    // are live next to the state.  Returns the movers' count.  The emptiness
    // the vertical phase needs is recomputed there from the planes (no
    // array of it stays live).
    auto hphase = [&]() {
        uint32_t c0 = 0, c1 = 0;
        const uint32_t q0 = L0[0] | T0[0], q1 = L1[0] | T1[0];   // word 0 before the phase
        const uint32_t last0 = L0[W - 1] & ~__builtin_amdgcn_alignbit(q0, L0[W - 1] | T0[W - 1], 1);
        const uint32_t last1 = L1[W - 1] & ~__builtin_amdgcn_alignbit(q1, L1[W - 1] | T1[W - 1], 1);
        uint32_t p0 = last0, p1 = last1, o0 = q0, o1 = q1;
#pragma unroll
        for (int g = 0; g < W; g += RES_GROUP) {
            uint32_t m0[RES_GROUP], m1[RES_GROUP];
#pragma unroll
            for (int j = 0; j < RES_GROUP; ++j) {     // movers: the next cell is empty
                const int i = g + j;
                if (i + 1 < W) {
                    const uint32_t on0 = L0[i + 1] | T0[i + 1], on1 = L1[i + 1] | T1[i + 1];
                    m0[j] = L0[i] & ~__builtin_amdgcn_alignbit(on0, o0, 1);
                    m1[j] = L1[i] & ~__builtin_amdgcn_alignbit(on1, o1, 1);
                    o0 = on0;
                    o1 = on1;
                } else if (i + 1 == W) {
                    m0[j] = last0;
                    m1[j] = last1;
                }
            }
#pragma unroll
            for (int j = 0; j < RES_GROUP; ++j) {     // movers leave, arrivals land (disjoint)
                const int i = g + j;
                if (i < W) {
                    L0[i] = xor3(L0[i], m0[j], __builtin_amdgcn_alignbit(m0[j], j ? m0[j - 1] : p0, 31));
                    L1[i] = xor3(L1[i], m1[j], __builtin_amdgcn_alignbit(m1[j], j ? m1[j - 1] : p1, 31));
                    c0 = __builtin_popcount(m0[j]) + c0;
                    c1 = __builtin_popcount(m1[j]) + c1;
                    asm("" : "+v"(c0), "+v"(c1));
                }
            }
            const int last = (W - g < RES_GROUP ? W - g : RES_GROUP) - 1;
            p0 = m0[last];
            p1 = m1[last];
            // Opaque new values: updated in place here, not carried as
            // pieces to the end of the step.
#pragma unroll
            for (int j = 0; j < RES_GROUP; ++j) {
                const int i = g + j;
                if (i < W)
                    asm("" : "+v"(L0[i]), "+v"(L1[i]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        return c0 + c1;
    };

    for (int s = 0; s < n_steps; ++s) {
        const int p = s & 1;
        uint32_t c_lr = 0, c_tb = 0, c_tb1 = 0;
        if (wave_on) {
            c_lr = hphase();
            // Exchange: the wave's first row's emptiness goes to the wave
            // above, its last row's TB plane (unchanged by this phase) to
            // the wave below.
            if (lane == 0) {
#pragma unroll
                for (int i = 0; i < W; ++i)
                    sh.x[p][wave][0][i] = ~(L0[i] | T0[i]);
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
            // Vertical phase: a TB car moves when the cell below is EMPTY
            // after the horizontal phase; it lands one row lower.  The
            // upper row's cars move into the lower row of the same lane;
            // the lower row's into the next lane's upper row, or, for the
            // item's last lane (63, or 15, 31 or 47 in a short last wave),
            // into the wave below.  The neighbour waves' rows are read four
            // words at a time, one group ahead of their use, so that LDS
            // latency hides behind the previous group.
            u32x4 nb = *reinterpret_cast<const u32x4 *>(xb);
            u32x4 na = *reinterpret_cast<const u32x4 *>(xa);
#pragma unroll
            for (int g = 0; g < W; g += 4) {
                const u32x4 cb = nb, ca = na;   // first row of the wave below, last row above
                if (g + 4 < W) {
                    nb = *reinterpret_cast<const u32x4 *>(xb + g + 4);
                    na = *reinterpret_cast<const u32x4 *>(xa + g + 4);
                }
                uint32_t e0[4], eb[4], mv0[4], mv1[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = g + j;
                    if (i < W) {
                        e0[j] = ~(L0[i] | T0[i]);
                        eb[j] = from_below_or(cb[j], e0[j]);
                        // The lane shift must run with every lane on: the
                        // compiler would otherwise turn the select into a
                        // branch around a shift with the last lane switched
                        // off, and a lane whose source lane is off keeps its
                        // old value.
                        asm volatile("" : "+v"(eb[j]));
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = g + j;
                    if (i < W) {
                        // The item's last row takes the row below it from
                        // LDS (a whole lattice's first row) where it does
                        // not sit in lane 63, i.e. when N is not a multiple
                        // of the 128 rows of a wave.  A slab's last held row
                        // is a halo row of its open lower end, whose error
                        // reaches the stored rows only after more than
                        // H >= n_steps steps: it may see the unused lane.
                        if constexpr (!SLAB && (32 * W) % RES_WAVE_ROWS != 0)
                            eb[j] = lane == last_lane ? cb[j] : eb[j];
                        mv0[j] = T0[i] & ~(L1[i] | T1[i]);
                        mv1[j] = T1[i] & eb[j];
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = g + j;
                    if (i < W) {
                        const uint32_t arrive = from_above_or(ca[j] & e0[j], mv1[j]);
                        T0[i] = xor3(T0[i], mv0[j], arrive);
                        T1[i] = xor3(T1[i], mv1[j], mv0[j]);
                        c_tb = __builtin_popcount(mv0[j]) + c_tb;
                        c_tb1 = __builtin_popcount(mv1[j]) + c_tb1;
                        asm("" : "+v"(c_tb), "+v"(c_tb1));
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = g + j;
                    if (i < W)
                        asm("" : "+v"(T0[i]), "+v"(T1[i]));
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            c_tb += c_tb1;
            const uint32_t tot = wave_total(counted ? (c_lr | (c_tb << 16)) : 0u);
            if (lane == 0) {
                const int kb = (s / RES_CHUNK) & 1, c = s % RES_CHUNK;
                atomicAdd(&sh.cnt[kb][c][slot][0], tot & 0xffffu);
                atomicAdd(&sh.cnt[kb][c][slot][1], tot >> 16);
            }
            // At the first step of a chunk the previous chunk's counts are
            // complete (every wave added them before this step's barrier),
            // and its slots are next used two chunks on.
            if (s >= RES_CHUNK && s % RES_CHUNK == 0 && wl == 0)
                flush(s - RES_CHUNK, s);
        }
    }
    __syncthreads();
    if (wave_on) {
        if (n_steps > 0 && wl == 0) {
            const int c0 = (n_steps - 1) / RES_CHUNK * RES_CHUNK;   // the last chunk
            flush(c0, n_steps);
        }
        if (counted) {
            store_row(g0, L0, T0);
            store_row(g1, L1, T1);
        }
    }
}

template <int IO, int W>
__device__ __forceinline__ void resident_dispatch(const ResidentArgs &a, const ResidentBin &bin,
                                                  ResidentShared &sh, int words, bool slab)
{
    if constexpr (W <= RES_MAX_WORDS) {
        if (words == W) {
            if (slab)
                resident_body<IO, W, true>(a, bin, sh);
            else
                resident_body<IO, W, false>(a, bin, sh);
        } else {
            resident_dispatch<IO, W + 1>(a, bin, sh, words, slab);
        }
    }
}

// One block per bin; blockDim.x == 64 * RES_WAVES.
template <int IO>
__global__ __launch_bounds__(64 * RES_WAVES, 3) void resident_kernel(ResidentArgs a)
{
    __shared__ ResidentShared sh;
    const ResidentBin &bin = a.bins[blockIdx.x];
    const int words = __builtin_amdgcn_readfirstlane(bin.words);
    if (__builtin_amdgcn_readfirstlane(bin.n_items) > 0)   // padding bins only take a ticket
        resident_dispatch<IO, 1>(a, bin, sh, words,
                                 __builtin_amdgcn_readfirstlane(bin.item[0].halo) > 0);

    // The last block to finish advances the device-side step and pass (one
    // pass: every lattice's state moved once between its two buffers).
    __shared__ uint32_t is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(&a.ctr->ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        is_last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (is_last && threadIdx.x == 0) {
        a.ctr->step = __builtin_amdgcn_readfirstlane(a.ctr->step) + (uint32_t)a.n_steps;
        a.ctr->pass = a.ctr->pass + 1u;
        __hip_atomic_store(&a.ctr->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

using ResidentFn = void (*)(ResidentArgs);
ResidentFn resident_kernel_u8();
ResidentFn resident_kernel_bp();

} // namespace bml
