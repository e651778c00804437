// bml_resident.hpp -- register-resident batched BML kernel (gfx950): every
// lattice of a batch with N <= 1024 stays in VGPRs for a whole run of many
// steps, in one launch.
//
// Layout: one row per lane.  Lane l of wave w of a lattice holds row
// 64 w + l as W = N / 32 LR words and W TB words (bit b of word i = cell
// 32 i + b), so the horizontal phase (Marzolla, arXiv:1804.07981, Sec. 2
// case table for LR cars) is entirely inside the lane: a ring of W words,
// periodic in x with no halo.  The vertical phase needs the rows above and
// below, which are the neighbouring lanes (DPP wave shifts); the rows
// across a wave boundary (and across the periodic top/bottom edge) come
// from the neighbouring wave through LDS.  One barrier per step separates
// the exchange writes (after the horizontal phase) from the reads; the
// exchange slots alternate between two buffers by step parity, so a wave
// can never overwrite a slot a slower wave has yet to read.  Both phases
// read only the state before the phase (the synchronous rule of Sec. 3):
// the horizontal phase decides every move from the words before any of
// them changes, and the vertical phase from the post-horizontal occupancy.
//
// A block (16 waves) holds a bin of lattices of one size: as many as fit,
// ceil(W / 2) waves each.  Per step and lattice the moved counts of the
// two phases are summed (wave total, then LDS) and stored in the trace.
// The state is read from HBM once at the start of the run and written once
// at the end: the step loop itself touches only VGPRs and LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bml_batch.hpp"
#include "bml_tile.hpp"

namespace bml {

constexpr int RES_MAX_WORDS = 32;   // N <= 1024
constexpr int RES_WAVES = 16;       // waves per block
constexpr int RES_MAX_LAT = 16;     // lattices per block (N <= 64: one wave each)
constexpr int RES_GROUP = 4;        // words per scheduling group of the step loop

// Lattices of one size run by one block.
struct ResidentBin {
    int32_t words;                  // W = N / 32 of every lattice in the bin
    int32_t n_lat;                  // lattices in the bin
    int32_t lat[RES_MAX_LAT];       // batch indices
};

struct ResidentArgs {
    const BatchLattice *lat;
    const ResidentBin *bins;
    BatchCounters *ctr;
    uint32_t *trace;                // [lattice][trace_steps][2]: LR moved, TB moved
    int32_t trace_steps;
    int32_t n_steps;                // steps of this launch
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
// after the horizontal phase, 1: TB plane of its last row][word].
struct ResidentShared {
    uint32_t x[2][RES_WAVES][2][RES_MAX_WORDS];
    uint32_t cnt[2][RES_MAX_LAT][2];     // [step parity][lattice][LR, TB moved]
};

template <int IO, int W>
__device__ __forceinline__ void resident_body(const ResidentArgs &a, const ResidentBin &bin,
                                              ResidentShared &sh)
{
    constexpr int WPL = (W + 1) / 2;     // waves per lattice: 32 W rows, 64 per wave
    constexpr int N = 32 * W;
    constexpr bool HALF = (W & 1) != 0;  // the last wave of a lattice holds 32 rows
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_lat = __builtin_amdgcn_readfirstlane(bin.n_lat);
    const int slot = wave / WPL;                 // lattice of this wave within the bin
    const int wl = wave - slot * WPL;            // wave within its lattice
    const bool wave_on = slot < n_lat;
    const int row = wl * 64 + lane;
    const bool row_ok = wave_on && row < N;
    const bool tail = HALF && wl == WPL - 1;     // lanes 0..31 only
    const int wdown = slot * WPL + (wl + 1 == WPL ? 0 : wl + 1);   // wave below (wrapping)
    const int wup = slot * WPL + (wl == 0 ? WPL - 1 : wl - 1);     // wave above
    const int last_lane = tail ? 31 : 63;
    const uint32_t step0 = __builtin_amdgcn_readfirstlane(a.ctr->step);
    const uint32_t pass = __builtin_amdgcn_readfirstlane(a.ctr->pass);
    const int n_steps = a.n_steps;

    int li = 0;
    uint8_t *dst = nullptr;
    uint32_t L[W], T[W];
#pragma unroll
    for (int i = 0; i < W; ++i)
        L[i] = T[i] = 0;
    if (wave_on) {
        li = __builtin_amdgcn_readfirstlane(bin.lat[slot]);
        const BatchLattice &d = a.lat[li];
        const int par = (__builtin_amdgcn_readfirstlane(d.parity_base) +
                         (int)(pass - (uint32_t)__builtin_amdgcn_readfirstlane(d.pass_base))) & 1;
        const uint8_t *src = (const uint8_t *)d.buf[par];
        dst = (uint8_t *)d.buf[par ^ 1];
        if (row_ok) {
            if constexpr (IO == IO_U8) {
                const uint4 *p = (const uint4 *)(src + (size_t)row * N);
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const uint4 u0 = p[2 * i], u1 = p[2 * i + 1];
                    const uint32_t dw[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
                    bytes_to_planes(dw, L[i], T[i]);
                }
            } else {
                const uint32_t *pl = (const uint32_t *)src + (size_t)row * W;
                const uint32_t *pt = pl + (size_t)N * W;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    L[i] = pl[i];
                    T[i] = pt[i];
                }
            }
        }
    }

    // The count slots are first added to after the first step's barrier.
    static_assert(2 * RES_MAX_LAT * 2 <= 64, "one wave clears the count slots");
    if (threadIdx.x < 2 * RES_MAX_LAT * 2)
        (&sh.cnt[0][0][0])[threadIdx.x] = 0;

    for (int s = 0; s < n_steps; ++s) {
        const int p = s & 1;
        // Emptiness after the horizontal phase, kept per word while the
        // VGPRs allow it (the 128 of a 16-wave block hold 3 W words and the
        // rest up to W = 28); the widest rows recompute it where it is used.
        constexpr bool KEEP_E = W <= 28;
        uint32_t E[KEEP_E ? W : 1];
        auto empty = [&](int i) { return KEEP_E ? E[i] : ~(L[i] | T[i]); };
        uint32_t c_lr = 0, c_tb = 0;
        if (wave_on) {
            // Horizontal phase: an LR car moves when the next cell (bit
            // j + 1, continued into the next word, word W-1 wrapping to
            // word 0) is EMPTY; it lands one cell further.  Every mover is
            // decided before any word changes.
            // Words are processed in groups of RES_GROUP with scheduling
            // barriers between groups, so that only a group's temporaries
            // are live next to the state (the compiler would otherwise
            // compute every word's movers first and run out of VGPRs).
            const uint32_t o0 = L[0] | T[0];
            const uint32_t mv_last =
                L[W - 1] & ~__builtin_amdgcn_alignbit(o0, L[W - 1] | T[W - 1], 1);
            uint32_t mv_prev = mv_last, o = o0;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                uint32_t mv;
                if (i + 1 < W) {
                    const uint32_t on = L[i + 1] | T[i + 1];
                    mv = L[i] & ~__builtin_amdgcn_alignbit(on, o, 1);
                    o = on;
                } else {
                    mv = mv_last;
                }
                const uint32_t arrive = __builtin_amdgcn_alignbit(mv, mv_prev, 31);
                c_lr += __builtin_popcount(mv);
                L[i] = L[i] ^ mv ^ arrive;    // movers leave, arrivals land (disjoint)
                // Opaque new values: updated in place here, not carried as
                // pieces to the end of the step.
                if constexpr (KEEP_E) {
                    E[i] = ~(L[i] | T[i]);
                    asm("" : "+v"(L[i]), "+v"(E[i]));
                } else {
                    asm("" : "+v"(L[i]));
                }
                mv_prev = mv;
                if ((i + 1) % RES_GROUP == 0)
                    __builtin_amdgcn_sched_barrier(0);
            }
            // Exchange: the first row's emptiness goes to the wave above,
            // the last row's TB plane (unchanged by this phase) to the
            // wave below.
            if (lane == 0) {
#pragma unroll
                for (int i = 0; i < W; ++i)
                    sh.x[p][wave][0][i] = empty(i);
            }
            if (lane == last_lane) {
#pragma unroll
                for (int i = 0; i < W; ++i)
                    sh.x[p][wave][1][i] = T[i];
            }
        }
        __syncthreads();
        if (wave_on) {
            // Vertical phase: a TB car moves when the cell below is EMPTY
            // after the horizontal phase; it lands one row lower.
            auto vphase = [&](auto tail_tag) {
                constexpr bool TAIL = decltype(tail_tag)::value;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const uint32_t e_x = sh.x[p][wdown][0][i];   // first row of the wave below
                    const uint32_t t_x = sh.x[p][wup][1][i];     // last row of the wave above
                    const uint32_t e = empty(i);
                    uint32_t e_below = from_below_or(e_x, e);
                    if constexpr (TAIL) {
                        // Lane 31 holds the last row.  The lane shift must
                        // run with every lane on: the compiler would
                        // otherwise turn the select into a branch around a
                        // shift with lane 31 switched off, and a lane whose
                        // source lane is off keeps its old value (lane 30
                        // would see the wrong row below).
                        asm volatile("" : "+v"(e_below));
                        e_below = lane == 31 ? e_x : e_below;
                    }
                    const uint32_t mvt = T[i] & e_below;
                    const uint32_t arrive = from_above_or(t_x & e, mvt);
                    c_tb += __builtin_popcount(mvt);
                    T[i] = T[i] ^ mvt ^ arrive;
                    asm("" : "+v"(T[i]));
                    if ((i + 1) % RES_GROUP == 0)
                        __builtin_amdgcn_sched_barrier(0);
                }
            };
            if (HALF && tail)
                vphase(std::true_type{});
            else
                vphase(std::false_type{});
            const uint32_t tot = wave_total(row_ok ? (c_lr | (c_tb << 16)) : 0u);
            if (lane == 0) {
                atomicAdd(&sh.cnt[p][slot][0], tot & 0xffffu);
                atomicAdd(&sh.cnt[p][slot][1], tot >> 16);
            }
            // The counts of step s-1 are complete: every wave added them
            // before this step's barrier.
            if (s > 0 && wl == 0 && lane == 0) {
                const uint32_t gs = step0 + (uint32_t)(s - 1);
                if (gs < (uint32_t)a.trace_steps) {
                    uint32_t *tr = a.trace + ((size_t)li * a.trace_steps + gs) * 2;
                    tr[0] = sh.cnt[p ^ 1][slot][0];
                    tr[1] = sh.cnt[p ^ 1][slot][1];
                }
                sh.cnt[p ^ 1][slot][0] = 0;
                sh.cnt[p ^ 1][slot][1] = 0;
            }
        }
    }
    __syncthreads();
    if (wave_on) {
        if (n_steps > 0 && wl == 0 && lane == 0) {
            const int p = (n_steps - 1) & 1;
            const uint32_t gs = step0 + (uint32_t)(n_steps - 1);
            if (gs < (uint32_t)a.trace_steps) {
                uint32_t *tr = a.trace + ((size_t)li * a.trace_steps + gs) * 2;
                tr[0] = sh.cnt[p][slot][0];
                tr[1] = sh.cnt[p][slot][1];
            }
        }
        if (row_ok) {
            if constexpr (IO == IO_U8) {
                uint4 *q = (uint4 *)(dst + (size_t)row * N);
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    uint32_t b[8];
                    planes_to_bytes(L[i], T[i], b);
                    q[2 * i] = make_uint4(b[0], b[1], b[2], b[3]);
                    q[2 * i + 1] = make_uint4(b[4], b[5], b[6], b[7]);
                }
            } else {
                uint32_t *pl = (uint32_t *)dst + (size_t)row * W;
                uint32_t *pt = pl + (size_t)N * W;
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    pl[i] = L[i];
                    pt[i] = T[i];
                }
            }
        }
    }
}

template <int IO, int W>
__device__ __forceinline__ void resident_dispatch(const ResidentArgs &a, const ResidentBin &bin,
                                                  ResidentShared &sh, int words)
{
    if constexpr (W <= RES_MAX_WORDS) {
        if (words == W)
            resident_body<IO, W>(a, bin, sh);
        else
            resident_dispatch<IO, W + 1>(a, bin, sh, words);
    }
}

// One block per bin; blockDim.x == 64 * RES_WAVES.
template <int IO>
__global__ __launch_bounds__(64 * RES_WAVES) void resident_kernel(ResidentArgs a)
{
    __shared__ ResidentShared sh;
    const ResidentBin &bin = a.bins[blockIdx.x];
    const int words = __builtin_amdgcn_readfirstlane(bin.words);
    if (__builtin_amdgcn_readfirstlane(bin.n_lat) > 0)   // padding bins only take a ticket
        resident_dispatch<IO, 1>(a, bin, sh, words);

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
void resident_kernels(ResidentFn *u8, ResidentFn *bp);

} // namespace bml
