// bml_batch.hpp -- batched BML step kernel: many lattices of different N
// (each a multiple of 32, at most 65504) advanced by one launch per pass.
//
// It is the streaming register pipeline of bml_pass.hpp (see there for the
// per-row algorithm), generalised in three ways:
//  * Work items come from a device-side list of (lattice, first strip,
//    column block); every lattice has its own descriptor (size, state
//    buffers, strip height).
//  * Narrow lattices (W = N/32 words per row, W <= 62) put several strips
//    into one wavefront: lanes form groups of W + 2 (a halo lane on each
//    side of W exact words), group g streaming strip first + g.  The DPP
//    lane shifts cross group borders, but only into halo lanes, whose
//    stale bits never reach the exact words within 31 steps.  Row offsets
//    then differ per group, so they are per-lane (VGPR) offsets.
//  * Everything that changes from pass to pass -- the global step, each
//    lattice's ping-pong parity and the active item list -- is read from
//    device memory, so a run of passes can be captured once in a hipGraph
//    and replayed.
// Per step and lattice the kernel adds the number of LR cars and TB cars
// that moved to a trace (the car counts themselves are conserved and are
// checked separately).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "bml_pass.hpp"
#include "bml_tile.hpp"

namespace bml {

struct BatchLattice {        // device descriptor of one lattice
    const void *buf[2];      // ping-pong state buffers
    int32_t n;               // side
    int32_t words;           // n / 32
    int32_t strip_rows;      // H: output rows per strip, divides n
    int32_t groups;          // strips per wavefront (lane groups)
    int32_t group_lanes;     // lanes per group (W + 2, or 64 when W > 62)
    int32_t parity_base;     // parity of the state when the lattice was activated
    int32_t pass_base;       // global pass count at that time
    int32_t pad;
};

struct BatchItem {
    int32_t lattice;
    int32_t strip0;          // strip of lane group 0
    int32_t tx;              // column block (only when words > 62)
    int32_t pad;
};

struct BatchCounters {       // device-side progress, advanced by the last block
    uint32_t step;           // global step of the next pass
    uint32_t pass;           // global pass count
    uint32_t n_items;        // active work items
    uint32_t ticket;         // last-block detection
};

struct BatchArgs {
    const BatchLattice *lat;
    const BatchItem *items;
    BatchCounters *ctr;
    uint32_t *trace;         // [lattice][trace_steps][2]: LR moved, TB moved
    int32_t trace_steps;
    int32_t k;               // steps in this pass (== template K)
    int32_t xcd_split;
};

using BatchFn = void (*)(BatchArgs);

template <int IO, int K>
__global__ __launch_bounds__(256) void batch_kernel(BatchArgs a)
{
    static_assert(K >= 1 && K <= MAX_K, "bad steps per pass");
    constexpr int D = IO == IO_U8 ? U8_RING : BP_RING;   // prefetched rows
    constexpr int NW = IO == IO_U8 ? 8 : 2;
    const int lane = threadIdx.x & 63;
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
    const uint32_t step0 = __builtin_amdgcn_readfirstlane(a.ctr->step);
    const uint32_t pass = __builtin_amdgcn_readfirstlane(a.ctr->pass);
    const int n_items = (int)__builtin_amdgcn_readfirstlane(a.ctr->n_items);

    for (int item = first; item < n_items; item += total_waves) {
        const BatchItem it = a.items[item];
        const int li = __builtin_amdgcn_readfirstlane(it.lattice);
        const BatchLattice &d = a.lat[li];
        const int n = __builtin_amdgcn_readfirstlane(d.n);
        const int words = __builtin_amdgcn_readfirstlane(d.words);
        const int H = __builtin_amdgcn_readfirstlane(d.strip_rows);
        const int GW = __builtin_amdgcn_readfirstlane(d.group_lanes);
        const int G = __builtin_amdgcn_readfirstlane(d.groups);
        const int par = (__builtin_amdgcn_readfirstlane(d.parity_base) +
                         (int)(pass - (uint32_t)__builtin_amdgcn_readfirstlane(d.pass_base))) & 1;
        const uint32_t row_bytes = IO == IO_U8 ? (uint32_t)n : (uint32_t)words * 4u;
        const uint32_t plane_bytes = row_bytes * (uint32_t)n;
        const uint32_t state_bytes = IO == IO_U8 ? plane_bytes : 2u * plane_bytes;
        const __amdgpu_buffer_rsrc_t src = make_rsrc(d.buf[par], state_bytes);
        const __amdgpu_buffer_rsrc_t dst = make_rsrc(d.buf[par ^ 1], state_bytes);

        const int g = lane / GW;                  // lane group
        const int j = lane - g * GW;              // lane within the group
        const int strip = it.strip0 + g;
        const int row_a = strip * H;
        const int w0 = it.tx * TILE_WORDS;
        const int vwords = min(GW - 2, words - w0);
        const uint32_t word = (uint32_t)((w0 + j - 1 + words) % words);
        const bool lane_ok = g < G && row_a < n && j >= 1 && j <= vwords;
        const uint32_t voff = IO == IO_U8 ? word * 32u : word * 4u;
        const int h = H;                          // every strip is full (H divides n)
        const int total_in = h + 2 * K;
        const int total_it = h + 3 * K - 1;

        // Per-lane row offsets (groups stream different strips).
        uint32_t ld_off = (uint32_t)(((row_a % n) - K + n) % n) * row_bytes;
        uint32_t st_off = (uint32_t)(row_a < n ? row_a : 0) * row_bytes;
        auto advance = [&](uint32_t o) {
            const uint32_t x = o + row_bytes;
            return x >= plane_bytes ? x - plane_bytes : x;
        };
        uint32_t ring[D][NW];
        auto issue = [&](uint32_t (&dstw)[NW], uint32_t off) {
            if constexpr (IO == IO_U8) {
                const u32x4 u0 = __builtin_amdgcn_raw_buffer_load_b128(src, voff + off, 0, 0);
                const u32x4 u1 =
                    __builtin_amdgcn_raw_buffer_load_b128(src, voff + off + 16, 0, 0);
                dstw[0] = u0.x; dstw[1] = u0.y; dstw[2] = u0.z; dstw[3] = u0.w;
                dstw[4] = u1.x; dstw[5] = u1.y; dstw[6] = u1.z; dstw[7] = u1.w;
            } else {
                dstw[0] = __builtin_amdgcn_raw_buffer_load_b32(src, voff + off, 0, 0);
                dstw[1] = __builtin_amdgcn_raw_buffer_load_b32(src, voff + off, plane_bytes, 0);
            }
        };
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            if (dd < total_in) {
                issue(ring[dd], ld_off);
                ld_off = advance(ld_off);
            }
        }

        Level<1> lv[K];
        uint32_t bl[K][1], bt[K][1];
        uint32_t acc[K][2];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            lv[k].L[0] = lv[k].T[0] = lv[k].mvp[0] = 0;
            bl[k][0] = bt[k][0] = 0;
            acc[k][0] = acc[k][1] = 0;
        }

        auto body = [&](int t0, auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
            for (int dd = 0; dd < D; ++dd) {
                const int t = t0 + dd;
                if (!FULL && t >= total_it)
                    break;
                uint32_t L0[1] = {0}, T0[1] = {0};
                if (FULL || t < total_in) {
                    if constexpr (IO == IO_U8) {
                        bytes_to_planes(ring[dd], L0[0], T0[0]);
                        asm("" : "+v"(L0[0]), "+v"(T0[0]));
                    } else {
                        L0[0] = ring[dd][0];
                        T0[0] = ring[dd][1];
                    }
                    if (FULL || t + D < total_in) {
                        issue(ring[dd], ld_off);
                        ld_off = advance(ld_off);
                    }
                }
#pragma unroll
                for (int k = K - 1; k >= 0; --k) {
                    if (!FULL && (t < 3 * k || t > h + 2 * K - 1 + k))
                        continue;   // level idle in the prologue / drain
                    const LevelOut<1> o =
                        level_push<1, false>(lv[k], k ? bl[k - 1] : L0, k ? bt[k - 1] : T0);
                    const int rh = t - 2 * k - K;
                    if (FULL || (rh >= 0 && rh < h))
                        acc[k][0] += __builtin_popcount(o.mv_h[0]);
                    if (FULL || (rh >= 1 && rh <= h))
                        acc[k][1] += __builtin_popcount(o.mv_v[0]);
                    asm("" : "+v"(acc[k][0]), "+v"(acc[k][1]));
                    bl[k][0] = o.L[0];
                    bt[k][0] = o.T[0];
                }
                if (FULL || (t >= 3 * K - 1 && t < 3 * K - 1 + h)) {
                    if (lane_ok) {
                        if constexpr (IO == IO_U8) {
                            uint32_t b[8];
                            planes_to_bytes(bl[K - 1][0], bt[K - 1][0], b);
                            __builtin_amdgcn_raw_buffer_store_b128(
                                (u32x4){b[0], b[1], b[2], b[3]}, dst, voff + st_off, 0, 0);
                            __builtin_amdgcn_raw_buffer_store_b128(
                                (u32x4){b[4], b[5], b[6], b[7]}, dst, voff + st_off + 16, 0, 0);
                        } else {
                            __builtin_amdgcn_raw_buffer_store_b32(bl[K - 1][0], dst, voff + st_off,
                                                                  0, 0);
                            __builtin_amdgcn_raw_buffer_store_b32(bt[K - 1][0], dst, voff + st_off,
                                                                  plane_bytes, 0);
                        }
                    }
                    st_off += row_bytes;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        for (int t0 = 0; t0 < total_it; t0 += D) {
            if (t0 >= 3 * K - 1 && t0 + D <= h + K && t0 + 2 * D <= total_in)
                body(t0, std::true_type{});
            else
                body(t0, std::false_type{});
        }

        // Moved counts of this item, one trace entry per step (all groups
        // of an item belong to the same lattice).
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t v = wave_total(lane_ok ? acc[k][q] : 0u);
                const uint32_t s = step0 + (uint32_t)k;
                if (lane == 0 && v && s < (uint32_t)a.trace_steps)
                    atomicAdd(&a.trace[((size_t)li * a.trace_steps + s) * 2 + q], v);
            }
        }
    }

    // The last block to finish advances the device-side step and pass.  By
    // then every block has read them (each reads them first and takes its
    // ticket last); the next launch sees the new values after the kernel
    // boundary.  Only the ticket is shared during the launch, through a
    // device-scope atomic, so no device-wide fence is needed.
    __shared__ uint32_t is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(&a.ctr->ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        is_last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (is_last && threadIdx.x == 0) {
        a.ctr->step = step0 + (uint32_t)K;
        a.ctr->pass = pass + 1u;
        __hip_atomic_store(&a.ctr->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int IO, int KLO, int... Ks>
inline void fill_batch_table(BatchFn *tab, std::integer_sequence<int, Ks...>)
{
    ((tab[KLO + Ks] = batch_kernel<IO, KLO + Ks>), ...);
}

void batch_table_u8(BatchFn *tab);   // K = 1..MAX_K
void batch_table_bp(BatchFn *tab);

} // namespace bml
