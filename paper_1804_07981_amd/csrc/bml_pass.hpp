// bml_pass.hpp -- the temporally blocked BML step kernel (gfx950).
//
// One wavefront holds a tile of R = VR + 2K lattice rows x 64 words (2048
// cells) in VGPRs as two bitplanes and advances it K steps (2K phases)
// before writing its VR middle rows back, so each HBM pass costs one read
// and one write of the state for K steps (temporal blocking).  Neighbours across the tile edge come from a
// periodic halo: K rows above and below and one word on each side (lanes 0
// and 63), addressed modulo N, so no ghost cells are ever stored (the ghost
// cells of Marzolla, arXiv:1804.07981, Sec. 3, become modular addressing of
// the halo).  Each phase invalidates one more halo row on each side
// (vertical) and one more bit in lanes 0 and 63 (horizontal), so the VR
// middle rows of lanes 1..62 are exact after K steps; only those are written
// and counted.  VR is 32 or 64 and divides N, so every tile row is full.
//
// Memory access: buffer loads/stores with the per-lane word offset in a VGPR
// and the row offset in an SGPR, so an in-flight row costs no address
// registers.  Byte lattices are read 32 bytes per lane (two dwordx4) in
// chunks of rows, one chunk in flight while the previous one is packed into
// bitplanes; bitplane lattices are read straight into the tile registers.
//
// Grids are persistent: every wavefront walks a strided list of tiles.
// Blocks are dispatched round-robin over the 8 XCDs, so block b is mapped to
// the (b % 8)-th eighth of every round of tiles: each XCD works on a band of
// vertically adjacent tiles, which share halo rows in that XCD's L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "bml_tile.hpp"

namespace bml {

enum { IO_U8 = 0, IO_BP = 1 };
constexpr int MAX_K = 8;        // steps per pass
constexpr int TILE_WORDS = 62;  // output words per wavefront tile (lanes 1..62)

constexpr int ACC_STRIPES = 8;  // one stats accumulator stripe per XCD

// Library-owned scratch of the stats reduction; all zero between launches.
struct PassScratch {
    uint32_t acc[ACC_STRIPES][MAX_K][4];
    uint32_t ticket;
};

struct PassArgs {
    const void *src;
    void *dst;
    uint32_t *stats;         // caller's ring, 4 u32 per slot
    PassScratch *scratch;
    int32_t n;               // lattice side
    int32_t words;           // n / 32
    int32_t tiles_x;         // tiles across a row
    int32_t n_tiles;         // tiles_x * (n / VR)
    int32_t xcd_split;       // 1: gridDim.x % 8 == 0, give each XCD a band of tiles
    uint32_t rec_mask;       // bit k set: record the counts of step k of this pass
    int32_t slot[MAX_K];     // ring slot of step k
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

__device__ __forceinline__ void wave_reduce_to_lds(uint32_t v, uint32_t *dst)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += (uint32_t)__shfl_xor((int)v, off, 64);
    if ((threadIdx.x & 63) == 0 && v)
        atomicAdd(dst, v);
}

template <int IO, int K, int VR>
__global__ __launch_bounds__(256) void pass_kernel(PassArgs a)
{
    static_assert(K >= 1 && K <= MAX_K, "bad steps per pass");
    constexpr int R = VR + 2 * K;   // tile rows held in registers, halo included
    constexpr int CH = 4;           // rows per load chunk (byte lattices)
    constexpr int NCH = (R + CH - 1) / CH;
    const int lane = threadIdx.x & 63;
    // Wave-uniform values must be visibly uniform so that tile and row
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
    const uint32_t row_bytes = IO == IO_U8 ? (uint32_t)a.n : (uint32_t)a.words * 4u;
    const uint32_t plane_bytes = row_bytes * (uint32_t)a.n;   // lattice bytes (one plane)
    const uint32_t state_bytes = IO == IO_U8 ? plane_bytes : 2u * plane_bytes;
    const __amdgpu_buffer_rsrc_t src = make_rsrc(a.src, state_bytes);
    const __amdgpu_buffer_rsrc_t dst = make_rsrc(a.dst, state_bytes);

    uint32_t acc[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
        acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0;

    for (int t = first; t < a.n_tiles; t += total_waves) {
        const int ty = t / a.tiles_x;
        const int tx = t - ty * a.tiles_x;
        const int w0 = tx * TILE_WORDS;
        const int vwords = min(TILE_WORDS, a.words - w0);
        const uint32_t word = (uint32_t)((w0 + lane - 1 + a.words) % a.words);
        const uint32_t lane_ok = (lane >= 1 && lane <= vwords) ? 1u : 0u;
        const uint32_t voff = IO == IO_U8 ? word * 32u : word * 4u;
        // Byte offset of tile row 0 (lattice row ty*VR - K, periodic); later
        // rows follow with a wrap at the end of the lattice.
        const uint32_t roff0 = (uint32_t)((ty * VR - K + a.n) % a.n) * row_bytes;
        auto roff = [&](int r) {
            // 64-bit: for N near 65504 a byte lattice is close to 2^32 bytes.
            // A tile has at most VR + 2*MAX_K = 80 rows and N >= 32, so the
            // row index wraps at most three times.
            uint64_t o = (uint64_t)roff0 + (uint64_t)r * row_bytes;
            static_assert(VR + 2 * MAX_K <= 3 * 32, "row wrap needs more steps");
#pragma unroll
            for (int w = 0; w < 3; ++w)
                o = o >= plane_bytes ? o - plane_bytes : o;
            return (uint32_t)o;
        };

        uint32_t L[R], T[R];
        if (IO == IO_U8) {
            u32x4 buf[2][CH][2];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                buf[0][i][0] = __builtin_amdgcn_raw_buffer_load_b128(src, voff, roff(i), 0);
                buf[0][i][1] = __builtin_amdgcn_raw_buffer_load_b128(src, voff + 16, roff(i), 0);
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (c + 1 < NCH) {
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        const int r = (c + 1) * CH + i;
                        if (r < R) {
                            buf[(c + 1) & 1][i][0] =
                                __builtin_amdgcn_raw_buffer_load_b128(src, voff, roff(r), 0);
                            buf[(c + 1) & 1][i][1] =
                                __builtin_amdgcn_raw_buffer_load_b128(src, voff + 16, roff(r), 0);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    if (c * CH + i < R) {
                        const u32x4 u0 = buf[c & 1][i][0], u1 = buf[c & 1][i][1];
                        const uint32_t d[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
                        bytes_to_planes(d, L[c * CH + i], T[c * CH + i]);
                        // Materialise the planes: otherwise the last swap of
                        // the bit transpose is folded into every consumer and
                        // each plane occupies two registers.
                        asm("" : "+v"(L[c * CH + i]), "+v"(T[c * CH + i]));
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                L[r] = __builtin_amdgcn_raw_buffer_load_b32(src, voff, roff(r), 0);
                T[r] = __builtin_amdgcn_raw_buffer_load_b32(src, voff, roff(r) + plane_bytes, 0);
            }
        }

        // Step k updates rows [k, R-k) in the H phase (all still exact) and
        // rows [k+1, R-k-1) in the V phase; rows [K, K+VR) are counted.
        [&]<int... ks>(std::integer_sequence<int, ks...>) {
            (([&] {
                 uint32_t mlr = 0, nlr = 0, mtb = 0, ntb = 0;
                 __builtin_amdgcn_sched_barrier(0);
                 h_phase<R, ks, R - ks, K, K + VR>(L, T, mlr, nlr);
                 __builtin_amdgcn_sched_barrier(0);
                 v_phase<R, ks, R - ks, K, K + VR>(L, T, mtb, ntb);
                 __builtin_amdgcn_sched_barrier(0);
                 acc[ks][0] += lane_ok * nlr;
                 acc[ks][1] += lane_ok * mlr;
                 acc[ks][2] += lane_ok * ntb;
                 acc[ks][3] += lane_ok * mtb;
             }()),
             ...);
        }(std::make_integer_sequence<int, K>{});

        if (lane_ok) {
            const uint32_t out0 = (uint32_t)(ty * VR) * row_bytes;
#pragma unroll
            for (int r = K; r < K + VR; ++r) {
                const uint32_t ro = out0 + (uint32_t)(r - K) * row_bytes;
                if (IO == IO_U8) {
                    uint32_t d[8];
                    planes_to_bytes(L[r], T[r], d);
                    __builtin_amdgcn_raw_buffer_store_b128((u32x4){d[0], d[1], d[2], d[3]}, dst,
                                                           voff, ro, 0);
                    __builtin_amdgcn_raw_buffer_store_b128((u32x4){d[4], d[5], d[6], d[7]}, dst,
                                                           voff + 16, ro, 0);
                    if ((r - K) % 2 == 1)
                        __builtin_amdgcn_sched_barrier(0);
                } else {
                    __builtin_amdgcn_raw_buffer_store_b32(L[r], dst, voff, ro, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(T[r], dst, voff, ro + plane_bytes, 0);
                }
            }
        }
    }

    // Counts: wave -> block (LDS) -> one of 8 device-wide stripes (block b
    // adds to stripe b % 8) -> the last block to finish sums the stripes,
    // writes the ring slots and clears the scratch for the next launch.
    if (a.rec_mask == 0)
        return;
    __shared__ uint32_t red[MAX_K * 4];
    __shared__ uint32_t is_last;
    if (threadIdx.x < MAX_K * 4)
        red[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            wave_reduce_to_lds(acc[k][q], &red[k * 4 + q]);
    __syncthreads();
    uint32_t *stripe = &a.scratch->acc[blockIdx.x % ACC_STRIPES][0][0];
    if (threadIdx.x < K * 4 && red[threadIdx.x])
        __hip_atomic_fetch_add(&stripe[threadIdx.x], red[threadIdx.x], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(&a.scratch->ticket, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        is_last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!is_last)
        return;
    if (threadIdx.x < K * 4) {
        const int k = threadIdx.x >> 2, q = threadIdx.x & 3;
        uint32_t sum = 0;
#pragma unroll
        for (int st = 0; st < ACC_STRIPES; ++st) {
            uint32_t *p = &a.scratch->acc[st][k][q];
            sum += __hip_atomic_exchange(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if ((a.rec_mask >> k) & 1u)
            a.stats[(size_t)a.slot[k] * 4 + q] = sum;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(&a.scratch->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fills tab[k] (k = 1..MAX_K) with pass_kernel<IO, k, VR>.
template <int IO, int VR, int... Ks>
inline void fill_pass_table(PassFn *tab, std::integer_sequence<int, Ks...>)
{
    ((tab[Ks + 1] = pass_kernel<IO, Ks + 1, VR>), ...);
}

// Defined in one translation unit per (layout, output rows per tile).
void pass_table_u8_r32(PassFn *tab);
void pass_table_u8_r64(PassFn *tab);
void pass_table_bp_r32(PassFn *tab);
void pass_table_bp_r64(PassFn *tab);

} // namespace bml
