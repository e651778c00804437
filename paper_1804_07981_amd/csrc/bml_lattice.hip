// bml_lattice.hip -- single-lattice BML step on gfx950: initial placement,
// byte/bitplane conversion, car counting and the temporally blocked step
// kernels, plus the host side of the single-lattice C ABI (include/bml.h).
//
// Model: Marzolla, arXiv:1804.07981, Sec. 2 (periodic N x N lattice, H phase
// then V phase, case tables) and Sec. 3 (synchronous update through two
// grids, row-major layout, one byte per cell; two bits would suffice).
//
// The step kernel itself (temporal blocking over register tiles) is in
// bml_pass.hpp, instantiated in bml_pass_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "bml.h"
#include "bml_block.hpp"
#include "bml_common.hpp"
#include "bml_pass.hpp"
#include "bml_tile.hpp"

namespace bml {

// ============================================================================
// Errors and device properties
// ============================================================================

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

int device_info(DeviceInfo *out)
{
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    BML_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev)
        cache.resize(dev + 1);
    if (cache[dev].device < 0) {
        hipDeviceProp_t p;
        BML_HIP(hipGetDeviceProperties(&p, dev));
        cache[dev].device = dev;
        cache[dev].cu_count = p.multiProcessorCount;
    }
    *out = cache[dev];
    return BML_OK;
}

// ============================================================================
// Kernels
// ============================================================================

// SplitMix64 (Steele, Lea & Flood 2014): k-th output of the stream whose
// state starts at `seed`.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One thread per 32-cell word: cells k0 .. k0+31 of row-major index.
template <int IO>
__global__ __launch_bounds__(256) void init_kernel(void *out, int32_t n, int32_t words,
                                                   uint64_t seed, uint64_t thr_lr,
                                                   uint64_t thr_tb)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n * words;
    if (idx >= total)
        return;
    const uint64_t k0 = (uint64_t)idx * 32u;   // row*n + 32*w == 32*(row*words + w)
    uint32_t lr = 0, tb = 0;
#pragma unroll 4
    for (int j = 0; j < 32; ++j) {
        const uint64_t u = splitmix64_at(seed, k0 + j) >> 11;
        lr |= (uint32_t)(u < thr_lr) << j;
        tb |= (uint32_t)(u >= thr_lr && u < thr_tb) << j;
    }
    if (IO == IO_U8) {
        uint32_t d[8];
        planes_to_bytes(lr, tb, d);
        uint4 *p = (uint4 *)((uint8_t *)out + k0);
        p[0] = make_uint4(d[0], d[1], d[2], d[3]);
        p[1] = make_uint4(d[4], d[5], d[6], d[7]);
    } else {
        uint32_t *pl = (uint32_t *)out;
        pl[idx] = lr;
        pl[total + idx] = tb;
    }
}

// Byte cells -> bitplanes, one thread per word: cells 32 idx .. 32 idx + 31
// become word idx of the LR plane `lr` and of the TB plane `tb`.
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *cells, uint32_t *lr_out,
                                                   uint32_t *tb_out, int64_t total_words)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total_words)
        return;
    const uint4 *p = (const uint4 *)(cells + idx * 32);
    const uint4 u0 = p[0], u1 = p[1];
    const uint32_t d[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
    uint32_t lr, tb;
    bytes_to_planes(d, lr, tb);
    lr_out[idx] = lr;
    tb_out[idx] = tb;
}

// Bitplanes -> byte cells, one thread per word: word idx of the LR plane
// `lr` and of the TB plane `tb` become cells 32 idx .. 32 idx + 31.
__global__ __launch_bounds__(256) void unpack_kernel(const uint32_t *lr, const uint32_t *tb,
                                                     uint8_t *cells, int64_t total_words)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total_words)
        return;
    uint32_t d[8];
    planes_to_bytes(lr[idx], tb[idx], d);
    uint4 *p = (uint4 *)(cells + idx * 32);
    p[0] = make_uint4(d[0], d[1], d[2], d[3]);
    p[1] = make_uint4(d[4], d[5], d[6], d[7]);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += (uint32_t)__shfl_xor((int)v, off, 64);
    return v;
}

// Counts LR and TB cells; out[0] += LR, out[1] += TB.  One thread per word.
template <int IO>
__global__ __launch_bounds__(256) void count_kernel(const void *state, int64_t total_words,
                                                    unsigned long long *out)
{
    __shared__ uint32_t s[2];
    if (threadIdx.x < 2)
        s[threadIdx.x] = 0;
    __syncthreads();
    uint32_t lr = 0, tb = 0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total_words;
         idx += (int64_t)gridDim.x * blockDim.x) {
        if (IO == IO_U8) {
            const uint4 *p = (const uint4 *)((const uint8_t *)state + idx * 32);
            const uint4 u0 = p[0], u1 = p[1];
            const uint32_t d[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                lr += __builtin_popcount(d[q] & 0x01010101u);
                tb += __builtin_popcount(d[q] & 0x02020202u);
            }
        } else {
            const uint32_t *pl = (const uint32_t *)state;
            lr += __builtin_popcount(pl[idx]);
            tb += __builtin_popcount(pl[total_words + idx]);
        }
    }
    lr = wave_sum(lr);
    tb = wave_sum(tb);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&s[0], lr);
        atomicAdd(&s[1], tb);
    }
    __syncthreads();
    if (threadIdx.x < 2)
        atomicAdd(&out[threadIdx.x], (unsigned long long)s[threadIdx.x]);
}

__global__ void zero_words_kernel(uint32_t *p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ============================================================================
// Kernel table
// ============================================================================

// fn[mode][io][k]: mode 0 = tile mode (any N), mode m = 1, 2 = row mode
// for N = 2048 m (the wavefront holds a whole row, m words per lane).
constexpr int PASS_MODES = 3;

// Kernel kinds: the model of Sec. 2 on the torus or the Klein bottle, and
// Model II on the torus.
enum { KIND_TORUS = 0, KIND_KLEIN = 1, KIND_MODEL2 = 2, KIND_MODEL3 = 3, PASS_KINDS = 4 };

struct KernelTable {
    PassFn fn[PASS_KINDS][PASS_MODES][2][MAX_K + 1] = {};   // [kind][mode][io][k]
    KernelTable()
    {
#define BML_FILL(io, range, kind, KIND, MODE, IO) pass_table_##io##_##range##_##kind(fn[KIND][MODE][IO]);
#define BML_FILL_KIND(kind, KIND)                                                          \
    BML_FILL(u8, lo, kind, KIND, 0, IO_U8) BML_FILL(u8, hi, kind, KIND, 0, IO_U8)             \
    BML_FILL(bp, lo, kind, KIND, 0, IO_BP) BML_FILL(bp, hi, kind, KIND, 0, IO_BP)             \
    BML_FILL(u8, row1, kind, KIND, 1, IO_U8) BML_FILL(bp, row1, kind, KIND, 1, IO_BP)         \
    BML_FILL(u8, row2, kind, KIND, 2, IO_U8) BML_FILL(bp, row2, kind, KIND, 2, IO_BP)
        BML_FILL_KIND(torus, KIND_TORUS)
        BML_FILL_KIND(klein, KIND_KLEIN)
        BML_FILL_KIND(model2, KIND_MODEL2)
        BML_FILL_KIND(model3, KIND_MODEL3)
#undef BML_FILL_KIND
#undef BML_FILL
    }
};

static const KernelTable &kernels()
{
    static KernelTable t;
    return t;
}

// Row mode when a row is exactly 64 or 128 words (one wavefront).
static int pass_mode(int cols)
{
    const int words = cols / 32;
    return words == 64 ? 1 : words == 128 ? 2 : 0;
}

// Resident blocks per CU of a pass kernel at `threads` threads per block.
static int resident_blocks(int kind, int mode, int io, int k, int threads, int *out)
{
    static std::mutex mu;
    static int cache[8][PASS_KINDS][PASS_MODES][2][MAX_K + 1][3];   // [dev][kind][mode][io][k][wpb]
    int dev = 0;
    BML_HIP(hipGetDevice(&dev));
    int wl = threads == 64 ? 0 : threads == 128 ? 1 : 2;
    std::lock_guard<std::mutex> lock(mu);
    int *c = dev < 8 ? &cache[dev][kind][mode][io][k][wl] : nullptr;
    if (c && *c > 0) {
        *out = *c;
        return BML_OK;
    }
    int nb = 0;
    BML_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, reinterpret_cast<const void *>(kernels().fn[kind][mode][io][k]), threads, 0));
    if (nb < 1)
        nb = 1;
    if (c)
        *c = nb;
    *out = nb;
    return BML_OK;
}

static int launch_1d_grid(int64_t work, int threads, unsigned *grid)
{
    const int64_t g = (work + threads - 1) / threads;
    if (g > 0x7fffffff)
        return fail(BML_EINVAL, "launch too large");
    *grid = (unsigned)std::max<int64_t>(g, 1);
    return BML_OK;
}

int launch_zero(uint32_t *p, int64_t words, hipStream_t stream)
{
    if (words <= 0)
        return BML_OK;
    const unsigned grid = (unsigned)std::min<int64_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid), dim3(256), 0, stream, p, words);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int launch_init(void *state, int32_t rows, int32_t cols, int32_t layout, uint64_t seed,
                double rho_lr, double rho_tb, hipStream_t stream)
{
    const int32_t words = cols / 32;
    unsigned grid;
    int rc = launch_1d_grid((int64_t)rows * words, 256, &grid);
    if (rc)
        return rc;
    // Thresholds on the 53-bit uniform, truncated from IEEE double: LR below
    // rho_lr, TB below rho_lr + rho_tb (for rho/2 each: rho/2 and rho).
    const uint64_t thr_lr = (uint64_t)ldexp(rho_lr, 53);
    const uint64_t thr_tb = (uint64_t)ldexp(rho_lr + rho_tb, 53);
    if (layout == BML_LAYOUT_U8)
        hipLaunchKernelGGL(init_kernel<IO_U8>, dim3(grid), dim3(256), 0, stream, state, rows,
                           words, seed, thr_lr, thr_tb);
    else
        hipLaunchKernelGGL(init_kernel<IO_BP>, dim3(grid), dim3(256), 0, stream, state, rows,
                           words, seed, thr_lr, thr_tb);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int launch_count(const void *state, int32_t rows, int32_t cols, int32_t layout,
                 unsigned long long *counts, hipStream_t stream)
{
    int rc = launch_zero((uint32_t *)counts, 4, stream);
    if (rc)
        return rc;
    DeviceInfo dev;
    if ((rc = device_info(&dev)))
        return rc;
    const int64_t total_words = (int64_t)rows * (cols / 32);
    const unsigned grid =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>((total_words + 255) / 256,
                                                         (int64_t)dev.cu_count * 8));
    if (layout == BML_LAYOUT_U8)
        hipLaunchKernelGGL(count_kernel<IO_U8>, dim3(grid), dim3(256), 0, stream, state,
                           total_words, counts);
    else
        hipLaunchKernelGGL(count_kernel<IO_BP>, dim3(grid), dim3(256), 0, stream, state,
                           total_words, counts);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int launch_pack(const uint8_t *cells, uint32_t *planes, int32_t rows, int32_t cols,
                hipStream_t stream)
{
    const int64_t total_words = (int64_t)rows * (cols / 32);
    unsigned grid;
    int rc = launch_1d_grid(total_words, 256, &grid);
    if (rc)
        return rc;
    hipLaunchKernelGGL(pack_kernel, dim3(grid), dim3(256), 0, stream, cells, planes,
                       planes + total_words, total_words);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int launch_unpack_rows(const uint32_t *lr, const uint32_t *tb, uint8_t *cells, int64_t n_words,
                       hipStream_t stream)
{
    unsigned grid;
    int rc = launch_1d_grid(n_words, 256, &grid);
    if (rc)
        return rc;
    hipLaunchKernelGGL(unpack_kernel, dim3(grid), dim3(256), 0, stream, lr, tb, cells, n_words);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int launch_unpack(const uint32_t *planes, uint8_t *cells, int32_t rows, int32_t cols,
                  hipStream_t stream)
{
    const int64_t total_words = (int64_t)rows * (cols / 32);
    unsigned grid;
    int rc = launch_1d_grid(total_words, 256, &grid);
    if (rc)
        return rc;
    hipLaunchKernelGGL(unpack_kernel, dim3(grid), dim3(256), 0, stream, planes,
                       planes + total_words, cells, total_words);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

} // namespace bml

// ============================================================================
// Handle and C ABI
// ============================================================================

using namespace bml;

struct bml_lattice {
    int32_t rows = 0, cols = 0, layout = 0;
    int32_t topology = 0;                     // BML_TOPO_TORUS / BML_TOPO_KLEIN
    int32_t model = 1;                        // 1: Sec. 2's model; 2: Model II; 3: Model III
    bool both_cells = false;                  // may hold LR+TB cells (Model III only)
    uint64_t coin_seed = 0;                   // Model II conflict coins
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    uint32_t *stats = nullptr;
    int64_t cap = 0;
    hipStream_t stream = nullptr;
    int64_t steps_done = 0;
    uint64_t n_lr0 = 0, n_tb0 = 0;
    int32_t tile_rows = 0, t_phases = 8, wpb = 4;   // tile_rows: strip rows (0 = auto)
    int32_t last_strip_rows = 0;                    // strip height of the last pass
    int32_t auto_rows[MAX_K + 1][3] = {};           // automatic strip height per (k, wpb)
    DeviceInfo dev;
    unsigned long long *d_counts = nullptr;   // library scratch: 2 counters
    PassScratch *d_scratch = nullptr;         // library scratch: stats reduction
    uint8_t *d_stage = nullptr;               // bitplane read-back staging (stage_rows rows)
    int32_t stage_rows = 0;
    // Register-resident tile kernel (bml_block.hpp): steps per launch (0 =
    // the streaming pass kernel) and its per-tile counts.
    int32_t block_steps = 0;
    uint32_t *d_partial = nullptr;            // tiles * BLK_MAX_K * 4 counts
};

static int block_slabs(int rows, int halo);

// Bytes of the bitplane read-back staging buffer: whole rows, at most
// STAGE_BYTES (or one row when a row alone is larger).
constexpr size_t STAGE_BYTES = 16u << 20;

static std::mutex g_handles_mu;
static std::unordered_set<const bml_lattice *> g_handles;

static bool live(const bml_lattice *L)
{
    if (!L)
        return false;
    std::lock_guard<std::mutex> lock(g_handles_mu);
    return g_handles.count(L) != 0;
}

static int count_cars(bml_lattice *L, const void *state, uint64_t *n_lr, uint64_t *n_tb)
{
    int rc = launch_count(state, L->rows, L->cols, L->layout, L->d_counts, L->stream);
    if (rc)
        return rc;
    unsigned long long h[2] = {0, 0};
    BML_HIP(hipMemcpyAsync(h, L->d_counts, sizeof h, hipMemcpyDeviceToHost, L->stream));
    BML_HIP(hipStreamSynchronize(L->stream));
    *n_lr = h[0];
    *n_tb = h[1];
    return BML_OK;
}

extern "C" {

const char *bml_last_error(void) { return g_err; }

int bml_state_bytes_rect(int32_t rows, int32_t cols, int32_t layout, size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(BML_EINVAL, "bytes is NULL");
    if (!valid_shape(rows, cols))
        return fail(BML_EINVAL,
                    "%d x %d: rows must be in [32, 65504], columns a multiple of 32 in "
                    "[32, 65504]", rows, cols);
    if (layout == BML_LAYOUT_U8)
        *bytes = (size_t)rows * cols;
    else if (layout == BML_LAYOUT_BITPLANE)
        *bytes = (size_t)rows * cols / 4;
    else
        return fail(BML_EINVAL, "unknown layout %d", layout);
    return BML_OK;
}

int bml_state_bytes(int32_t n, int32_t layout, size_t *bytes)
{
    clear_error();
    if (!valid_n(n)) {
        if (bytes)
            *bytes = 0;
        return fail(BML_EINVAL, "n=%d must be a multiple of 32 in [32, 65504]", n);
    }
    return bml_state_bytes_rect(n, n, layout, bytes);
}

// Plain streaming copy: the memory-bandwidth reference the benchmark
// reports next to the step kernels (what a kernel that only reads and
// writes each byte once reaches on this device).  Grid-stride, four
// 16-byte loads in flight per thread before their stores.
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src,
                                                   uint4 *__restrict__ dst, int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                    d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride)
        dst[i] = src[i];
}

int bml_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream)
{
    clear_error();
    if (!d_dst || !d_src)
        return fail(BML_EINVAL, "bml_copy: NULL buffer");
    if (!aligned256(d_dst) || !aligned256(d_src) || bytes % 16)
        return fail(BML_EINVAL, "bml_copy: buffers must be 256-byte aligned and bytes a "
                                "multiple of 16");
    const uintptr_t d = (uintptr_t)d_dst, s = (uintptr_t)d_src;
    if (d < s + bytes && s < d + bytes)
        return fail(BML_EINVAL, "bml_copy: buffers overlap");
    if (bytes == 0)
        return BML_OK;
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc)
        return rc;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t blocks = std::min<int64_t>((int64_t)dev.cu_count * 8, (n16 + 255) / 256);
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)hip_stream, (const uint4 *)d_src, (uint4 *)d_dst, n16);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_pack(int32_t n, const uint8_t *d_cells, uint32_t *d_planes, void *hip_stream)
{
    clear_error();
    if (!valid_n(n) || !d_cells || !d_planes)
        return fail(BML_EINVAL, "bml_pack: bad n or NULL buffer");
    if (!aligned256(d_cells) || !aligned256(d_planes))
        return fail(BML_EINVAL, "bml_pack: buffers must be 256-byte aligned");
    const int64_t total_words = (int64_t)n * (n / 32);
    unsigned grid;
    int rc = launch_1d_grid(total_words, 256, &grid);
    if (rc)
        return rc;
    hipLaunchKernelGGL(pack_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream,
                       d_cells, d_planes, d_planes + total_words, total_words);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_unpack(int32_t n, const uint32_t *d_planes, uint8_t *d_cells, void *hip_stream)
{
    clear_error();
    if (!valid_n(n) || !d_cells || !d_planes)
        return fail(BML_EINVAL, "bml_unpack: bad n or NULL buffer");
    if (!aligned256(d_cells) || !aligned256(d_planes))
        return fail(BML_EINVAL, "bml_unpack: buffers must be 256-byte aligned");
    const int64_t total_words = (int64_t)n * (n / 32);
    unsigned grid;
    int rc = launch_1d_grid(total_words, 256, &grid);
    if (rc)
        return rc;
    hipLaunchKernelGGL(unpack_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream,
                       d_planes, d_planes + total_words, d_cells, total_words);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_init_rect(bml_lattice **out, int32_t rows, int32_t cols, int32_t layout, uint64_t seed,
                  double rho_lr, double rho_tb, const uint8_t *cells_host, void *d_state_a,
                  void *d_state_b, bml_step_stats *d_stats, int64_t stats_cap,
                  void *hip_stream)
{
    clear_error();
    if (!out)
        return fail(BML_EINVAL, "out is NULL");
    *out = nullptr;
    size_t bytes = 0;
    int rc = bml_state_bytes_rect(rows, cols, layout, &bytes);
    if (rc)
        return rc;
    if (!d_state_a || !d_state_b || !d_stats)
        return fail(BML_EINVAL, "state or stats buffer is NULL");
    if (d_state_a == d_state_b)
        return fail(BML_EINVAL, "the two state buffers must differ");
    if (!aligned256(d_state_a) || !aligned256(d_state_b) || !aligned256(d_stats))
        return fail(BML_EINVAL, "device buffers must be 256-byte aligned");
    {
        const uintptr_t a = (uintptr_t)d_state_a, b = (uintptr_t)d_state_b;
        if (a < b + bytes && b < a + bytes)
            return fail(BML_EINVAL, "state buffers overlap");
    }
    if (stats_cap < 1 || stats_cap > 0x7fffffff)
        return fail(BML_EINVAL, "stats_cap=%lld must be in [1, 2^31-1]", (long long)stats_cap);
    if (!cells_host && !(rho_lr >= 0.0 && rho_tb >= 0.0 && rho_lr + rho_tb <= 1.0))
        return fail(BML_EINVAL, "densities must be >= 0 with a sum in [0, 1]");
    const size_t n_cells = (size_t)rows * cols;
    bool both_cells = false;   // an LR and a TB car in one cell (Model III)
    if (cells_host) {
        for (size_t k = 0; k < n_cells; ++k) {
            if (cells_host[k] > 3)
                return fail(BML_EINVAL, "cell %zu has value %d (must be 0, 1, 2 or 3)", k,
                            (int)cells_host[k]);
            both_cells |= cells_host[k] == 3;
        }
    }

    bml_lattice *L = new (std::nothrow) bml_lattice();
    if (!L)
        return fail(BML_EDEVICE, "out of host memory");
    L->rows = rows;
    L->cols = cols;
    L->layout = layout;
    L->both_cells = both_cells;
    L->buf[0] = d_state_a;
    L->buf[1] = d_state_b;
    L->stats = (uint32_t *)d_stats;
    L->cap = stats_cap;
    L->stream = (hipStream_t)hip_stream;
    L->t_phases = layout == BML_LAYOUT_U8 ? 8 : 16;
    L->tile_rows = 0;
    L->wpb = 4;
    auto cleanup = [&](int code) {
        if (L->d_counts)
            (void)hipFree(L->d_counts);
        if (L->d_scratch)
            (void)hipFree(L->d_scratch);
        if (L->d_stage)
            (void)hipFree(L->d_stage);
        delete L;
        return code;
    };
    if ((rc = device_info(&L->dev)))
        return cleanup(rc);
    if (hipMalloc(&L->d_counts, 2 * sizeof(unsigned long long)) != hipSuccess) {
        L->d_counts = nullptr;
        return cleanup(fail(BML_EDEVICE, "hipMalloc of count scratch failed"));
    }
    if (hipMalloc(&L->d_scratch, sizeof(PassScratch)) != hipSuccess) {
        L->d_scratch = nullptr;
        return cleanup(fail(BML_EDEVICE, "hipMalloc of stats scratch failed"));
    }
    if ((rc = launch_zero((uint32_t *)L->d_scratch, sizeof(PassScratch) / 4, L->stream)))
        return cleanup(rc);
    if (layout == BML_LAYOUT_BITPLANE) {
        // bml_get_cells unpacks through this buffer in chunks of whole rows
        L->stage_rows = (int32_t)std::max<size_t>(1, std::min<size_t>(rows, STAGE_BYTES / cols));
        if (hipMalloc(&L->d_stage, (size_t)L->stage_rows * cols) != hipSuccess) {
            L->d_stage = nullptr;
            return cleanup(fail(BML_EDEVICE, "hipMalloc of the read-back staging buffer failed"));
        }
    }

    if (!cells_host) {
        if ((rc = launch_init(d_state_a, rows, cols, layout, seed, rho_lr, rho_tb, L->stream)))
            return cleanup(rc);
    } else if (layout == BML_LAYOUT_U8) {
        if (hipMemcpyAsync(d_state_a, cells_host, bytes, hipMemcpyHostToDevice, L->stream) !=
            hipSuccess)
            return cleanup(fail(BML_EDEVICE, "hipMemcpyAsync of the initial cells failed"));
    } else {
        // The byte lattice is 4x larger than a bitplane state buffer: it is
        // uploaded into the staging buffer stage_rows rows at a time and
        // packed from there.
        const int64_t words = cols / 32;
        uint32_t *lr = (uint32_t *)d_state_a;
        uint32_t *tb = lr + (int64_t)rows * words;
        for (int64_t r0 = 0; r0 < rows; r0 += L->stage_rows) {
            const int64_t nr = std::min<int64_t>(L->stage_rows, rows - r0);
            const int64_t n_words = nr * words;
            unsigned grid;
            if ((rc = launch_1d_grid(n_words, 256, &grid)))
                return cleanup(rc);
            if (hipMemcpyAsync(L->d_stage, cells_host + r0 * cols, (size_t)(nr * cols),
                               hipMemcpyHostToDevice, L->stream) != hipSuccess)
                return cleanup(fail(BML_EDEVICE, "upload of the initial cells failed"));
            hipLaunchKernelGGL(pack_kernel, dim3(grid), dim3(256), 0, L->stream, L->d_stage,
                               lr + r0 * words, tb + r0 * words, n_words);
            if (hipGetLastError() != hipSuccess)
                return cleanup(fail(BML_EDEVICE, "pack of the initial cells failed"));
        }
    }
    if ((rc = count_cars(L, d_state_a, &L->n_lr0, &L->n_tb0)))
        return cleanup(rc);
    {
        std::lock_guard<std::mutex> lock(g_handles_mu);
        g_handles.insert(L);
    }
    *out = L;
    return BML_OK;
}

int bml_init(bml_lattice **out, int32_t n, int32_t layout, uint64_t seed, double rho,
             const uint8_t *cells_host, void *d_state_a, void *d_state_b,
             bml_step_stats *d_stats, int64_t stats_cap, void *hip_stream)
{
    clear_error();
    if (out)
        *out = nullptr;
    if (!valid_n(n))
        return fail(BML_EINVAL, "n=%d must be a multiple of 32 in [32, 65504]", n);
    if (!cells_host && !(rho >= 0.0 && rho <= 1.0))
        return fail(BML_EINVAL, "rho must be in [0, 1]");
    // rho/2 + rho/2 == rho exactly, so these are the symmetric thresholds.
    return bml_init_rect(out, n, n, layout, seed, rho * 0.5, rho * 0.5, cells_host, d_state_a,
                         d_state_b, d_stats, stats_cap, hip_stream);
}

int bml_set_topology(bml_lattice *L, int32_t topology)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (topology != BML_TOPO_TORUS && topology != BML_TOPO_KLEIN)
        return fail(BML_EINVAL, "unknown topology %d", topology);
    if (topology == BML_TOPO_KLEIN && L->model != 1)
        return fail(BML_EINVAL, "Models II and III run on the torus only");
    L->topology = topology;
    return BML_OK;
}

int bml_set_model(bml_lattice *L, int32_t model, uint64_t coin_seed)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (model < 1 || model > 3)
        return fail(BML_EINVAL, "model=%d must be 1, 2 or 3", model);
    if (model != 1 && L->topology != BML_TOPO_TORUS)
        return fail(BML_EINVAL, "Models II and III run on the torus only");
    if (model != 3 && L->both_cells)
        return fail(BML_EINVAL, "the lattice may hold cells with both an LR and a TB car, "
                                "which only Model III defines");
    if (model == 2 && L->block_steps)
        return fail(BML_EINVAL, "the register-resident tile kernel runs the model of "
                                "Sec. 2 and Model III only");
    L->model = model;
    L->coin_seed = coin_seed;
    return BML_OK;
}

int bml_get_topology(const bml_lattice *L)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    return L->topology;
}

int bml_get_model(const bml_lattice *L)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    return L->model;
}

int bml_set_tuning(bml_lattice *L, int32_t tile_rows, int32_t t_phases, int32_t waves_per_block)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    const int R = tile_rows >= 0 ? tile_rows : L->tile_rows;
    const int T = t_phases > 0 ? t_phases : L->t_phases;
    const int W = waves_per_block > 0 ? waves_per_block : L->wpb;
    if (R > 65504)
        return fail(BML_EINVAL, "tile_rows=%d must be 0 (auto) or in [1, 65504]", R);
    if (T < 2 || T > 2 * MAX_K || T % 2)
        return fail(BML_EINVAL, "t_phases=%d must be even in [2, %d]", T, 2 * MAX_K);
    if (W != 1 && W != 2 && W != 4)
        return fail(BML_EINVAL, "waves_per_block=%d must be 1, 2 or 4", W);
    L->tile_rows = R;
    L->t_phases = T;
    L->wpb = W;
    return BML_OK;
}

int bml_set_resident(bml_lattice *L, int32_t steps)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (steps < 0 || steps > BLK_MAX_K || steps % 2)
        return fail(BML_EINVAL, "steps=%d must be 0 or even in [2, %d]", steps, BLK_MAX_K);
    if (steps) {
        if (L->model == 2)
            return fail(BML_EINVAL, "the register-resident tile kernel runs the model of "
                                    "Sec. 2 (torus or Klein bottle) and Model III (torus)");
        if (L->rows % 32 || L->cols % (32 * BLK_CHUNK))
            return fail(BML_EINVAL, "%d x %d: the register-resident tile kernel needs rows "
                                    "a multiple of 32 and columns a multiple of %d",
                        L->rows, L->cols, 32 * BLK_CHUNK);
        // counts of the narrowest tiles (the most tiles a launch may use)
        const int64_t tiles = (int64_t)(L->cols / 32 / BLK_CHUNK) * block_slabs(L->rows, steps);
        const size_t bytes = (size_t)tiles * BLK_MAX_K * 4 * sizeof(uint32_t);
        BML_HIP(hipStreamSynchronize(L->stream));   // the old buffer may be in use
        if (L->d_partial)
            (void)hipFree(L->d_partial);
        L->d_partial = nullptr;
        if (hipMalloc(&L->d_partial, bytes) != hipSuccess) {
            L->d_partial = nullptr;
            L->block_steps = 0;
            return fail(BML_EDEVICE, "hipMalloc of the tile kernel's counts failed");
        }
    }
    L->block_steps = steps;
    return BML_OK;
}

int bml_get_resident(const bml_lattice *L)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    return L->block_steps;
}

int bml_get_tuning(const bml_lattice *L, int32_t *tile_rows, int32_t *t_phases,
                   int32_t *waves_per_block)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (tile_rows)
        *tile_rows = L->tile_rows;
    if (t_phases)
        *t_phases = L->t_phases;
    if (waves_per_block)
        *waves_per_block = L->wpb;
    return BML_OK;
}

// One kernel pass of k steps starting at global step `step0`.
// Automatic strip height.  A wavefront's time is (rounds of strips it
// takes) x (cost of one strip); a strip of h rows costs about K h + K^2 + K
// level-rows of pipeline work (its idle levels skipped) plus the conversion
// of h + 2K input rows and h output rows (a byte row costs about as much as
// 1.5 / 1.8 level-rows, a bitplane row almost nothing).  Short strips give
// more waves to spread over the device but pay the halo and pipeline
// fill more often; the rounds term is what punishes a strip count just
// above a multiple of the resident wave count.  Tries every strip count.
static int auto_strip_rows(int n, int tiles_x, int k, int64_t waves, int io)
{
    const double c_in = io == IO_U8 ? 1.5 : 0.1, c_out = io == IO_U8 ? 1.8 : 0.1;
    int best_h = n;
    double best = 0;
    int last_h = 0;
    for (int strips = 1; strips <= n; ++strips) {
        const int h = (n + strips - 1) / strips;
        if (h == last_h)
            continue;
        last_h = h;
        const int s = (n + h - 1) / h;   // strips at this height
        const int64_t items = (int64_t)s * tiles_x;
        const int64_t rounds = (items + waves - 1) / waves;
        const double cost = (double)rounds * ((double)k * h + (double)k * k + k +
                                              c_in * (h + 2 * k) + c_out * h);
        if (best == 0 || cost < best) {
            best = cost;
            best_h = h;
        }
    }
    return best_h;
}

// One launch: lattices G[0..count) (same size, layout, tuning and stream)
// advance k steps.  Lattice i is at global step step0[i]; steps at or after
// rec_from[i] have their counts recorded in its ring.
static int run_pass(bml_lattice *const *G, int count, int k, const int64_t *step0,
                    const int64_t *rec_from)
{
    bml_lattice *L = G[0];
    const int io = L->layout == BML_LAYOUT_U8 ? IO_U8 : IO_BP;
    PassArgs a;
    std::memset(&a, 0, sizeof a);
    a.n_lat = count;
    a.any_rec = 0;
    for (int i = 0; i < count; ++i) {
        PassLattice &pl = a.lat[i];
        pl.src = G[i]->buf[G[i]->cur];
        pl.dst = G[i]->buf[G[i]->cur ^ 1];
        pl.stats = G[i]->stats;
        pl.scratch = G[i]->d_scratch;
        pl.rec_mask = 0;
        for (int j = 0; j < k; ++j)
            if (step0[i] + j >= rec_from[i]) {
                pl.rec_mask |= 1u << j;
                pl.slot[j] = (int32_t)((step0[i] + j) % G[i]->cap);
            }
        a.any_rec |= pl.rec_mask;
        pl.step0 = (uint64_t)step0[i];
        pl.coin_seed = G[i]->coin_seed;
    }
    a.rows = L->rows;
    a.words = L->cols / 32;
    const int mode = pass_mode(L->cols);
    a.tiles_x = mode ? 1 : (a.words + TILE_WORDS - 1) / TILE_WORDS;
    const int threads = 64 * L->wpb;
    int per_cu = 1;
    const int kind = L->model == 2                    ? KIND_MODEL2
                     : L->model == 3                  ? KIND_MODEL3
                     : L->topology == BML_TOPO_KLEIN ? KIND_KLEIN
                                                      : KIND_TORUS;
    int rc = resident_blocks(kind, mode, io, k, threads, &per_cu);
    if (rc)
        return rc;
    const int64_t max_blocks = (int64_t)per_cu * L->dev.cu_count;
    // Strip height: the tuned value, or the automatic one for this pass
    // length, block size and group size (a group spreads count times as
    // many strips over the device).
    int H = L->tile_rows;
    if (H <= 0) {
        int32_t &cached = L->auto_rows[k][L->wpb == 1 ? 0 : L->wpb == 2 ? 1 : 2];
        if (count > 1 || cached <= 0) {
            const int h = auto_strip_rows(L->rows, a.tiles_x * count, k, max_blocks * L->wpb, io);
            if (count > 1)
                H = h;
            else
                cached = h;
        }
        if (count == 1)
            H = cached;
    }
    H = std::min(H, L->rows);
    a.strip_rows = H;
    a.n_tiles = a.tiles_x * ((L->rows + H - 1) / H);
    const int64_t items = (int64_t)a.n_tiles * count;
    const int64_t tile_blocks = (items + L->wpb - 1) / L->wpb;
    // Even out the rounds: every wavefront gets ceil(items / waves) items.
    const int64_t rounds = (tile_blocks + max_blocks - 1) / max_blocks;
    int64_t grid = (tile_blocks + rounds - 1) / rounds;
    if (grid >= 8) {
        grid = (grid + 7) / 8 * 8;
        if (grid > max_blocks)
            grid = max_blocks / 8 * 8;
    }
    a.xcd_split = (grid >= 8 && grid % 8 == 0) ? 1 : 0;
    hipLaunchKernelGGL(kernels().fn[kind][mode][io][k], dim3((unsigned)grid), dim3(threads), 0,
                       L->stream, a);
    BML_HIP(hipGetLastError());
    for (int i = 0; i < count; ++i) {
        G[i]->cur ^= 1;
        G[i]->last_strip_rows = H;
    }
    return BML_OK;
}

// ---- register-resident tile kernel ---------------------------------------

// Tile widths (own words per row) of the tile kernel, widest first.
constexpr int BLK_WIDTHS[3] = {32, 16, 8};

struct BlockTable {
    // [layout][0: the two-phase rule, 1: Model III, 2: the two-phase rule on
    // the Klein bottle][width index]
    BlockFn fn[2][3][3] = {};
    BlockTable() { block_kernels(fn); }
};

// Compute units of the current device (256 when the query fails).
static int block_device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        return 256;
    return n;
}

static const BlockTable &block_table()
{
    static BlockTable t;
    return t;
}

// Row slabs of a lattice of `rows` rows for the tile kernel with `halo`
// halo rows: the fewest that, cut at even rows and held with the halo,
// fit 512 rows.
static int block_slabs(int rows, int halo)
{
    const int per = BLK_ROWS - 2 * halo;          // own rows a slab can hold
    return (rows + per - 1) / per;
}

// Per-step counts of every tile summed per lattice, one block per
// (lattice, step, count); steps at or after rec_from go to the ring.
struct BlockSumArgs {
    const uint32_t *partial[MAX_GROUP];
    uint32_t *stats[MAX_GROUP];
    int64_t step0[MAX_GROUP], rec_from[MAX_GROUP], cap[MAX_GROUP];
    int32_t tiles;
    int32_t n_steps;
};

__global__ __launch_bounds__(256) void block_sum_kernel(BlockSumArgs a)
{
    const int li = blockIdx.x / (a.n_steps * 4);
    const int j = blockIdx.x - li * a.n_steps * 4;    // step * 4 + count
    uint32_t v = 0;
    for (int t = threadIdx.x; t < a.tiles; t += blockDim.x)
        v += a.partial[li][(size_t)t * BLK_MAX_K * 4 + j];
    v = wave_sum(v);
    __shared__ uint32_t part[4];
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t sum = part[0] + part[1] + part[2] + part[3];
        const int64_t step = a.step0[li] + (j >> 2);
        if (step >= a.rec_from[li])
            a.stats[li][(size_t)(step % a.cap[li]) * 4 + (j & 3)] = sum;
    }
}

// One launch of the tile kernel: lattices G[0..count) (same size, layout,
// stream) advance k <= block_steps steps; lattice i is at global step
// step0[i], and steps at or after rec_from[i] are recorded in its ring.
static int run_block(bml_lattice *const *G, int count, int k, const int64_t *step0,
                     const int64_t *rec_from)
{
    bml_lattice *L = G[0];
    const int io = L->layout == BML_LAYOUT_U8 ? IO_U8 : IO_BP;
    BlockArgs a;
    std::memset(&a, 0, sizeof a);
    a.n_lat = count;
    a.rows = L->rows;
    a.words = L->cols / 32;
    a.halo = L->block_steps;
    a.slabs = block_slabs(L->rows, a.halo);
    a.n_steps = k;
    // The widest tiles that still give every CU two workgroups (narrower
    // tiles hold more halo columns per own column), else the narrowest
    // that divide the row.
    static const int cus = block_device_cus();
    int wi = -1;
    for (int i = 0; i < 3; ++i) {
        if (a.words % BLK_WIDTHS[i])
            continue;
        wi = i;
        if ((int64_t)count * (a.words / BLK_WIDTHS[i]) * a.slabs >= 2 * cus)
            break;
    }
    if (wi < 0)
        return fail(BML_EINVAL, "%d columns: not a whole number of tiles", L->cols);
    a.tiles_x = a.words / BLK_WIDTHS[wi];
    const int tiles = a.tiles_x * a.slabs;
    BlockSumArgs b;
    std::memset(&b, 0, sizeof b);
    b.tiles = tiles;
    b.n_steps = k;
    for (int i = 0; i < count; ++i) {
        a.lat[i].src = G[i]->buf[G[i]->cur];
        a.lat[i].dst = G[i]->buf[G[i]->cur ^ 1];
        a.lat[i].partial = G[i]->d_partial;
        b.partial[i] = G[i]->d_partial;
        b.stats[i] = G[i]->stats;
        b.step0[i] = step0[i];
        b.rec_from[i] = rec_from[i];
        b.cap[i] = G[i]->cap;
    }
    const int rule = L->model == 3 ? 1 : L->topology == BML_TOPO_KLEIN ? 2 : 0;
    hipLaunchKernelGGL(block_table().fn[io][rule][wi], dim3((unsigned)(tiles * count)),
                       dim3(64 * BLK_WAVES), 0, L->stream, a);
    BML_HIP(hipGetLastError());
    hipLaunchKernelGGL(block_sum_kernel, dim3((unsigned)(count * k * 4)), dim3(256), 0,
                       L->stream, b);
    BML_HIP(hipGetLastError());
    for (int i = 0; i < count; ++i)
        G[i]->cur ^= 1;
    return BML_OK;
}

// Advances lattices G[0..count) by n_steps in joint launches.
static int step_group(bml_lattice *const *G, int count, int64_t n_steps)
{
    int64_t end[MAX_GROUP], rec_from[MAX_GROUP], s[MAX_GROUP];
    for (int i = 0; i < count; ++i) {
        end[i] = G[i]->steps_done + n_steps;
        // earlier steps of this call would be overwritten in the ring
        rec_from[i] = end[i] - std::min<int64_t>(n_steps, G[i]->cap);
        s[i] = G[i]->steps_done;
    }
    const bool block = G[0]->block_steps > 0;
    const int K = block ? G[0]->block_steps : G[0]->t_phases / 2;
    int64_t done = 0;
    while (done < n_steps) {
        const int k = (int)std::min<int64_t>(K, n_steps - done);
        int rc = block ? run_block(G, count, k, s, rec_from) : run_pass(G, count, k, s, rec_from);
        if (rc)
            return rc;
        done += k;
        for (int i = 0; i < count; ++i) {
            s[i] += k;
            G[i]->steps_done = s[i];
            G[i]->both_cells |= G[i]->model == 3;
        }
    }
    return BML_OK;
}

int bml_step(bml_lattice *L, int64_t n_steps)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (n_steps < 0)
        return fail(BML_EINVAL, "n_steps must be >= 0");
    if (L->both_cells && L->model != 3)
        return fail(BML_EINVAL, "the lattice holds cells with both an LR and a TB car; "
                                "select Model III (bml_set_model) to step it");
    if (n_steps == 0)
        return BML_OK;
    bml_lattice *G[1] = {L};
    return step_group(G, 1, n_steps);
}

int bml_step_group(bml_lattice *const *handles, int32_t count, int64_t n_steps)
{
    clear_error();
    if (!handles || count < 1 || count > MAX_GROUP)
        return fail(BML_EINVAL, "count=%d must be in [1, %d]", count, MAX_GROUP);
    if (n_steps < 0)
        return fail(BML_EINVAL, "n_steps must be >= 0");
    for (int i = 0; i < count; ++i) {
        if (!live(handles[i]))
            return fail(BML_ESTATE, "handle %d is invalid", i);
        for (int j = 0; j < i; ++j)
            if (handles[j] == handles[i])
                return fail(BML_EINVAL, "handle %d appears twice", i);
        const bml_lattice *L0 = handles[0], *Li = handles[i];
        if (Li->rows != L0->rows || Li->cols != L0->cols || Li->layout != L0->layout ||
            Li->topology != L0->topology || Li->model != L0->model)
            return fail(BML_EINVAL, "lattice %d differs in size, layout, topology or model from "
                                    "lattice 0", i);
        if (Li->tile_rows != L0->tile_rows || Li->t_phases != L0->t_phases ||
            Li->wpb != L0->wpb || Li->block_steps != L0->block_steps)
            return fail(BML_EINVAL, "lattice %d has another tuning than lattice 0", i);
        if (Li->stream != L0->stream || Li->dev.device != L0->dev.device)
            return fail(BML_EINVAL, "lattice %d is on another stream or device", i);
        if (Li->both_cells && Li->model != 3)
            return fail(BML_EINVAL, "lattice %d holds cells with both an LR and a TB car; "
                                    "select Model III (bml_set_model) to step it", i);
    }
    if (n_steps == 0)
        return BML_OK;
    return step_group(handles, count, n_steps);
}

} // extern "C"

// ============================================================================
// Allocation-free stepping
// ============================================================================

namespace bml {

// Stats-reduction scratch of bml_step_group_static: one PassScratch per
// lattice of a call, in device memory the library never allocates.  In
// host code this name is a host-side stand-in, not a device address; the
// device address is looked up once per device and only that pointer is
// passed to kernels.  Each device holds its own copy until the process ends.
constexpr int STATIC_MAX_LATTICES = BML_STATIC_MAX_LATTICES;
static_assert(STATIC_MAX_LATTICES <= MAX_GROUP, "a launch advances at most MAX_GROUP lattices");
static __device__ __align__(256) PassScratch scratch[STATIC_MAX_LATTICES];

constexpr int STATIC_MAX_DEVICES = 64;

// Device address of `scratch` on the current device (looked up on the
// first call on that device, with that device current).
static int static_scratch(PassScratch **out)
{
    static std::mutex mu;
    static PassScratch *addr[STATIC_MAX_DEVICES] = {};
    int dev = 0;
    BML_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAX_DEVICES)
        return fail(BML_EDEVICE, "device %d: the static scratch table holds %d devices", dev,
                    STATIC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(BML_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        addr[dev] = (PassScratch *)p;
    }
    *out = addr[dev];
    return BML_OK;
}

} // namespace bml

extern "C" {

int bml_step_group_static(int32_t count, int32_t rows, int32_t cols, int32_t layout,
                          void *const *d_state_a, void *const *d_state_b,
                          bml_step_stats *const *d_stats, int64_t stats_cap,
                          int64_t first_step, int64_t n_steps, int32_t t_phases,
                          void *hip_stream, int32_t *result_in_b)
{
    clear_error();
    if (count < 1 || count > STATIC_MAX_LATTICES)
        return fail(BML_EINVAL, "count=%d: the static scratch holds 1 to %d lattices", count,
                    STATIC_MAX_LATTICES);
    size_t bytes = 0;
    int rc = bml_state_bytes_rect(rows, cols, layout, &bytes);
    if (rc)
        return rc;
    if (!d_state_a || !d_state_b || !d_stats || !result_in_b)
        return fail(BML_EINVAL, "NULL argument");
    if (stats_cap < 1 || stats_cap > 0x7fffffff)
        return fail(BML_EINVAL, "stats_cap=%lld must be in [1, 2^31-1]", (long long)stats_cap);
    if (first_step < 0 || n_steps < 0)
        return fail(BML_EINVAL, "first_step and n_steps must be >= 0");
    if (t_phases < 2 || t_phases > 2 * MAX_K || t_phases % 2)
        return fail(BML_EINVAL, "t_phases=%d must be even in [2, %d]", t_phases, 2 * MAX_K);
    for (int i = 0; i < count; ++i) {
        if (!d_state_a[i] || !d_state_b[i] || !d_stats[i])
            return fail(BML_EINVAL, "lattice %d: NULL buffer", i);
        if (!aligned256(d_state_a[i]) || !aligned256(d_state_b[i]) || !aligned256(d_stats[i]))
            return fail(BML_EINVAL, "lattice %d: device buffers must be 256-byte aligned", i);
        const uintptr_t a = (uintptr_t)d_state_a[i], b = (uintptr_t)d_state_b[i];
        if (a < b + bytes && b < a + bytes)
            return fail(BML_EINVAL, "lattice %d: state buffers overlap", i);
    }
    *result_in_b = 0;
    if (n_steps == 0)
        return BML_OK;
    PassScratch *ptr = nullptr;
    if ((rc = static_scratch(&ptr)))
        return rc;
    // Host-side descriptors only (no device memory): the same launches as
    // bml_step_group with the automatic strip height and 4 waves per block.
    bml_lattice lats[STATIC_MAX_LATTICES];
    bml_lattice *G[STATIC_MAX_LATTICES];
    DeviceInfo dev;
    if ((rc = device_info(&dev)))
        return rc;
    for (int i = 0; i < count; ++i) {
        bml_lattice &L = lats[i];
        L.rows = rows;
        L.cols = cols;
        L.layout = layout;
        L.buf[0] = d_state_a[i];
        L.buf[1] = d_state_b[i];
        L.stats = (uint32_t *)d_stats[i];
        L.cap = stats_cap;
        L.stream = (hipStream_t)hip_stream;
        L.steps_done = first_step;
        L.t_phases = t_phases;
        L.tile_rows = 0;
        L.wpb = 4;
        L.dev = dev;
        L.d_scratch = ptr + i;
        G[i] = &L;
    }
    // The reduction needs its scratch at zero; the array keeps whatever the
    // last call (possibly one that failed mid-way) left there.
    if ((rc = launch_zero((uint32_t *)ptr, (int64_t)count * sizeof(PassScratch) / 4,
                          (hipStream_t)hip_stream)))
        return rc;
    if ((rc = step_group(G, count, n_steps)))
        return rc;
    *result_in_b = lats[0].cur;
    return BML_OK;
}

int bml_stats(bml_lattice *L, int64_t first_step, int64_t count, bml_step_stats *out_host)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (count < 0 || (count > 0 && !out_host))
        return fail(BML_EINVAL, "bad count or NULL output");
    if (first_step < 0 || first_step + count > L->steps_done ||
        first_step < L->steps_done - L->cap)
        return fail(BML_ERANGE, "steps [%lld, %lld) not retained (done %lld, ring %lld)",
                    (long long)first_step, (long long)(first_step + count),
                    (long long)L->steps_done, (long long)L->cap);
    int64_t i = 0;
    while (i < count) {
        const int64_t slot = (first_step + i) % L->cap;
        const int64_t run = std::min<int64_t>(count - i, L->cap - slot);
        BML_HIP(hipMemcpyAsync(out_host + i, L->stats + slot * 4, run * sizeof(bml_step_stats),
                               hipMemcpyDeviceToHost, L->stream));
        i += run;
    }
    BML_HIP(hipStreamSynchronize(L->stream));
    for (int64_t j = 0; j < count; ++j)
        if (out_host[j].n_lr != L->n_lr0 || out_host[j].n_tb != L->n_tb0)
            return fail(BML_ECORRUPT,
                        "step %lld: car counts (%u, %u) differ from the initial (%llu, %llu)",
                        (long long)(first_step + j), out_host[j].n_lr, out_host[j].n_tb,
                        (unsigned long long)L->n_lr0, (unsigned long long)L->n_tb0);
    return BML_OK;
}

int bml_get_cells(bml_lattice *L, uint8_t *out_host)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (!out_host)
        return fail(BML_EINVAL, "out_host is NULL");
    const size_t cells = (size_t)L->rows * L->cols;
    if (L->layout == BML_LAYOUT_U8) {
        BML_HIP(hipMemcpyAsync(out_host, L->buf[L->cur], cells, hipMemcpyDeviceToHost,
                               L->stream));
        BML_HIP(hipStreamSynchronize(L->stream));
        return BML_OK;
    }
    // Bitplanes: unpack stage_rows rows at a time into the handle's staging
    // buffer and copy each chunk out (stream order keeps a chunk's copy
    // ahead of the next unpack into the same buffer).
    const int64_t words = L->cols / 32;
    const int64_t plane_words = (int64_t)L->rows * words;
    const uint32_t *lr = (const uint32_t *)L->buf[L->cur];
    const uint32_t *tb = lr + plane_words;
    for (int64_t r0 = 0; r0 < L->rows; r0 += L->stage_rows) {
        const int64_t nr = std::min<int64_t>(L->stage_rows, L->rows - r0);
        const int64_t n_words = nr * words;
        int rc = launch_unpack_rows(lr + r0 * words, tb + r0 * words, L->d_stage, n_words,
                                    L->stream);
        if (rc)
            return rc;
        BML_HIP(hipMemcpyAsync(out_host + r0 * L->cols, L->d_stage, (size_t)(nr * L->cols),
                               hipMemcpyDeviceToHost, L->stream));
    }
    BML_HIP(hipStreamSynchronize(L->stream));
    return BML_OK;
}

int bml_initial_counts(const bml_lattice *L, uint64_t *n_lr, uint64_t *n_tb)
{
    clear_error();
    if (!live(L))
        return fail(BML_ESTATE, "invalid handle");
    if (n_lr)
        *n_lr = L->n_lr0;
    if (n_tb)
        *n_tb = L->n_tb0;
    return BML_OK;
}

int64_t bml_step_count(const bml_lattice *L) { return live(L) ? L->steps_done : -1; }

const void *bml_current_state(const bml_lattice *L) { return live(L) ? L->buf[L->cur] : nullptr; }

void bml_free(bml_lattice *L)
{
    if (!live(L))
        return;
    {
        std::lock_guard<std::mutex> lock(g_handles_mu);
        g_handles.erase(L);
    }
    (void)hipStreamSynchronize(L->stream);
    if (L->d_counts)
        (void)hipFree(L->d_counts);
    if (L->d_scratch)
        (void)hipFree(L->d_scratch);
    if (L->d_stage)
        (void)hipFree(L->d_stage);
    if (L->d_partial)
        (void)hipFree(L->d_partial);
    delete L;
}

} // extern "C"
