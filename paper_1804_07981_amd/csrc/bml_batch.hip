// bml_batch.hip -- host side of the batched BML sweep (include/bml.h,
// bml_batch_*): many lattices of uneven size and density advanced together,
// one kernel launch per pass over all active lattices, optionally captured
// in a hipGraph and replayed.  The kernel is in bml_batch.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "bml.h"
#include "bml_batch.hpp"
#include "bml_common.hpp"
#include "bml_resident.hpp"

namespace bml {

struct BatchTable {
    BatchFn fn[2][MAX_K + 1] = {};
    BatchTable()
    {
        batch_table_u8(fn[IO_U8]);
        batch_table_bp(fn[IO_BP]);
    }
};

static const BatchTable &batch_kernels()
{
    static BatchTable t;
    return t;
}

struct ResidentTable {
    ResidentFn fn[2] = {};
    ResidentTable()
    {
        fn[IO_U8] = resident_kernel_u8();
        fn[IO_BP] = resident_kernel_bp();
    }
};

static const ResidentTable &resident_table()
{
    static ResidentTable t;
    return t;
}

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t lattice_state_bytes(int32_t n, int32_t layout)
{
    return layout == BML_LAYOUT_U8 ? (size_t)n * n : (size_t)n * n / 4;
}

// Largest divisor of n that is <= target (and >= 1).
static int divisor_at_most(int n, int target)
{
    target = std::max(1, std::min(target, n));
    for (int d = target; d >= 1; --d)
        if (n % d == 0)
            return d;
    return 1;
}

} // namespace bml

using namespace bml;

struct bml_batch {
    int32_t count = 0, layout = 0;
    std::vector<int32_t> n;
    std::vector<void *> buf[2];
    std::vector<uint64_t> n_lr0, n_tb0;
    std::vector<uint8_t> active;
    std::vector<int32_t> parity_base, pass_base;   // host copy of the descriptors
    std::vector<int64_t> steps;                    // steps run by each lattice
    uint32_t *trace = nullptr;
    int64_t trace_steps = 0;
    hipStream_t stream = nullptr;
    int32_t strip_target = 64, t_phases = 16, wpb = 4;
    // Register-resident runs (bml_resident.hpp) when every lattice has
    // N <= resident_max_n (at most 32 * RES_MAX_WORDS; 0 = never).
    int32_t resident_max_n = 32 * RES_MAX_WORDS;
    // Halo rows of the slabs that lattices taller than a workgroup are cut
    // into (0 = the default); a launch then runs at most that many steps.
    int32_t resident_split = 0;
    int32_t res_grid = 0;                   // bins per resident launch (fixed while captured)
    int64_t host_step = 0, host_pass = 0;
    DeviceInfo dev;
    // Library-owned device memory.
    BatchLattice *d_lat = nullptr;
    BatchItem *d_items = nullptr;
    ResidentBin *d_bins = nullptr;
    int32_t res_cut = 0, res_halo = 0;      // lattices cut into slabs; their halo rows
    BatchCounters *d_ctr = nullptr;
    unsigned long long *d_counts = nullptr;
    uint8_t *d_stage = nullptr;   // bitplane read-back staging, stage_bytes
    size_t stage_bytes = 0;
    int64_t items_cap = 0;
    // Captured run.
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_steps = 0, graph_passes = 0;
};

static std::mutex g_batch_mu;
static std::unordered_set<const bml_batch *> g_batches;

static bool batch_live(const bml_batch *B)
{
    if (!B)
        return false;
    std::lock_guard<std::mutex> lock(g_batch_mu);
    return g_batches.count(B) != 0;
}

static void batch_release(bml_batch *B)
{
    if (B->graph_exec)
        (void)hipGraphExecDestroy(B->graph_exec);
    if (B->graph)
        (void)hipGraphDestroy(B->graph);
    if (B->d_lat)
        (void)hipFree(B->d_lat);
    if (B->d_items)
        (void)hipFree(B->d_items);
    if (B->d_bins)
        (void)hipFree(B->d_bins);
    if (B->d_ctr)
        (void)hipFree(B->d_ctr);
    if (B->d_counts)
        (void)hipFree(B->d_counts);
    if (B->d_stage)
        (void)hipFree(B->d_stage);
    delete B;
}

// Geometry of lattice b under the current tuning.
static void lattice_geometry(const bml_batch *B, int b, int *H, int *groups, int *group_lanes,
                             int *tiles_x)
{
    const int n = B->n[b];
    const int words = n / 32;
    const int K = B->t_phases / 2;
    int h = divisor_at_most(n, B->strip_target);
    // Keep the 2K halo rows a minor part of a strip when n allows it.
    if (h < 4 * K && n >= 4 * K)
        h = divisor_at_most(n, std::max(B->strip_target, 4 * K) * 2);
    *H = h;
    if (words <= TILE_WORDS) {
        *group_lanes = words + 2;
        *groups = 64 / (words + 2);
        *tiles_x = 1;
    } else {
        *group_lanes = 64;
        *groups = 1;
        *tiles_x = (words + TILE_WORDS - 1) / TILE_WORDS;
    }
}

// True when the batch runs register-resident: every lattice (active or not,
// so the mode does not change as lattices retire) fits.
static bool use_resident(const bml_batch *B)
{
    if (B->resident_max_n <= 0)
        return false;
    const int nmax = *std::max_element(B->n.begin(), B->n.end());
    return nmax <= std::min(B->resident_max_n, 32 * RES_MAX_WORDS);
}

// Work of a resident workgroup per step: row-words held (its items' width
// times the rows they hold, halo rows included).
static int64_t item_work(const ResidentItem &it, int W)
{
    return (int64_t)W * (it.rows + 2 * it.halo);
}

static int rows_waves(int rows) { return (rows + RES_WAVE_ROWS - 1) / RES_WAVE_ROWS; }

// Compute units of the current device (256 when the query fails).
static int device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        return 256;
    return n;
}

static int held_waves(const ResidentItem &it) { return rows_waves(it.rows + 2 * it.halo); }

constexpr int RES_BLOCK_ROWS = RES_WAVES * RES_WAVE_ROWS;   // rows one workgroup holds
constexpr int RES_DEFAULT_SPLIT = 64;                       // halo when a cut is required
constexpr int RES_MAX_SPLIT = (RES_BLOCK_ROWS - 32) / 2 / 16 * 16;   // a 32-row slab still fits

// Halo rows of the slab plan: the configured value, or, when some lattice
// is taller than a workgroup holds and none is configured, the default.
static int plan_halo(const bml_batch *B)
{
    if (B->resident_split > 0)
        return B->resident_split;
    const int nmax = *std::max_element(B->n.begin(), B->n.end());
    return nmax > RES_BLOCK_ROWS ? RES_DEFAULT_SPLIT : 0;
}

// How lattice n is cut for the resident kernel: 1 (whole) or the fewest
// slabs of whole 32-row blocks that, held with K halo rows, fit one
// workgroup.
static int slab_count(int n, int K)
{
    if (n <= RES_BLOCK_ROWS)
        return 1;
    int P = 2;
    while ((n / 32 + P - 1) / P * 32 + 2 * K > RES_BLOCK_ROWS)
        ++P;
    return P;
}

// Slabs of lattice b under the current plan (B->res_halo is set when the
// plan is made).
static int lattice_slabs(const bml_batch *B, int b) { return slab_count(B->n[b], B->res_halo); }

// Bins of the resident kernel for the lattices flagged in `on`.  Slabs
// take a bin each; whole lattices of one width share bins, as many as the
// workgroup's waves hold.  The most expensive bins come first, so that
// they start first.
static std::vector<ResidentBin> resident_bins(const bml_batch *B, const std::vector<uint8_t> &on)
{
    std::vector<ResidentBin> bins;
    const int K = B->res_halo;
    for (int W = 1; W <= RES_MAX_WORDS; ++W) {
        const int n = 32 * W;
        ResidentBin cur{};
        cur.words = W;
        int cur_waves = 0;
        for (int b = 0; b < B->count; ++b) {
            if (!on[b] || B->n[b] != n)
                continue;
            const int P = lattice_slabs(B, b);
            if (P > 1) {
                for (int i = 0; i < P; ++i) {
                    const int lo = (n / 32) * i / P * 32, hi = (n / 32) * (i + 1) / P * 32;
                    ResidentBin sb{};
                    sb.words = W;
                    sb.n_items = 1;
                    sb.item[0] = ResidentItem{b, lo, hi - lo, K, i};
                    bins.push_back(sb);
                }
                continue;
            }
            const ResidentItem it{b, 0, n, 0, -1};
            if (cur_waves + held_waves(it) > RES_WAVES || cur.n_items == RES_MAX_ITEMS) {
                bins.push_back(cur);
                cur = ResidentBin{};
                cur.words = W;
                cur_waves = 0;
            }
            cur.item[cur.n_items++] = it;
            cur_waves += held_waves(it);
        }
        if (cur.n_items)
            bins.push_back(cur);
    }
    auto cost = [](const ResidentBin &x) {
        int64_t w = 0;
        for (int i = 0; i < x.n_items; ++i)
            w += item_work(x.item[i], x.words);
        return w;
    };
    std::stable_sort(bins.begin(), bins.end(),
                     [&](const ResidentBin &x, const ResidentBin &y) { return cost(x) > cost(y); });
    // Workgroup b shares a CU with b + cus and b + 2 cus (the dispatcher
    // fills one slot of every CU before the next): alternate the direction
    // of each run of `cus` bins, so that a CU that takes one of the heaviest
    // bins takes one of the lightest of the next run.
    const int cus = device_cus();
    for (size_t t = cus; t < bins.size(); t += 2 * (size_t)cus)
        std::reverse(bins.begin() + t, bins.begin() + std::min(bins.size(), t + cus));
    return bins;
}


// Uploads the descriptors and the item list of the active lattices.
// Synchronises the stream.
static int upload_work(bml_batch *B)
{
    std::vector<BatchLattice> lat(B->count);
    std::vector<BatchItem> items;
    for (int b = 0; b < B->count; ++b) {
        int H, G, GW, TX;
        lattice_geometry(B, b, &H, &G, &GW, &TX);
        BatchLattice &d = lat[b];
        d.buf[0] = B->buf[0][b];
        d.buf[1] = B->buf[1][b];
        d.n = B->n[b];
        d.words = B->n[b] / 32;
        d.strip_rows = H;
        d.groups = G;
        d.group_lanes = GW;
        d.parity_base = B->parity_base[b];
        d.pass_base = (int32_t)B->pass_base[b];
        d.pad = 0;
        if (!B->active[b])
            continue;
        const int strips = B->n[b] / H;
        for (int s0 = 0; s0 < strips; s0 += G)
            for (int tx = 0; tx < TX; ++tx)
                items.push_back(BatchItem{b, s0, tx, 0});
    }
    if ((int64_t)items.size() > B->items_cap) {
        if (B->d_items)
            (void)hipFree(B->d_items);
        B->d_items = nullptr;
        B->items_cap = 0;
        if (hipMalloc(&B->d_items, std::max<size_t>(1, items.size()) * sizeof(BatchItem)) !=
            hipSuccess)
            return fail(BML_EDEVICE, "hipMalloc of the batch item list failed");
        B->items_cap = (int64_t)items.size();
    }
    if (use_resident(B)) {
        // The launch grid is the bin count with every lattice active, so a
        // captured run stays valid as lattices retire: the bins of the
        // active lattices come first, padding bins (no lattice) after.
        if (B->res_grid == 0) {
            // The plan's target is fixed with every lattice active: a
            // subset then cuts the same lattices and needs no more bins.
            B->res_halo = plan_halo(B);
            const std::vector<uint8_t> all(B->count, 1);
            const int32_t grid = std::max<int32_t>(1, (int32_t)resident_bins(B, all).size());
            int32_t cut = 0;
            for (int b = 0; b < B->count; ++b)
                cut += lattice_slabs(B, b) > 1;
            if (B->d_bins)
                (void)hipFree(B->d_bins);
            B->d_bins = nullptr;
            if (hipMalloc(&B->d_bins, (size_t)grid * sizeof(ResidentBin)) != hipSuccess) {
                B->res_grid = 0;
                return fail(BML_EDEVICE, "hipMalloc of the resident plan failed");
            }
            B->res_grid = grid;
            B->res_cut = cut;
        }
        std::vector<ResidentBin> bins = resident_bins(B, B->active);
        if ((int64_t)bins.size() > B->res_grid)
            return fail(BML_EDEVICE, "resident plan of %zu bins exceeds the %d of the launch",
                        bins.size(), B->res_grid);
        bins.resize(B->res_grid, ResidentBin{1, 0, {}});
        BML_HIP(hipMemcpyAsync(B->d_bins, bins.data(), bins.size() * sizeof(ResidentBin),
                               hipMemcpyHostToDevice, B->stream));
    }
    BML_HIP(hipMemcpyAsync(B->d_lat, lat.data(), lat.size() * sizeof(BatchLattice),
                           hipMemcpyHostToDevice, B->stream));
    if (!items.empty())
        BML_HIP(hipMemcpyAsync(B->d_items, items.data(), items.size() * sizeof(BatchItem),
                               hipMemcpyHostToDevice, B->stream));
    BatchCounters c;
    c.step = (uint32_t)B->host_step;
    c.pass = (uint32_t)B->host_pass;
    c.n_items = (uint32_t)items.size();
    c.ticket = 0;
    BML_HIP(hipMemcpyAsync(B->d_ctr, &c, sizeof c, hipMemcpyHostToDevice, B->stream));
    BML_HIP(hipStreamSynchronize(B->stream));
    return BML_OK;
}

// Zeroes the trace entries of steps [step, step + n_steps) of every lattice;
// `step` is read on the device so that a captured graph stays correct.
__global__ void zero_trace_kernel(uint32_t *trace, int32_t count, int64_t trace_steps,
                                  const BatchCounters *ctr, int64_t n_steps)
{
    const int64_t s0 = __hip_atomic_load(&ctr->step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t s1 = std::min<int64_t>(s0 + n_steps, trace_steps);
    if (s1 <= s0)
        return;
    const int64_t per = (s1 - s0) * 2;
    const int64_t total = per * count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / per, r = i - b * per;
        trace[(b * trace_steps + s0) * 2 + r] = 0;
    }
}

static int batch_blocks_per_cu(int io, int k, int threads, int *out)
{
    static std::mutex mu;
    static int cache[8][2][MAX_K + 1][3];
    int dev = 0;
    BML_HIP(hipGetDevice(&dev));
    const int wl = threads == 64 ? 0 : threads == 128 ? 1 : 2;
    std::lock_guard<std::mutex> lock(mu);
    int *c = dev < 8 ? &cache[dev][io][k][wl] : nullptr;
    if (c && *c > 0) {
        *out = *c;
        return BML_OK;
    }
    int nb = 0;
    BML_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, reinterpret_cast<const void *>(batch_kernels().fn[io][k]), threads, 0));
    nb = std::max(nb, 1);
    if (c)
        *c = nb;
    *out = nb;
    return BML_OK;
}

// Enqueues n_steps steps of every active lattice (no synchronisation).
static int enqueue_run(bml_batch *B, int64_t n_steps, int64_t *passes)
{
    const int io = B->layout == BML_LAYOUT_U8 ? IO_U8 : IO_BP;
    const unsigned zgrid = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(4096, (B->count * std::min(n_steps, B->trace_steps) * 2 + 255) / 256));
    hipLaunchKernelGGL(zero_trace_kernel, dim3(zgrid), dim3(256), 0, B->stream, B->trace,
                       B->count, B->trace_steps, B->d_ctr, n_steps);
    BML_HIP(hipGetLastError());
    if (use_resident(B)) {
        // One launch runs every step (up to 2^30 per launch), the states
        // staying in registers throughout; with slabs, at most as many
        // steps as their halo rows.
        const ResidentFn fn = resident_table().fn[io];
        const int64_t per = B->res_cut ? B->res_halo : (int64_t)1 << 30;
        int64_t s = 0, p = 0;
        while (s < n_steps) {
            const int64_t k = std::min<int64_t>(n_steps - s, per);
            ResidentArgs a;
            a.lat = B->d_lat;
            a.bins = B->d_bins;
            a.ctr = B->d_ctr;
            a.trace = B->trace;
            a.trace_steps = (int32_t)B->trace_steps;
            a.n_steps = (int32_t)k;
            hipLaunchKernelGGL(fn, dim3((unsigned)B->res_grid), dim3(64 * RES_WAVES), 0,
                               B->stream, a);
            BML_HIP(hipGetLastError());
            s += k;
            ++p;
        }
        *passes = p;
        return BML_OK;
    }
    const int K = B->t_phases / 2;
    const int threads = 64 * B->wpb;
    int64_t s = 0, p = 0;
    while (s < n_steps) {
        const int k = (int)std::min<int64_t>(K, n_steps - s);
        int per_cu = 1;
        int rc = batch_blocks_per_cu(io, k, threads, &per_cu);
        if (rc)
            return rc;
        int64_t grid = (int64_t)per_cu * B->dev.cu_count;
        grid = std::max<int64_t>(8, grid / 8 * 8);
        BatchArgs a;
        a.lat = B->d_lat;
        a.items = B->d_items;
        a.ctr = B->d_ctr;
        a.trace = B->trace;
        a.trace_steps = (int32_t)B->trace_steps;
        a.k = k;
        a.xcd_split = 1;
        hipLaunchKernelGGL(batch_kernels().fn[io][k], dim3((unsigned)grid), dim3(threads), 0,
                           B->stream, a);
        BML_HIP(hipGetLastError());
        s += k;
        ++p;
    }
    *passes = p;
    return BML_OK;
}

static void account_run(bml_batch *B, int64_t n_steps, int64_t passes)
{
    B->host_step += n_steps;
    B->host_pass += passes;
    for (int b = 0; b < B->count; ++b)
        if (B->active[b])
            B->steps[b] += n_steps;
}

// Current parity of lattice b (which of its buffers holds the state).
static int lattice_parity(const bml_batch *B, int b)
{
    if (!B->active[b])
        return B->parity_base[b] & 1;
    return (int)((B->parity_base[b] + (B->host_pass - B->pass_base[b])) & 1);
}

extern "C" {

int bml_batch_arena_bytes(int32_t count, const int32_t *n, int32_t layout, size_t *bytes)
{
    clear_error();
    if (count < 1 || !n || !bytes)
        return fail(BML_EINVAL, "bml_batch_arena_bytes: bad count or NULL pointer");
    if (layout != BML_LAYOUT_U8 && layout != BML_LAYOUT_BITPLANE)
        return fail(BML_EINVAL, "unknown layout %d", layout);
    size_t total = 0;
    for (int b = 0; b < count; ++b) {
        if (!valid_n(n[b]))
            return fail(BML_EINVAL, "lattice %d: n=%d must be a multiple of 32 in [32, 65504]",
                        b, n[b]);
        total += 2 * round256(lattice_state_bytes(n[b], layout));
    }
    *bytes = total;
    return BML_OK;
}

int bml_batch_init(bml_batch **out, int32_t count, const int32_t *n, const double *rho,
                   const uint64_t *seed, int32_t layout, void *d_arena, size_t arena_bytes,
                   uint32_t *d_trace, int64_t trace_steps, void *hip_stream)
{
    clear_error();
    if (!out)
        return fail(BML_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = bml_batch_arena_bytes(count, n, layout, &need);
    if (rc)
        return rc;
    if (!rho || !seed || !d_arena || !d_trace)
        return fail(BML_EINVAL, "NULL rho, seed, arena or trace");
    if (!aligned256(d_arena) || !aligned256(d_trace))
        return fail(BML_EINVAL, "arena and trace must be 256-byte aligned");
    if (arena_bytes < need)
        return fail(BML_EINVAL, "arena of %zu bytes is smaller than the %zu needed", arena_bytes,
                    need);
    if (trace_steps < 1 || trace_steps > 0x7fffffff)
        return fail(BML_EINVAL, "trace_steps must be in [1, 2^31-1]");
    for (int b = 0; b < count; ++b)
        if (!(rho[b] >= 0.0 && rho[b] <= 1.0))
            return fail(BML_EINVAL, "lattice %d: rho must be in [0, 1]", b);

    bml_batch *B = new (std::nothrow) bml_batch();
    if (!B)
        return fail(BML_EDEVICE, "out of host memory");
    B->count = count;
    B->layout = layout;
    B->n.assign(n, n + count);
    B->trace = d_trace;
    B->trace_steps = trace_steps;
    B->stream = (hipStream_t)hip_stream;
    B->t_phases = 16;
    B->active.assign(count, 1);
    B->parity_base.assign(count, 0);
    B->pass_base.assign(count, 0);
    B->steps.assign(count, 0);
    B->n_lr0.assign(count, 0);
    B->n_tb0.assign(count, 0);
    auto bail = [&](int code) {
        batch_release(B);
        return code;
    };
    if ((rc = device_info(&B->dev)))
        return bail(rc);
    uint8_t *p = (uint8_t *)d_arena;
    for (int b = 0; b < count; ++b) {
        const size_t sb = round256(lattice_state_bytes(n[b], layout));
        B->buf[0].push_back(p);
        B->buf[1].push_back(p + sb);
        p += 2 * sb;
    }
    if (hipMalloc(&B->d_lat, count * sizeof(BatchLattice)) != hipSuccess ||
        hipMalloc(&B->d_ctr, sizeof(BatchCounters)) != hipSuccess ||
        hipMalloc(&B->d_counts, (size_t)count * 2 * sizeof(unsigned long long)) != hipSuccess)
        return bail(fail(BML_EDEVICE, "hipMalloc of batch scratch failed"));
    if (layout == BML_LAYOUT_BITPLANE) {
        // bml_batch_get_cells unpacks through this buffer, whole rows at a
        // time: the largest lattice, or 16 MiB (at least one row)
        const int nmax = *std::max_element(n, n + count);
        B->stage_bytes = std::max<size_t>((size_t)nmax,
                                          std::min<size_t>((size_t)nmax * nmax, 16u << 20));
        if (hipMalloc(&B->d_stage, B->stage_bytes) != hipSuccess) {
            B->d_stage = nullptr;
            return bail(fail(BML_EDEVICE, "hipMalloc of the read-back staging buffer failed"));
        }
    }
    for (int b = 0; b < count; ++b) {
        if ((rc = launch_init(B->buf[0][b], n[b], n[b], layout, seed[b], rho[b] * 0.5, rho[b] * 0.5,
                               B->stream)))
            return bail(rc);
        if ((rc = launch_count(B->buf[0][b], n[b], n[b], layout, B->d_counts + 2 * b, B->stream)))
            return bail(rc);
    }
    std::vector<unsigned long long> h((size_t)count * 2);
    if (hipMemcpyAsync(h.data(), B->d_counts, h.size() * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, B->stream) != hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess)
        return bail(fail(BML_EDEVICE, "initial counts of the batch failed"));
    for (int b = 0; b < count; ++b) {
        B->n_lr0[b] = h[2 * b];
        B->n_tb0[b] = h[2 * b + 1];
    }
    if ((rc = upload_work(B)))
        return bail(rc);
    {
        std::lock_guard<std::mutex> lock(g_batch_mu);
        g_batches.insert(B);
    }
    *out = B;
    return BML_OK;
}

int bml_batch_set_tuning(bml_batch *B, int32_t strip_rows, int32_t t_phases,
                         int32_t waves_per_block)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    const int R = strip_rows > 0 ? strip_rows : B->strip_target;
    const int T = t_phases > 0 ? t_phases : B->t_phases;
    const int W = waves_per_block > 0 ? waves_per_block : B->wpb;
    if (R < 1 || R > 65504)
        return fail(BML_EINVAL, "strip_rows=%d must be in [1, 65504]", R);
    if (T < 2 || T > 2 * MAX_K || T % 2)
        return fail(BML_EINVAL, "t_phases=%d must be even in [2, %d]", T, 2 * MAX_K);
    if (W != 1 && W != 2 && W != 4)
        return fail(BML_EINVAL, "waves_per_block=%d must be 1, 2 or 4", W);
    B->strip_target = R;
    B->t_phases = T;
    B->wpb = W;
    if (B->graph_exec) {
        (void)hipGraphExecDestroy(B->graph_exec);
        (void)hipGraphDestroy(B->graph);
        B->graph_exec = nullptr;
        B->graph = nullptr;
    }
    return upload_work(B);
}

int bml_batch_set_resident(bml_batch *B, int32_t max_n, int32_t split_steps)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    if (max_n < 0 || max_n > 32 * RES_MAX_WORDS)
        return fail(BML_EINVAL, "max_n=%d must be in [0, %d]", max_n, 32 * RES_MAX_WORDS);
    if (split_steps < 0 || split_steps > RES_MAX_SPLIT || split_steps % 16)
        return fail(BML_EINVAL, "split_steps=%d must be 0 or a multiple of 16 up to %d",
                    split_steps, RES_MAX_SPLIT);
    B->resident_max_n = max_n;
    B->resident_split = split_steps;
    B->res_grid = 0;
    if (B->graph_exec) {
        (void)hipGraphExecDestroy(B->graph_exec);
        (void)hipGraphDestroy(B->graph);
        B->graph_exec = nullptr;
        B->graph = nullptr;
    }
    return upload_work(B);
}

int bml_batch_get_resident(const bml_batch *B)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    return use_resident(B) ? 1 : 0;
}

int bml_batch_set_active(bml_batch *B, const uint8_t *active_host)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    for (int b = 0; b < B->count; ++b) {
        const uint8_t want = active_host ? (active_host[b] ? 1 : 0) : 1;
        if (want == B->active[b])
            continue;
        // Freeze or restart the parity bookkeeping at the current pass.
        B->parity_base[b] = lattice_parity(B, b);
        B->pass_base[b] = (int32_t)B->host_pass;
        B->active[b] = want;
    }
    return upload_work(B);
}

int bml_batch_run(bml_batch *B, int64_t n_steps)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    if (n_steps < 0)
        return fail(BML_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0)
        return BML_OK;
    int64_t passes = 0;
    int rc = enqueue_run(B, n_steps, &passes);
    if (rc)
        return rc;
    account_run(B, n_steps, passes);
    return BML_OK;
}

int bml_batch_capture(bml_batch *B, int64_t n_steps)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    if (n_steps < 1)
        return fail(BML_EINVAL, "n_steps must be >= 1");
    if (!B->stream)
        return fail(BML_EINVAL, "graph capture needs a non-null stream");
    if (B->graph_exec) {
        (void)hipGraphExecDestroy(B->graph_exec);
        (void)hipGraphDestroy(B->graph);
        B->graph_exec = nullptr;
        B->graph = nullptr;
    }
    // Resolve the occupancy queries before capturing.
    const int io = B->layout == BML_LAYOUT_U8 ? IO_U8 : IO_BP;
    for (int k = 1; k <= MAX_K; ++k) {
        int nb;
        int rc = batch_blocks_per_cu(io, k, 64 * B->wpb, &nb);
        if (rc)
            return rc;
    }
    BML_HIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeRelaxed));
    int64_t passes = 0;
    int rc = enqueue_run(B, n_steps, &passes);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->stream, &g);
    if (rc) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return fail(BML_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&B->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(BML_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    B->graph = g;
    B->graph_steps = n_steps;
    B->graph_passes = passes;
    return BML_OK;
}

int bml_batch_replay(bml_batch *B)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    if (!B->graph_exec)
        return fail(BML_ESTATE, "no captured run");
    BML_HIP(hipGraphLaunch(B->graph_exec, B->stream));
    account_run(B, B->graph_steps, B->graph_passes);
    return BML_OK;
}

int64_t bml_batch_step_count(const bml_batch *B) { return batch_live(B) ? B->host_step : -1; }

int bml_batch_lattice_steps(const bml_batch *B, int32_t idx, int64_t *steps)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    if (idx < 0 || idx >= B->count || !steps)
        return fail(BML_EINVAL, "bad lattice index or NULL output");
    *steps = B->steps[idx];
    return BML_OK;
}

int bml_batch_initial_counts(const bml_batch *B, int32_t idx, uint64_t *n_lr, uint64_t *n_tb)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    if (idx < 0 || idx >= B->count)
        return fail(BML_EINVAL, "bad lattice index");
    if (n_lr)
        *n_lr = B->n_lr0[idx];
    if (n_tb)
        *n_tb = B->n_tb0[idx];
    return BML_OK;
}

int bml_batch_get_cells(bml_batch *B, int32_t idx, uint8_t *out_host)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    if (idx < 0 || idx >= B->count || !out_host)
        return fail(BML_EINVAL, "bad lattice index or NULL output");
    const int n = B->n[idx];
    const void *state = B->buf[lattice_parity(B, idx)][idx];
    const size_t cells = (size_t)n * n;
    if (B->layout == BML_LAYOUT_U8) {
        BML_HIP(hipMemcpyAsync(out_host, state, cells, hipMemcpyDeviceToHost, B->stream));
        BML_HIP(hipStreamSynchronize(B->stream));
        return BML_OK;
    }
    // unpack whole rows at a time through the staging buffer; stream order
    // keeps each chunk's copy ahead of the next unpack
    const int64_t words = n / 32;
    const int64_t plane_words = (int64_t)n * words;
    const uint32_t *lr = (const uint32_t *)state;
    const int64_t chunk = std::max<int64_t>(1, (int64_t)(B->stage_bytes / (size_t)n));
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t nr = std::min<int64_t>(chunk, n - r0);
        int rc = launch_unpack_rows(lr + r0 * words, lr + plane_words + r0 * words, B->d_stage,
                                    nr * words, B->stream);
        if (rc)
            return rc;
        BML_HIP(hipMemcpyAsync(out_host + r0 * n, B->d_stage, (size_t)(nr * n),
                               hipMemcpyDeviceToHost, B->stream));
    }
    BML_HIP(hipStreamSynchronize(B->stream));
    return BML_OK;
}

int bml_batch_check(bml_batch *B)
{
    clear_error();
    if (!batch_live(B))
        return fail(BML_ESTATE, "invalid batch handle");
    for (int b = 0; b < B->count; ++b) {
        int rc = launch_count(B->buf[lattice_parity(B, b)][b], B->n[b], B->n[b], B->layout,
                              B->d_counts + 2 * b, B->stream);
        if (rc)
            return rc;
    }
    std::vector<unsigned long long> h((size_t)B->count * 2);
    BML_HIP(hipMemcpyAsync(h.data(), B->d_counts, h.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, B->stream));
    BML_HIP(hipStreamSynchronize(B->stream));
    for (int b = 0; b < B->count; ++b)
        if (h[2 * b] != B->n_lr0[b] || h[2 * b + 1] != B->n_tb0[b])
            return fail(BML_ECORRUPT, "lattice %d: car counts (%llu, %llu) differ from (%llu, %llu)",
                        b, h[2 * b], h[2 * b + 1], (unsigned long long)B->n_lr0[b],
                        (unsigned long long)B->n_tb0[b]);
    return BML_OK;
}

void bml_batch_free(bml_batch *B)
{
    if (!batch_live(B))
        return;
    {
        std::lock_guard<std::mutex> lock(g_batch_mu);
        g_batches.erase(B);
    }
    (void)hipStreamSynchronize(B->stream);
    batch_release(B);
}

} // extern "C"
