// bml_mlp.hip -- the learned early exit: trajectory features and a small
// MLP (65 -> 64 -> 64 -> 1, ReLU, logit) trained in fp32 and run in BF16,
// all in hand-written HIP kernels.
//
// The physics it predicts (Marzolla, arXiv:1804.07981, Sec. 2): below a
// critical density the lattice self-organises into free flow (every car
// moves), above it a global jam forms and motion stops; near the critical
// point both outcomes can occur.  The network reads the early trajectory of
// the mobile fraction and the density and predicts the final phase.
//
// Parameter vector (fp32, BML_MLP_PARAMS = 8449 entries, row-major out x in):
//   W1[64][65] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3
#include <hip/hip_runtime.h>

#include <math.h>

#include "bml.h"
#include "bml_common.hpp"

namespace bml {

constexpr int NI = BML_MLP_INPUTS;   // 65
constexpr int NH = BML_MLP_HIDDEN;   // 64
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NH * NI;
constexpr int OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + NH;
constexpr int NP = OFF_B3 + 1;
static_assert(NP == BML_MLP_PARAMS, "parameter layout");
constexpr int MAX_BATCH = 256;

// ---------------------------------------------------------------------------
// Features: f_m = sum over steps 8m+1 .. 8m+8 of (LR moved + TB moved),
// divided by 8 * (number of cars), m = 0..63 (the mobile fraction averaged
// over windows of 8 steps), computed in double and rounded to float; f_64 =
// rho.  A lattice without cars has mobile fraction 1 by definition.  One
// thread per (lattice, feature).
// ---------------------------------------------------------------------------
__global__ void features_kernel(const uint32_t *trace, int64_t trace_steps, int32_t count,
                                const uint64_t *cars, const double *rho, int32_t window,
                                float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)count * NI)
        return;
    const int64_t b = i / NI;
    const int m = (int)(i - b * NI);
    if (m == NI - 1) {
        out[i] = (float)rho[b];
        return;
    }
    const uint64_t c = cars[b];
    if (c == 0) {
        out[i] = 1.0f;
        return;
    }
    uint64_t moved = 0;
    for (int s = m * window; s < (m + 1) * window; ++s) {
        const uint32_t *p = trace + (b * trace_steps + s) * 2;
        moved += (uint64_t)p[0] + p[1];
    }
    out[i] = (float)((double)moved / ((double)window * (double)c));
}

// frozen[b] = 1 if some step s in [s0, s1) of lattice b moved no car.  A
// step without moves leaves the lattice unchanged, so it stays frozen for
// good (the exact stop rule).  One wave per lattice.
__global__ __launch_bounds__(256) void trace_frozen_kernel(const uint32_t *trace,
                                                           int64_t trace_steps, int32_t count,
                                                           int64_t s0, int64_t s1,
                                                           uint8_t *frozen)
{
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x / 64);
    if (b >= count)
        return;
    const int lane = threadIdx.x & 63;
    int any = 0;
    for (int64_t s = s0 + lane; s < s1; s += 64) {
        const uint32_t *p = trace + (b * trace_steps + s) * 2;
        any |= (p[0] + p[1]) == 0u;
    }
    const unsigned long long m = __ballot(any);
    if (lane == 0)
        frozen[b] = m ? 1 : 0;
}

// mean[b] = mean over steps [s0, s1) of (LR moved + TB moved) / cars[b]
// (1 for a lattice without cars), in double.  One wave per lattice.
__global__ __launch_bounds__(256) void trace_mobility_kernel(const uint32_t *trace,
                                                             int64_t trace_steps, int32_t count,
                                                             const uint64_t *cars, int64_t s0,
                                                             int64_t s1, double *mean)
{
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x / 64);
    if (b >= count)
        return;
    const int lane = threadIdx.x & 63;
    unsigned long long moved = 0;
    for (int64_t s = s0 + lane; s < s1; s += 64) {
        const uint32_t *p = trace + (b * trace_steps + s) * 2;
        moved += (unsigned long long)p[0] + p[1];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        moved += __shfl_xor(moved, off, 64);
    if (lane == 0)
        mean[b] = cars[b] ? (double)moved / ((double)(s1 - s0) * (double)cars[b]) : 1.0;
}

// Column means and standard deviations (population, double accumulation) of
// x[n][NI]; one block per column.
__global__ __launch_bounds__(256) void feature_stats_kernel(const float *x, int32_t n,
                                                           float *mean, float *stdev)
{
    __shared__ double s1[256], s2[256];
    const int col = blockIdx.x;
    double a = 0, q = 0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const double v = x[(int64_t)r * NI + col];
        a += v;
        q += v * v;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = q;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = s1[0] / n;
        const double var = fmax(s2[0] / n - m * m, 0.0);
        mean[col] = (float)m;
        // A constant column is left unscaled.
        stdev[col] = var > 1e-24 ? (float)sqrt(var) : 1.0f;
    }
}

// x[i][c] = (x[i][c] - mean[c]) / stdev[c] in float.
__global__ void standardize_kernel(float *x, int32_t n, const float *mean, const float *stdev)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * NI)
        return;
    const int c = (int)(i % NI);
    x[i] = (x[i] - mean[c]) / stdev[c];
}

// ---------------------------------------------------------------------------
// Training: one block of MAX_BATCH threads runs the minibatch forward and
// back (thread i = sample i) and parks each sample's activations and
// pre-activation gradients in global scratch; then one thread per parameter
// (a grid over all NP parameters) sums its products over the samples and,
// for a training step, applies Adam.
// ---------------------------------------------------------------------------
struct SampleScratch {       // per sample, in global memory
    float x[NI];
    float h1[NH];
    float d1[NH];            // dL/d(pre-activation of layer 1)
    float h2[NH];
    float d2[NH];            // dL/d(pre-activation of layer 2)
    float dz;                // dL/dz
};

__device__ __forceinline__ float bce_with_logits(float z, float y)
{
    // max(z, 0) - z*y + log(1 + exp(-|z|)), stable for any z.
    return fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
}

__device__ __forceinline__ float sigmoidf(float z)
{
    return z >= 0.0f ? 1.0f / (1.0f + expf(-z)) : expf(z) / (1.0f + expf(z));
}


// Forward and backward of samples idx[0..n) (idx NULL = 0..n-1) of the mean
// BCE-with-logits loss: per-sample activations and pre-activation gradients
// into scr[0..n); the loss summed over each block's samples into
// part[block] (the parameter kernel adds the blocks in order).
//
// A block takes SPB = 64 samples with four threads each; thread (s, q) owns
// hidden units 16q .. 16q+15 of sample s in both layers.  The inputs, the
// layer-1 activations and the layer-2 gradients of the block's samples are
// staged in LDS (rows padded to an odd stride), so every per-thread loop
// over a vector reads LDS and the only register arrays are the thread's 16
// accumulators, indexed by unrolled constants.  Each weighted sum runs over
// its inputs in ascending order; the output logit adds the four threads'
// partial sums in thread order.
constexpr int SPB = 64;                  // samples per block (256 threads)
constexpr int UPT = NH / 4;              // hidden units per thread
constexpr int XS = NI;                   // staged input row stride (65)
constexpr int HS = NH + 1;               // staged hidden row stride (65)
static_assert(MAX_BATCH % SPB == 0 && (MAX_BATCH / SPB) * sizeof(float) <= 64,
              "loss partials fit the scratch tail");

__global__ __launch_bounds__(256) void mlp_sample_kernel(const float *params, const float *x,
                                                         const float *y, const int32_t *idx,
                                                         int32_t n, SampleScratch *scr,
                                                         float *part)
{
    __shared__ float P[NP];
    __shared__ float xs[SPB * XS];
    __shared__ float h1s[SPB * HS];
    __shared__ float d2s[SPB * HS];
    __shared__ float ls[SPB];
    const int s = threadIdx.x >> 2, q = threadIdx.x & 3;
    const int i = blockIdx.x * SPB + s;
    const bool live = i < n;
    for (int p = threadIdx.x; p < NP; p += blockDim.x)
        P[p] = params[p];
    for (int e = threadIdx.x; e < SPB * NI; e += blockDim.x) {
        const int ss = e / NI, c = e - ss * NI;
        const int ii = blockIdx.x * SPB + ss;
        float v = 0.0f;
        if (ii < n) {
            v = x[(int64_t)(idx ? idx[ii] : ii) * NI + c];
            scr[ii].x[c] = v;
        }
        xs[ss * XS + c] = v;
    }
    __syncthreads();
    const int u0 = q * UPT;
    SampleScratch *sc = scr + (live ? i : 0);   // dereferenced only when live

    // layer 1: h1 = relu(W1 x + b1)
    {
        float a[UPT];
#pragma unroll
        for (int u = 0; u < UPT; ++u)
            a[u] = P[OFF_B1 + u0 + u];
        for (int c = 0; c < NI; ++c) {
            const float xv = xs[s * XS + c];
#pragma unroll
            for (int u = 0; u < UPT; ++u)
                a[u] = fmaf(P[OFF_W1 + (u0 + u) * NI + c], xv, a[u]);
        }
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const float h = fmaxf(a[u], 0.0f);
            h1s[s * HS + u0 + u] = h;
            if (live)
                sc->h1[u0 + u] = h;
        }
    }
    __syncthreads();

    // layer 2 and the output: h2 = relu(W2 h1 + b2), z = w3 . h2 + b3
    float g[UPT];
    uint32_t active = 0;
    float zp = 0.0f;
    {
        float a[UPT];
#pragma unroll
        for (int u = 0; u < UPT; ++u)
            a[u] = P[OFF_B2 + u0 + u];
        for (int c = 0; c < NH; ++c) {
            const float hv = h1s[s * HS + c];
#pragma unroll
            for (int u = 0; u < UPT; ++u)
                a[u] = fmaf(P[OFF_W2 + (u0 + u) * NH + c], hv, a[u]);
        }
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            g[u] = fmaxf(a[u], 0.0f);
            if (live)
                sc->h2[u0 + u] = g[u];
            active |= (uint32_t)(g[u] > 0.0f) << u;
            zp = fmaf(P[OFF_W3 + u0 + u], g[u], zp);
        }
    }
    const int quad = (threadIdx.x & 63) & ~3;   // lane of thread (s, 0)
    float z = P[OFF_B3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        z += __shfl(zp, quad + k, 64);
    const float yi = live ? y[idx ? idx[i] : i] : 0.0f;
    const float li = live ? bce_with_logits(z, yi) : 0.0f;
    const float dz = live ? (sigmoidf(z) - yi) / (float)n : 0.0f;
    if (live && q == 0)
        sc->dz = dz;

    // backward: d2 = dz w3 on active units; d1 = (W2^T d2) on active
    // layer-1 units, the sum over j in ascending order
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const float d2 = ((active >> u) & 1u) ? dz * P[OFF_W3 + u0 + u] : 0.0f;
        d2s[s * HS + u0 + u] = d2;
        if (live)
            sc->d2[u0 + u] = d2;
    }
    __syncthreads();
    {
        float a[UPT];
#pragma unroll
        for (int u = 0; u < UPT; ++u)
            a[u] = 0.0f;
        for (int j = 0; j < NH; ++j) {
            const float dv = d2s[s * HS + j];
#pragma unroll
            for (int u = 0; u < UPT; ++u)
                a[u] = fmaf(P[OFF_W2 + j * NH + u0 + u], dv, a[u]);
        }
#pragma unroll
        for (int u = 0; u < UPT; ++u)
            if (live)
                sc->d1[u0 + u] = h1s[s * HS + u0 + u] > 0.0f ? a[u] : 0.0f;
    }
    if (q == 0)
        ls[s] = li;
    __syncthreads();
    if (threadIdx.x == 0) {
        float sum = 0.0f;
        for (int k = 0; k < SPB; ++k)
            sum += ls[k];
        part[blockIdx.x] = sum;
    }
}

// Parameter gradients, one thread per parameter: the sum over samples
// k = 0, 1, ..., n-1 (in that order) of its product of a pre-activation
// gradient and an input (weights) or of the gradient alone (biases), into
// grad[p].  With m != NULL also one Adam step (Kingma & Ba):
// m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, and
// theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  Thread 0
// also writes the mean loss.
__global__ __launch_bounds__(256) void mlp_param_kernel(const SampleScratch *scr, int32_t n,
                                                        float *grad, float *params, float *m,
                                                        float *v, int64_t t, float lr,
                                                        float beta1, float beta2, float eps,
                                                        const float *part, float *loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss) {
        // mean loss: the sample blocks' sums, added in block order
        float sum = 0.0f;
        for (int b = 0; b < (n + SPB - 1) / SPB; ++b)
            sum += part[b];
        *loss = sum / (float)n;
    }
    if (p >= NP)
        return;
    float g = 0.0f;
    if (p < OFF_B1) {
        const int j = p / NI, c = p - j * NI;
#pragma unroll 8
        for (int k = 0; k < n; ++k)
            g = fmaf(scr[k].d1[j], scr[k].x[c], g);
    } else if (p < OFF_W2) {
        const int j = p - OFF_B1;
#pragma unroll 8
        for (int k = 0; k < n; ++k)
            g += scr[k].d1[j];
    } else if (p < OFF_B2) {
        const int j = (p - OFF_W2) / NH, c = (p - OFF_W2) - j * NH;
#pragma unroll 8
        for (int k = 0; k < n; ++k)
            g = fmaf(scr[k].d2[j], scr[k].h1[c], g);
    } else if (p < OFF_W3) {
        const int j = p - OFF_B2;
#pragma unroll 8
        for (int k = 0; k < n; ++k)
            g += scr[k].d2[j];
    } else if (p < OFF_B3) {
        const int c = p - OFF_W3;
#pragma unroll 8
        for (int k = 0; k < n; ++k)
            g = fmaf(scr[k].dz, scr[k].h2[c], g);
    } else {
#pragma unroll 8
        for (int k = 0; k < n; ++k)
            g += scr[k].dz;
    }
    grad[p] = g;
    if (m) {
        const float c1 = 1.0f - powf(beta1, (float)t);
        const float c2 = 1.0f - powf(beta2, (float)t);
        const float mp = beta1 * m[p] + (1.0f - beta1) * g;
        const float vp = beta2 * v[p] + (1.0f - beta2) * g * g;
        m[p] = mp;
        v[p] = vp;
        params[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// Inference: one thread per sample, parameters in LDS.  fp32 version and a
// BF16 version in which the weights and each layer's input are rounded to
// bfloat16 (round to nearest even) and products are accumulated in fp32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)       // inf / nan pass through
        return __uint_as_float(u & 0xffff0000u);
    u += 0x7fffu + ((u >> 16) & 1u);             // round to nearest, ties to even
    return __uint_as_float(u & 0xffff0000u);
}

template <bool BF16>
__global__ __launch_bounds__(256) void mlp_infer_kernel(const float *params, const float *x,
                                                        int32_t n, float *logits)
{
    __shared__ float P[NP];
    for (int p = threadIdx.x; p < NP; p += blockDim.x)
        P[p] = BF16 && (p < OFF_B1 || (p >= OFF_W2 && p < OFF_B2) || (p >= OFF_W3 && p < OFF_B3))
                   ? to_bf16(params[p])
                   : params[p];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    // fixed trip counts, unrolled: the vectors stay in registers
    float xi[NI];
#pragma unroll
    for (int c = 0; c < NI; ++c)
        xi[c] = BF16 ? to_bf16(x[i * NI + c]) : x[i * NI + c];
    float h1[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float a = P[OFF_B1 + j];
#pragma unroll
        for (int c = 0; c < NI; ++c)
            a = fmaf(P[OFF_W1 + j * NI + c], xi[c], a);
        a = fmaxf(a, 0.0f);
        h1[j] = BF16 ? to_bf16(a) : a;
    }
    float h2[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float a = P[OFF_B2 + j];
#pragma unroll
        for (int c = 0; c < NH; ++c)
            a = fmaf(P[OFF_W2 + j * NH + c], h1[c], a);
        a = fmaxf(a, 0.0f);
        h2[j] = BF16 ? to_bf16(a) : a;
    }
    float z = P[OFF_B3];
#pragma unroll
    for (int c = 0; c < NH; ++c)
        z = fmaf(P[OFF_W3 + c], h2[c], z);
    logits[i] = z;
}

} // namespace bml

using namespace bml;

static int grid_for(int64_t work, unsigned *g)
{
    const int64_t b = (work + 255) / 256;
    if (b > 0x7fffffff)
        return fail(BML_EINVAL, "launch too large");
    *g = (unsigned)(b > 0 ? b : 1);
    return BML_OK;
}

extern "C" {

int bml_features(const uint32_t *d_trace, int64_t trace_steps, int32_t count,
                 const uint64_t *d_cars, const double *d_rho, int32_t window,
                 float *d_out, void *hip_stream)
{
    clear_error();
    if (!d_trace || !d_cars || !d_rho || !d_out || count < 1 || window < 1 ||
        (int64_t)window * (NI - 1) > trace_steps)
        return fail(BML_EINVAL, "bml_features: bad arguments (64 windows must fit the trace)");
    unsigned g;
    int rc = grid_for((int64_t)count * NI, &g);
    if (rc)
        return rc;
    hipLaunchKernelGGL(features_kernel, dim3(g), dim3(256), 0, (hipStream_t)hip_stream, d_trace,
                       trace_steps, count, d_cars, d_rho, window, d_out);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_trace_frozen(const uint32_t *d_trace, int64_t trace_steps, int32_t count,
                     int64_t first_step, int64_t end_step, uint8_t *d_frozen, void *hip_stream)
{
    clear_error();
    if (!d_trace || !d_frozen || count < 1 || first_step < 0 || end_step < first_step ||
        end_step > trace_steps)
        return fail(BML_EINVAL, "bml_trace_frozen: bad arguments");
    const unsigned g = (unsigned)((count + 3) / 4);
    hipLaunchKernelGGL(trace_frozen_kernel, dim3(g), dim3(256), 0, (hipStream_t)hip_stream,
                       d_trace, trace_steps, count, first_step, end_step, d_frozen);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_trace_mobility(const uint32_t *d_trace, int64_t trace_steps, int32_t count,
                       const uint64_t *d_cars, int64_t first_step, int64_t end_step,
                       double *d_mean, void *hip_stream)
{
    clear_error();
    if (!d_trace || !d_cars || !d_mean || count < 1 || first_step < 0 ||
        end_step <= first_step || end_step > trace_steps)
        return fail(BML_EINVAL, "bml_trace_mobility: bad arguments");
    const unsigned g = (unsigned)((count + 3) / 4);
    hipLaunchKernelGGL(trace_mobility_kernel, dim3(g), dim3(256), 0, (hipStream_t)hip_stream,
                       d_trace, trace_steps, count, d_cars, first_step, end_step, d_mean);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_feature_stats(const float *d_x, int32_t n, float *d_mean, float *d_std,
                      void *hip_stream)
{
    clear_error();
    if (!d_x || !d_mean || !d_std || n < 1)
        return fail(BML_EINVAL, "bml_feature_stats: bad arguments");
    hipLaunchKernelGGL(feature_stats_kernel, dim3(NI), dim3(256), 0, (hipStream_t)hip_stream,
                       d_x, n, d_mean, d_std);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_standardize(float *d_x, int32_t n, const float *d_mean, const float *d_std,
                    void *hip_stream)
{
    clear_error();
    if (!d_x || !d_mean || !d_std || n < 1)
        return fail(BML_EINVAL, "bml_standardize: bad arguments");
    unsigned g;
    int rc = grid_for((int64_t)n * NI, &g);
    if (rc)
        return rc;
    hipLaunchKernelGGL(standardize_kernel, dim3(g), dim3(256), 0, (hipStream_t)hip_stream, d_x,
                       n, d_mean, d_std);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

// Per-sample records, then the loss partial of every sample block.
size_t bml_mlp_scratch_bytes(void) { return sizeof(SampleScratch) * MAX_BATCH + 64; }

static float *loss_parts(void *d_scratch)
{
    return reinterpret_cast<float *>(static_cast<SampleScratch *>(d_scratch) + MAX_BATCH);
}

int bml_mlp_grad(const float *d_params, const float *d_x, const float *d_y, int32_t n,
                 void *d_scratch, float *d_grad, float *d_loss, void *hip_stream)
{
    clear_error();
    if (!d_params || !d_x || !d_y || !d_scratch || !d_grad || n < 1 || n > MAX_BATCH)
        return fail(BML_EINVAL, "bml_mlp_grad: bad arguments (1 <= n <= %d)", MAX_BATCH);
    hipLaunchKernelGGL(mlp_sample_kernel, dim3((n + SPB - 1) / SPB), dim3(256), 0,
                       (hipStream_t)hip_stream, d_params, d_x, d_y, (const int32_t *)nullptr, n,
                       (SampleScratch *)d_scratch, loss_parts(d_scratch));
    BML_HIP(hipGetLastError());
    hipLaunchKernelGGL(mlp_param_kernel, dim3((NP + 255) / 256), dim3(256), 0,
                       (hipStream_t)hip_stream, (const SampleScratch *)d_scratch, n, d_grad,
                       (float *)nullptr, (float *)nullptr, (float *)nullptr, (int64_t)0, 0.0f,
                       0.0f, 0.0f, 0.0f, (const float *)loss_parts(d_scratch), d_loss);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_mlp_train_step(float *d_params, float *d_m, float *d_v, float *d_grad, int64_t t,
                       const float *d_x, const float *d_y, const int32_t *d_idx, int32_t n,
                       float lr, float beta1, float beta2, float eps, void *d_scratch,
                       float *d_loss, void *hip_stream)
{
    clear_error();
    if (!d_params || !d_m || !d_v || !d_grad || !d_x || !d_y || !d_idx || !d_scratch ||
        n < 1 || n > MAX_BATCH || t < 1)
        return fail(BML_EINVAL, "bml_mlp_train_step: bad arguments (1 <= n <= %d, t >= 1)",
                    MAX_BATCH);
    hipLaunchKernelGGL(mlp_sample_kernel, dim3((n + SPB - 1) / SPB), dim3(256), 0,
                       (hipStream_t)hip_stream, d_params, d_x, d_y, d_idx, n,
                       (SampleScratch *)d_scratch, loss_parts(d_scratch));
    BML_HIP(hipGetLastError());
    hipLaunchKernelGGL(mlp_param_kernel, dim3((NP + 255) / 256), dim3(256), 0,
                       (hipStream_t)hip_stream, (const SampleScratch *)d_scratch, n, d_grad,
                       d_params, d_m, d_v, t, lr, beta1, beta2, eps,
                       (const float *)loss_parts(d_scratch), d_loss);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_mlp_forward(const float *d_params, const float *d_x, int32_t n, float *d_logits,
                    void *hip_stream)
{
    clear_error();
    if (!d_params || !d_x || !d_logits || n < 1)
        return fail(BML_EINVAL, "bml_mlp_forward: bad arguments");
    unsigned g;
    int rc = grid_for(n, &g);
    if (rc)
        return rc;
    hipLaunchKernelGGL(mlp_infer_kernel<false>, dim3(g), dim3(256), 0, (hipStream_t)hip_stream,
                       d_params, d_x, n, d_logits);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

int bml_mlp_infer_bf16(const float *d_params, const float *d_x, int32_t n, float *d_logits,
                       void *hip_stream)
{
    clear_error();
    if (!d_params || !d_x || !d_logits || n < 1)
        return fail(BML_EINVAL, "bml_mlp_infer_bf16: bad arguments");
    unsigned g;
    int rc = grid_for(n, &g);
    if (rc)
        return rc;
    hipLaunchKernelGGL(mlp_infer_kernel<true>, dim3(g), dim3(256), 0, (hipStream_t)hip_stream,
                       d_params, d_x, n, d_logits);
    BML_HIP(hipGetLastError());
    return BML_OK;
}

} // extern "C"
