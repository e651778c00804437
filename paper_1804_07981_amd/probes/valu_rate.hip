// valu_rate.hip -- issue rate of the vector ALU instructions the step
// kernels are made of, on gfx950: each kernel runs 20000 x 32 register-only
// instructions per lane (eight independent chains, or one dependent chain)
// with 1, 2, 4 or 8 waves per SIMD (1024 x w one-wave workgroups over 256
// CUs), and prints the time per wave64 instruction per SIMD.  The ALU
// roofline of the library counts its operations in full-rate slots from
// these rates.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       valu_rate.hip -o valu_rate && ./valu_rate
#include <hip/hip_runtime.h>
#include <stdio.h>
#define REP4(x) x x x x
__global__ void xor8(unsigned *out, int iters) {   // 8 independent chains
    unsigned a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7, b = blockIdx.x;
    for (int i = 0; i < iters; ++i) {
        asm volatile(REP4("v_xor_b32 %0, %0, %8\nv_xor_b32 %1, %1, %8\nv_xor_b32 %2, %2, %8\nv_xor_b32 %3, %3, %8\nv_xor_b32 %4, %4, %8\nv_xor_b32 %5, %5, %8\nv_xor_b32 %6, %6, %8\nv_xor_b32 %7, %7, %8\n")
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7) : "v"(b));
    }
    out[blockIdx.x * 64 + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}
__global__ void bit8(unsigned *out, int iters) {   // 8 independent v_bitop3 chains
    unsigned a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7, b = blockIdx.x, c = 5;
    for (int i = 0; i < iters; ++i) {
        asm volatile(REP4("v_bitop3_b32 %0, %0, %8, %9 bitop3:0x96\nv_bitop3_b32 %1, %1, %8, %9 bitop3:0x96\nv_bitop3_b32 %2, %2, %8, %9 bitop3:0x96\nv_bitop3_b32 %3, %3, %8, %9 bitop3:0x96\nv_bitop3_b32 %4, %4, %8, %9 bitop3:0x96\nv_bitop3_b32 %5, %5, %8, %9 bitop3:0x96\nv_bitop3_b32 %6, %6, %8, %9 bitop3:0x96\nv_bitop3_b32 %7, %7, %8, %9 bitop3:0x96\n")
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7) : "v"(b), "v"(c));
    }
    out[blockIdx.x * 64 + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}
__global__ void bcnt8(unsigned *out, int iters) {  // 8 independent popcount-accumulate chains
    unsigned a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7, b = blockIdx.x * 77;
    for (int i = 0; i < iters; ++i) {
        asm volatile(REP4("v_bcnt_u32_b32 %0, %8, %0\nv_bcnt_u32_b32 %1, %8, %1\nv_bcnt_u32_b32 %2, %8, %2\nv_bcnt_u32_b32 %3, %8, %3\nv_bcnt_u32_b32 %4, %8, %4\nv_bcnt_u32_b32 %5, %8, %5\nv_bcnt_u32_b32 %6, %8, %6\nv_bcnt_u32_b32 %7, %8, %7\n")
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7) : "v"(b));
    }
    out[blockIdx.x * 64 + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}
__global__ void align8(unsigned *out, int iters) {  // 8 independent alignbit chains
    unsigned a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7, b = blockIdx.x * 77;
    for (int i = 0; i < iters; ++i) {
        asm volatile(REP4("v_alignbit_b32 %0, %0, %8, 1\nv_alignbit_b32 %1, %1, %8, 1\nv_alignbit_b32 %2, %2, %8, 1\nv_alignbit_b32 %3, %3, %8, 1\nv_alignbit_b32 %4, %4, %8, 1\nv_alignbit_b32 %5, %5, %8, 1\nv_alignbit_b32 %6, %6, %8, 1\nv_alignbit_b32 %7, %7, %8, 1\n")
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7) : "v"(b));
    }
    out[blockIdx.x * 64 + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}
__global__ void xor1(unsigned *out, int iters) {   // one dependent chain
    unsigned a = threadIdx.x, b = blockIdx.x;
    for (int i = 0; i < iters; ++i) {
        asm volatile(REP4("v_xor_b32 %0, %0, %1\nv_xor_b32 %0, %0, %1\nv_xor_b32 %0, %0, %1\nv_xor_b32 %0, %0, %1\nv_xor_b32 %0, %0, %1\nv_xor_b32 %0, %0, %1\nv_xor_b32 %0, %0, %1\nv_xor_b32 %0, %0, %1\n") : "+v"(a) : "v"(b));
    }
    out[blockIdx.x * 64 + threadIdx.x] = a;
}
typedef void (*K)(unsigned *, int);
int main() {
    unsigned *out; (void)hipMalloc(&out, 8192 * 64 * 4);
    const int iters = 20000;   // 32 instructions per iteration
    K ks[] = {xor8, bit8, bcnt8, align8, xor1};
    const char *names[] = {"xor x8", "bitop3 x8", "bcnt x8", "alignbit x8", "xor dep"};
    hipEvent_t e0, e1; (void)hipEventCreate(&e0); (void)hipEventCreate(&e1);
    for (int k = 0; k < 5; ++k)
        for (int w = 1; w <= 8; w *= 2) {
            const int blocks = 1024 * w;    // 4 waves per CU per w, 256 CUs
            for (int rep = 0; rep < 2; ++rep) {
                (void)hipEventRecord(e0);
                hipLaunchKernelGGL(ks[k], dim3(blocks), dim3(64), 0, 0, out, iters);
                (void)hipEventRecord(e1);
                (void)hipEventSynchronize(e1);
                float ms; (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep) {
                    const double per_simd = ms * 1e6 / ((double)iters * 32 * w);   // ns per instruction per SIMD
                    printf("%-12s %d wave/SIMD: %.3f ms, %.3f ns per wave64 instruction per SIMD (%.2f cycles at 2.4 GHz)\n",
                           names[k], w, ms, per_simd, per_simd * 2.4);
                }
            }
        }
    (void)hipFree(out);
    return 0;
}
