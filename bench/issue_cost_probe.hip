// VALU issue cost of single gfx950 instructions, the basis of the walk's
// roofline: eight independent register chains of one instruction per lane,
// 1024-lane workgroups, two per CU (eight waves per SIMD), timed with HIP
// events; the cost is SIMD cycles per wave64 instruction at 2.4 GHz.  The
// instructions are written as inline assembly (register operands only, no
// memory access) so that the compiler neither folds nor re-selects them.
//
// Build and run (one GPU):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       bench/issue_cost_probe.hip -o /tmp/issue_cost_probe && /tmp/issue_cost_probe
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                        \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                               \
        }                                                                               \
    } while (0)

#define CHAINS(...) _Pragma("unroll") for (int c = 0; c < 8; ++c) asm volatile(__VA_ARGS__);

template <int OP>
__global__ __launch_bounds__(1024) void probe(uint32_t *out, int iters, float fa, float fb)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    float x[8];
    uint32_t u[8];
    double d[8];
    uint64_t q[8], m[8];
    float y[8], z[8], t[8], v[8];   // independent chains beside x and u (mixed probes)
    uint32_t u2[8];
    for (int c = 0; c < 8; ++c) {
        x[c] = 1.0f + (float)(threadIdx.x + c) * 1e-4f;
        y[c] = z[c] = t[c] = v[c] = x[c];
        u2[c] = gid * 40503u + c;
        u[c] = gid * 2654435761u + c;
        d[c] = 1.0 + (double)(threadIdx.x + c) * 1e-4;
        q[c] = gid + c;
        m[c] = 0;
    }
    const uint32_t ua = __float_as_uint(fa) | 1u, ub = __float_as_uint(fb);
    const double da = fa, db = fb;
    const uint64_t mask = 0x5555555555555555ull ^ (uint64_t)blockIdx.x;   // wave-uniform: an SGPR pair
    const float fs = __uint_as_float(__builtin_amdgcn_readfirstlane(ub));  // wave-uniform: an SGPR
    const uint32_t us = __builtin_amdgcn_readfirstlane(ua);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (OP == 0) CHAINS("v_fma_f32 %0, %0, %1, %2" : "+v"(x[c]) : "v"(fa), "v"(fb))
            if (OP == 1) CHAINS("v_add_f32 %0, %0, %1" : "+v"(x[c]) : "v"(fa))
            if (OP == 2) CHAINS("v_mul_f32 %0, %0, %1" : "+v"(x[c]) : "v"(fa))
            if (OP == 3) CHAINS("v_fma_f32 %0, %0, %1, %2" : "+v"(x[c]) : "s"(fs), "v"(fb))
            if (OP == 4) CHAINS("v_add_u32 %0, %0, %1" : "+v"(u[c]) : "v"(ua))
            if (OP == 5) CHAINS("v_xor_b32 %0, %0, %1" : "+v"(u[c]) : "v"(ua))
            if (OP == 6) CHAINS("v_add_u32 %0, %1, %0" : "+v"(u[c]) : "s"(us))
            if (OP == 7) CHAINS("v_mov_b32 %0, %1" : "=v"(u[c]) : "v"(u[(c + 1) & 7]))
            if (OP == 8) CHAINS("v_max_f32 %0, %0, %1" : "+v"(x[c]) : "v"(fa))
            if (OP == 9) CHAINS("v_med3_f32 %0, %0, %1, %2" : "+v"(x[c]) : "v"(fa), "v"(fb))
            if (OP == 10) CHAINS("v_lshlrev_b32 %0, %1, %0" : "+v"(u[c]) : "v"(ua))
            if (OP == 11) CHAINS("v_cvt_f32_u32 %0, %0" : "+v"(x[c]))
            if (OP == 12) CHAINS("v_floor_f32 %0, %0" : "+v"(x[c]))
            if (OP == 13) CHAINS("v_cmp_gt_f32_e64 %0, %1, %2" : "=s"(m[c]) : "v"(x[c]), "v"(fa))
            if (OP == 14) CHAINS("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(x[c]) : "v"(fa), "s"(mask))
            if (OP == 15) CHAINS("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(u[c]) : "v"(ua), "v"(ub))
            if (OP == 16) CHAINS("v_mul_hi_u32 %0, %0, %1" : "+v"(u[c]) : "v"(ua))
            if (OP == 17) CHAINS("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(q[c]), "=s"(m[c]) : "v"(ua), "v"(ub))
            if (OP == 18) CHAINS("v_rcp_f32 %0, %0" : "+v"(x[c]))
            if (OP == 19) CHAINS("v_sqrt_f32 %0, %0" : "+v"(x[c]))
            if (OP == 20) CHAINS("v_log_f32 %0, %0" : "+v"(x[c]))
            if (OP == 21) CHAINS("v_sin_f32 %0, %0" : "+v"(x[c]))
            if (OP == 22) CHAINS("v_fma_f64 %0, %0, %1, %2" : "+v"(d[c]) : "v"(da), "v"(db))
            // Mixed groups: does a transcendental overlap independent full-
            // or half-rate work, or do the costs add?
            if (OP == 23) CHAINS("v_rcp_f32 %0, %0\n\tv_fma_f32 %1, %1, %2, %3"
                                 : "+v"(x[c]), "+v"(y[c]) : "v"(fa), "v"(fb))
            if (OP == 24) CHAINS("v_rcp_f32 %0, %0\n\tv_fma_f32 %1, %1, %5, %6\n\tv_fma_f32 %2, %2, %5, %6\n\t"
                                 "v_fma_f32 %3, %3, %5, %6\n\tv_fma_f32 %4, %4, %5, %6"
                                 : "+v"(x[c]), "+v"(y[c]), "+v"(z[c]), "+v"(t[c]), "+v"(v[c]) : "v"(fa), "v"(fb))
            if (OP == 25) CHAINS("v_rcp_f32 %0, %0\n\tv_mul_hi_u32 %1, %1, %3\n\tv_mul_hi_u32 %2, %2, %3"
                                 : "+v"(x[c]), "+v"(u[c]), "+v"(u2[c]) : "v"(ua))
            if (OP == 26) CHAINS("v_mul_hi_u32 %0, %0, %3\n\tv_fma_f32 %1, %1, %4, %5\n\tv_fma_f32 %2, %2, %4, %5"
                                 : "+v"(u[c]), "+v"(y[c]), "+v"(z[c]) : "v"(ua), "v"(fa), "v"(fb))
            // Constant operands: a 32-bit literal (v_fmamk_f32 x * K + y) and an
            // inline constant (0.5).
            if (OP == 28) CHAINS("v_fmamk_f32 %0, %0, 0x3f800001, %1" : "+v"(x[c]) : "v"(fb))
            if (OP == 29) CHAINS("v_fma_f32 %0, %0, %1, 0.5" : "+v"(x[c]) : "v"(fa))
            // The group of probe 24 in another order: the eight chains' rcp
            // back to back, then their 32 fma.
            if (OP == 27) {
                CHAINS("v_rcp_f32 %0, %0" : "+v"(x[c]))
                CHAINS("v_fma_f32 %0, %0, %4, %5\n\tv_fma_f32 %1, %1, %4, %5\n\tv_fma_f32 %2, %2, %4, %5\n\t"
                       "v_fma_f32 %3, %3, %4, %5"
                       : "+v"(y[c]), "+v"(z[c]), "+v"(t[c]), "+v"(v[c]) : "v"(fa), "v"(fb))
            }
        }
    }
    uint32_t s = 0;
    for (int c = 0; c < 8; ++c)
        s += __float_as_uint(x[c]) + u[c] + (uint32_t)__double_as_longlong(d[c]) + (uint32_t)q[c] + (uint32_t)m[c] +
             __float_as_uint(y[c]) + __float_as_uint(z[c]) + __float_as_uint(t[c]) + __float_as_uint(v[c]) + u2[c];
    out[gid] = s;
}

template <int OP>
void run(const char *name, uint32_t *out, int blocks, int iters, int per_chain = 1)
{
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(probe<OP>, dim3(blocks), dim3(1024), 0, 0, out, 2, 1.0000001f, 1e-7f);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int rep = 0; rep < 5; ++rep) {
        CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(probe<OP>, dim3(blocks), dim3(1024), 0, 0, out, iters, 1.0000001f, 1e-7f);
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
    }
    // 16 waves per workgroup, 128 chain steps per wave and iteration (each
    // of per_chain instructions), 1024 SIMDs.
    const double per_simd = (double)blocks * 16 * iters * 128 / 1024.0;
    const double cyc = best * 1e-3 * 2.4e9 / per_simd;
    if (per_chain == 1)
        std::printf("%-34s %7.3f ms  %5.2f cycles per wave64 instruction\n", name, best, cyc);
    else
        std::printf("%-34s %7.3f ms  %5.2f cycles per group of %d\n", name, best, cyc, per_chain);
    std::fflush(stdout);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
}

int main()
{
    int dev;
    CHECK(hipGetDevice(&dev));
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, dev));
    std::printf("%s, %d CUs\n", p.gcnArchName, p.multiProcessorCount);
    const int blocks = 2 * p.multiProcessorCount;
    uint32_t *out;
    CHECK(hipMalloc(&out, (size_t)blocks * 1024 * sizeof(uint32_t)));
    const int it = 1000;
    run<0>("v_fma_f32 (VGPR operands)", out, blocks, it);
    run<1>("v_add_f32", out, blocks, it);
    run<2>("v_mul_f32", out, blocks, it);
    run<3>("v_fma_f32 (one SGPR operand)", out, blocks, it);
    run<4>("v_add_u32", out, blocks, it);
    run<5>("v_xor_b32", out, blocks, it);
    run<6>("v_add_u32 (one SGPR operand)", out, blocks, it);
    run<7>("v_mov_b32", out, blocks, it);
    run<8>("v_max_f32", out, blocks, it);
    run<9>("v_med3_f32", out, blocks, it);
    run<10>("v_lshlrev_b32", out, blocks, it);
    run<11>("v_cvt_f32_u32", out, blocks, it);
    run<12>("v_floor_f32", out, blocks, it);
    run<13>("v_cmp_gt_f32 (to an SGPR pair)", out, blocks, it);
    run<14>("v_cndmask_b32 (SGPR-pair mask)", out, blocks, it);
    run<15>("v_bitop3_b32 (three-input XOR)", out, blocks, it);
    run<16>("v_mul_hi_u32", out, blocks, it);
    run<17>("v_mad_u64_u32", out, blocks, it);
    run<18>("v_rcp_f32", out, blocks, it / 2);
    run<19>("v_sqrt_f32", out, blocks, it / 2);
    run<20>("v_log_f32", out, blocks, it / 2);
    run<21>("v_sin_f32", out, blocks, it / 2);
    run<22>("v_fma_f64", out, blocks, it);
    run<23>("mixed: rcp + fma", out, blocks, it / 2, 2);
    run<24>("mixed: rcp + 4 fma", out, blocks, it / 2, 5);
    run<25>("mixed: rcp + 2 mul_hi_u32", out, blocks, it / 2, 3);
    run<26>("mixed: mul_hi_u32 + 2 fma", out, blocks, it / 2, 3);
    run<27>("mixed: 8 rcp, then 32 fma", out, blocks, it / 2, 5);
    run<28>("v_fmamk_f32 (32-bit literal)", out, blocks, it);
    run<29>("v_fma_f32 (inline constant 0.5)", out, blocks, it);
    run<0>("v_fma_f32 (VGPR operands, again)", out, blocks, it);
    CHECK(hipFree(out));
    return 0;
}
