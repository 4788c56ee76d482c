// VALU issue-cost calibration for gfx950 (used to weight the roofline's
// algorithmic operation counts).  Each kernel runs 8 independent chains per
// lane of ONE instruction class, so that throughput, not latency, is timed;
// 8 waves per SIMD on every CU.  Prints the cost of one instruction of each
// class in units of one FP32 FMA issue slot.
//
//   hipcc --offload-arch=gfx950 -O3 valu_rates.hip -o valu_rates && ./valu_rates
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "device.hpp"

#define CH 8
#define ITERS 8192

#define CHAIN_KERNEL(name, T, init, body)                                        \
    __global__ void name(T* out, T s)                                            \
    {                                                                            \
        T a[CH];                                                                 \
        for (int c = 0; c < CH; ++c) a[c] = (T)(init);                           \
        for (int i = 0; i < ITERS; ++i) {                                        \
            _Pragma("unroll") for (int c = 0; c < CH; ++c) { T x = a[c]; a[c] = (body); } \
        }                                                                        \
        T r = a[0];                                                              \
        for (int c = 1; c < CH; ++c) r = r + a[c];                               \
        out[blockIdx.x * blockDim.x + threadIdx.x] = r;                          \
    }

CHAIN_KERNEL(k_fma32, float, 0.25f + threadIdx.x * 1e-6f + c, fmaf(x, s, 0.5f))
CHAIN_KERNEL(k_fma64, double, 0.25 + threadIdx.x * 1e-6 + c, fma(x, s, 0.5))
CHAIN_KERNEL(k_add_u32, uint32_t, threadIdx.x + c, x + s)
CHAIN_KERNEL(k_xor_b32, uint32_t, threadIdx.x * 7919u + c * 104729u + s, x ^ a[(c + 3) & (CH - 1)])
// three-input xor in one instruction (v_bitop3_b32, truth table 0x96)
CHAIN_KERNEL(k_xor3_b32, uint32_t, threadIdx.x * 7919u + c * 104729u + s,
             __builtin_amdgcn_bitop3_b32(x, a[(c + 3) & (CH - 1)], a[(c + 5) & (CH - 1)], 0x96))
CHAIN_KERNEL(k_log_f32, float, 0.5f + threadIdx.x * 1e-6f + c, __builtin_amdgcn_logf(x))
CHAIN_KERNEL(k_exp_f32, float, 0.5f + threadIdx.x * 1e-6f + c, __builtin_amdgcn_exp2f(x))
CHAIN_KERNEL(k_sin_f32, float, 0.5f + threadIdx.x * 1e-6f + c, __builtin_amdgcn_sinf(x))
CHAIN_KERNEL(k_sqrt_f32, float, 0.5f + threadIdx.x * 1e-6f + c, __builtin_amdgcn_sqrtf(x))
// FP64 device-library calls as the FP64 form of the continuation kernel makes
// them; each chain step adds one FP64 add or multiply to keep the argument in
// range (its cost, one FP64 FMA slot, is subtracted in the report).
CHAIN_KERNEL(k_log_f64, double, 0.5 + threadIdx.x * 1e-6 + c, log(x + 2.0))
CHAIN_KERNEL(k_exp_f64, double, 0.5 + threadIdx.x * 1e-6 + c, exp(x * -0.5))
CHAIN_KERNEL(k_sqrt_f64, double, 0.5 + threadIdx.x * 1e-6 + c, sqrt(x + 0.25))
// a conversion pair (FP64 to u32 and back) per step
CHAIN_KERNEL(k_cvt_f64, double, 0.5 + threadIdx.x * 1e-6 + c, (double)(uint32_t)(x * 0.5 + 1.0))

// sin and cos of pi x (one sincospi call) per chain step; the next argument
// is s + c (one FP64 add, subtracted in the report).
__global__ void k_sincospi_f64(double* out, double s0)
{
    double a[CH];
    for (int c = 0; c < CH; ++c) a[c] = 0.25 + threadIdx.x * 1e-6 + c * 0.01 + s0;
    for (int i = 0; i < ITERS; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            double sn, cs;
            sincospi(a[c], &sn, &cs);
            a[c] = sn + cs;
        }
    }
    double r = a[0];
    for (int c = 1; c < CH; ++c) r = r + a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// The continuation kernel's FP64 normal-map pieces (bmc::log_u32,
// bmc::sincos_2pi_u32, bmc::sqrt_pos) on words from a counter: F = 0 is the
// same loop with the word converted and added (the glue, subtracted).
template <int F>
__global__ void k_map64(double* out, uint32_t s)
{
    double acc[CH];
    for (int c = 0; c < CH; ++c) acc[c] = 0.0;
    const uint32_t x0 = threadIdx.x * 2654435761u + blockIdx.x * 40503u + s;
    for (int i = 0; i < ITERS; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const uint32_t w = x0 + (uint32_t)c * 69069u + (uint32_t)i * 1664525u;
            if (F == 0) acc[c] += (double)w;
            else if (F == 1) acc[c] += bmc::log_u32(w);
            else if (F == 2) {
                double sn, cs;
                bmc::sincos_2pi_u32(w, sn, cs);
                acc[c] += sn * cs;
            } else {
                acc[c] += bmc::sqrt_pos((double)w + 1.0);
            }
        }
    }
    double r = acc[0];
    for (int c = 1; c < CH; ++c) r += acc[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// 32x32->64 multiply-accumulate: acc = lo32(acc) * s + acc, one v_mad_u64_u32.
__global__ void k_mad_u64(uint64_t* out, uint64_t s)
{
    uint64_t a[CH];
    for (int c = 0; c < CH; ++c) a[c] = threadIdx.x + 977u * c;
    const uint32_t m = (uint32_t)s;
    for (int i = 0; i < ITERS; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) a[c] = (uint64_t)(uint32_t)a[c] * m + a[c];
    }
    uint64_t r = a[0];
    for (int c = 1; c < CH; ++c) r ^= a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

template <class F>
static double seconds(F launch)
{
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    launch();
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(a);
    launch();
    (void)hipEventRecord(b);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms * 1e-3;
}

int main()
{
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    const int threads = 256;
    const int blocks = cus * 8;                 // 8 waves per SIMD
    const size_t n = (size_t)blocks * threads;
    void* buf = nullptr;
    if (hipMalloc(&buf, n * 8) != hipSuccess) return 1;
    // ops: instructions of the class per lane per iteration, as emitted
    // (the xor chains lose one instruction in eight to the compiler).
    struct Row { const char* name; double t; double ops; double glue; } rows[24];
    int k = 0;
#define RUN(label, kern, T, s, per_iter) RUNG(label, kern, T, s, per_iter, 0.0)
#define RUNG(label, kern, T, s, per_iter, glue_f64) \
    rows[k].name = label;                 \
    rows[k].ops = per_iter;               \
    rows[k].glue = glue_f64;              \
    rows[k++].t = seconds([&] { hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, 0, (T*)buf, (T)(s)); })
    RUN("fma_f32", k_fma32, float, 0.999f, 8);
    RUN("fma_f64", k_fma64, double, 0.999, 8);
    RUN("add_u32", k_add_u32, uint32_t, 12345u, 8);
    RUN("xor_b32", k_xor_b32, uint32_t, 12345u, 7);
    RUN("xor3_b32", k_xor3_b32, uint32_t, 12345u, 8);
    RUN("mad_u64_u32", k_mad_u64, uint64_t, 0xD2511F53ull, 8);
    RUN("log_f32", k_log_f32, float, 0.f, 8);
    RUN("exp_f32", k_exp_f32, float, 0.f, 8);
    RUN("sin_f32", k_sin_f32, float, 0.f, 8);
    RUN("sqrt_f32", k_sqrt_f32, float, 0.f, 8);
    RUNG("log_f64", k_log_f64, double, 0.0, 8, 1.0);
    RUNG("exp_f64", k_exp_f64, double, 0.0, 8, 1.0);
    RUNG("sqrt_f64", k_sqrt_f64, double, 0.0, 8, 1.0);
    RUNG("sincospi_f64", k_sincospi_f64, double, 0.0, 8, 1.0);
    RUNG("cvt_pair_f64", k_cvt_f64, double, 0.0, 8, 1.0);
    RUN("map_glue", k_map64<0>, double, 0u, 8);
    const int g_map = k - 1;
    RUN("log_u32", k_map64<1>, double, 0u, 8);
    RUN("sincos_2pi_u32", k_map64<2>, double, 0u, 8);
    RUN("sqrt_pos", k_map64<3>, double, 0u, 8);
    const double fma_rate = (double)n * ITERS * rows[0].ops / rows[0].t;
    printf("CUs %d; fp32 fma: %.4e lane-ops/s (= %.3f GHz x 64 lanes x CUs)\n", cus, fma_rate,
           fma_rate / (64.0 * cus) * 1e-9);
    const double fma64_rate = (double)n * ITERS * rows[1].ops / rows[1].t;
    for (int i = 0; i < k; ++i) {
        const double rate = (double)n * ITERS * rows[i].ops / rows[i].t;
        printf("%-12s %8.3f ms  %.4e lane-ops/s  cost %.3f fma-slots", rows[i].name, rows[i].t * 1e3, rate,
               fma_rate / rate);
        // FP64 rows: cost in FP64-FMA slots with the chain's glue (FP64
        // adds/multiplies, one FP64 FMA slot each) taken out
        if (rows[i].glue > 0.0) printf("  = %.2f fp64-fma-slots", fma64_rate / rate - rows[i].glue);
        printf("\n");
    }
    // the normal-map pieces net of their loop glue (the sincos row also
    // pays one FP64 multiply), in FP64-FMA slots
    for (int i = g_map + 1; i < g_map + 4; ++i) {
        const double net = (rows[i].t - rows[g_map].t) * fma64_rate / ((double)n * ITERS * rows[i].ops);
        printf("%-14s net of glue: %.2f fp64-fma-slots\n", rows[i].name, net - (i == g_map + 2 ? 1.0 : 0.0));
    }
    (void)hipFree(buf);
    return 0;
}
