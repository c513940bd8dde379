// Issue rates of the vector instructions the force path is built from, measured
// on the device: the peaks against which the kernels' instruction counts are
// priced (fused multiply-add in FP32 and FP64, the 32-bit integer products of
// the fixed-point phases, the transcendentals of the structure factor, the far
// force and the pair kernel, and mixes of them that show whether a
// transcendental overlaps other vector work).
//
// Each thread runs kChains independent dependency chains of one instruction
// (or one mix), so that issue rather than latency bounds the loop; the grid
// holds 16 waves per SIMD.  The time of the whole launch (HIP events) gives
// lane-instructions per second.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rbsog_internal.h"

namespace rbsog {

rbsog_status fail_noctx(rbsog_status st, const char *fmt, ...);

namespace {

constexpr int kChains = 8;
constexpr int kProbeBlock = 256;
constexpr int kProbeBlocks = 256 * 16;  // 16 waves per SIMD of 256 CUs
constexpr int kIters = 2048;

enum ProbeOp : int {
    kFmaF32 = 0,
    kFmaF64,
    kMulLoU32,
    kMadU64U32,
    kMulU24,
    kAdd3U32,
    kSinF32,
    kCosF32,
    kExpF32,
    kRsqF32,
    kSinCosFma2,  // sin + cos + 2 FMA per step, on independent values (structure-factor mix)
    kMul3Add3,    // 3 mul_lo_u32 + add3 per step (fixed-point phase)
    kRndneF64,    // round to nearest integer, FP64 (the turn index of the FP64 phases)
    kCvtI32F64,   // FP64 to int32 conversion (the table index)
    kNumProbes
};

// instructions per chain and iteration
__host__ __device__ constexpr int insts_of(int op) {
    return op == kSinCosFma2 ? 4 : (op == kMul3Add3 ? 4 : 1);
}

const char *const kProbeNames[kNumProbes] = {
    "v_fma_f32", "v_fma_f64", "v_mul_lo_u32", "v_mad_u64_u32", "v_mul_u32_u24", "v_add3_u32",
    "v_sin_f32", "v_cos_f32", "v_exp_f32", "v_rsq_f32", "sin+cos+2fma", "3mul_lo+add3",
    "v_rndne_f64", "v_cvt_i32_f64"};

template <int OP>
__global__ __launch_bounds__(kProbeBlock) void k_probe(uint32_t seed, float *__restrict__ sink) {
    const uint32_t t = blockIdx.x * kProbeBlock + threadIdx.x;
    // values only known at run time, so that nothing folds
    const uint32_t s = seed ^ t;
    float f[kChains], g[kChains];
    double d[kChains];
    uint32_t u[kChains], v[kChains];
    uint64_t w[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        u[c] = s * (2u * c + 1u);
        v[c] = u[c] ^ 0x5bd1e995u;
        f[c] = (float)(u[c] & 0xffff) * 1.0e-5f;
        g[c] = f[c] + 0.25f;
        d[c] = (double)f[c];
        w[c] = u[c];
    }
    const float fa = __uint_as_float(0x3f7ffff0u ^ (seed & 7u));
    const float fb = 1.0e-7f * (float)(seed & 15u);
    const double da = 0.9999999 + 1e-9 * (double)(seed & 7u), db = 1e-9;
    const uint32_t ua = (seed | 1u) * 2654435761u, ub = seed + 12345u;
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (OP == kFmaF32) f[c] = fmaf(f[c], fa, fb);
            else if constexpr (OP == kFmaF64) d[c] = fma(d[c], da, db);
            // integer chains in inline asm: the compiler would fold a chain of
            // products or sums into one operation (no memory operands here)
            else if constexpr (OP == kMulLoU32) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(u[c]) : "s"(ua));
            else if constexpr (OP == kMadU64U32) {
                uint64_t cy;
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(w[c]), "=s"(cy) : "v"(u[c]), "s"(ua));
            } else if constexpr (OP == kMulU24) asm volatile("v_mul_u32_u24 %0, %1, %0" : "+v"(u[c]) : "s"(ua));
            else if constexpr (OP == kAdd3U32) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(u[c]) : "v"(v[c]), "s"(ua));
            else if constexpr (OP == kRndneF64) asm volatile("v_rndne_f64 %0, %0" : "+v"(d[c]));
            else if constexpr (OP == kCvtI32F64) asm volatile("v_cvt_i32_f64 %0, %1" : "=v"(u[c]) : "v"(d[c]));
            else if constexpr (OP == kSinF32) f[c] = __builtin_amdgcn_sinf(f[c]);
            else if constexpr (OP == kCosF32) f[c] = __builtin_amdgcn_cosf(f[c]);
            else if constexpr (OP == kExpF32) f[c] = __builtin_amdgcn_exp2f(f[c]) - 1.0f;
            else if constexpr (OP == kRsqF32) f[c] = __builtin_amdgcn_rsqf(f[c]);
            else if constexpr (OP == kSinCosFma2) {
                const float a = __builtin_amdgcn_sinf(f[c]), b = __builtin_amdgcn_cosf(f[c]);
                g[c] = fmaf(a, fa, g[c]);
                f[c] = fmaf(b, fb, f[c]);
            }
        }
        if constexpr (OP == kMul3Add3) {
            // three products of different chains summed: nothing to factor
            uint32_t nu[kChains];
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                nu[c] = u[c] * ua + u[(c + 1) % kChains] * ub + u[(c + 2) % kChains] * v[0];
#pragma unroll
            for (int c = 0; c < kChains; ++c) u[c] = nu[c];
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc += f[c] + g[c] + (float)d[c] + (float)u[c] + (float)(uint32_t)w[c];
    // never true for the seeds used; keeps every chain alive
    if (acc == 1.234567e-30f) sink[t] = acc;
}

template <int OP>
void launch_probe(uint32_t seed, float *sink, hipStream_t st) {
    hipLaunchKernelGGL((k_probe<OP>), dim3(kProbeBlocks), dim3(kProbeBlock), 0, st, seed, sink);
}

typedef void (*ProbeFn)(uint32_t, float *, hipStream_t);
const ProbeFn kProbeFns[kNumProbes] = {
    launch_probe<kFmaF32>,   launch_probe<kFmaF64>,  launch_probe<kMulLoU32>, launch_probe<kMadU64U32>,
    launch_probe<kMulU24>,   launch_probe<kAdd3U32>, launch_probe<kSinF32>,   launch_probe<kCosF32>,
    launch_probe<kExpF32>,   launch_probe<kRsqF32>,  launch_probe<kSinCosFma2>, launch_probe<kMul3Add3>,
    launch_probe<kRndneF64>, launch_probe<kCvtI32F64>};

}  // namespace
}  // namespace rbsog

using namespace rbsog;

extern "C" int32_t rbsog_probe_count(void) { return kNumProbes; }

extern "C" const char *rbsog_probe_name(int32_t i) {
    return (i >= 0 && i < kNumProbes) ? kProbeNames[i] : nullptr;
}

extern "C" rbsog_status rbsog_probe_rates(int32_t device, int32_t reps, double *rates, int32_t n) {
    if (!rates || n < kNumProbes || reps < 1) return fail_noctx(RBSOG_E_ARG, "rates needs %d entries, reps >= 1", (int)kNumProbes);
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail_noctx(RBSOG_E_DEVICE, "hipGetDevice failed");
    if (hipSetDevice(device) != hipSuccess) return fail_noctx(RBSOG_E_DEVICE, "hipSetDevice(%d) failed", (int)device);
    rbsog_status st = RBSOG_OK;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float *sink = nullptr;
    if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipMalloc(&sink, sizeof(float) * kProbeBlock * kProbeBlocks) != hipSuccess) {
        st = fail_noctx(RBSOG_E_DEVICE, "probe set-up failed");
    }
    const double lanes = (double)kProbeBlock * kProbeBlocks;
    for (int op = 0; op < kNumProbes && st == RBSOG_OK; ++op) {
        kProbeFns[op](1u, sink, s);  // warm-up (code load, clocks)
        float best = 0.f;
        for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess) { st = fail_noctx(RBSOG_E_DEVICE, "event"); break; }
            kProbeFns[op](2u + (uint32_t)r, sink, s);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail_noctx(RBSOG_E_DEVICE, "probe launch failed");
                break;
            }
            if (r == 0 || ms < best) best = ms;
        }
        if (st == RBSOG_OK)
            rates[op] = lanes * (double)kIters * kChains * insts_of(op) / (1e-3 * (double)best);
    }
    if (hipGetLastError() != hipSuccess && st == RBSOG_OK) st = fail_noctx(RBSOG_E_DEVICE, "probe kernel failed");
    if (sink) (void)hipFree(sink);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipSetDevice(prev);
    return st;
}
