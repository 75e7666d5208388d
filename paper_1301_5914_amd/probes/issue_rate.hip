// Issue-rate probe for the VALU roofline of the pair kernels: cycles per wave64 instruction
// on one SIMD for the instruction kinds the pair loops are made of.  Each lane runs kChains
// independent dependency chains of one instruction kind (all operands in vector
// registers), kSteps steps per chain, in a launch of kWavesPerSimd waves on every SIMD.
// Cycles per instruction per SIMD = launch time x 2.4 GHz x SIMDs / wave-instructions
// issued.  The transcendental rate per compute unit follows as 4 SIMDs x 64 lanes /
// (cycles of v_exp_f32 or v_rsq_f32).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kChains = 16;
constexpr int kSteps = 2048;
constexpr int kBlock = 256;
constexpr int kWavesPerSimd = 8;

enum Kind { EXP_F32, RSQ_F32, FMA_F32, MUL_F32, FMA_F64, RSQ_F64, NKINDS };
const char* kName[NKINDS] = {"v_exp_f32", "v_rsq_f32", "v_fma_f32", "v_mul_f32", "v_fma_f64", "v_rsq_f64"};

template <int K>
__global__ __launch_bounds__(kBlock) void chains(const float* __restrict__ in32, const double* __restrict__ in64,
                                                 float* __restrict__ out32, double* __restrict__ out64) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if constexpr (K == FMA_F64 || K == RSQ_F64) {
        double x[kChains];
        const double a = in64[t], b = in64[t + 1];
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = in64[t + c];
        for (int s = 0; s < kSteps; ++s) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (K == FMA_F64) x[c] = fma(x[c], a, b);             // -> b / (1 - a)
                else x[c] = __builtin_amdgcn_rsq(x[c]);                          // -> 1
            }
        }
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc += x[c];
        out64[t] = acc;
    } else {
        float x[kChains];
        const float a = in32[t], b = in32[t + 1];
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = in32[t + c];
        for (int s = 0; s < kSteps; ++s) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if constexpr (K == EXP_F32) x[c] = __builtin_amdgcn_exp2f(-x[c]);  // -> 0.64
                else if constexpr (K == RSQ_F32) x[c] = __builtin_amdgcn_rsqf(x[c]);  // -> 1
                else if constexpr (K == FMA_F32) x[c] = fmaf(x[c], a, b);
                else x[c] = x[c] * a;
            }
        }
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc += x[c];
        out32[t] = acc;
    }
}

#define CHK(e)                                                                                     \
    do {                                                                                           \
        hipError_t err_ = (e);                                                                     \
        if (err_ != hipSuccess) {                                                                  \
            std::fprintf(stderr, "%s failed: %s\n", #e, hipGetErrorString(err_));                  \
            std::exit(1);                                                                          \
        }                                                                                          \
    } while (0)

}  // namespace

int main() {
    int cus = 0;
    CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int simds = 4 * cus;
    const int waves = simds * kWavesPerSimd;
    const int blocks = waves / (kBlock / 64);
    const size_t n = (size_t)blocks * kBlock + kChains + 1;   // inputs read up to t + kChains
    float *in32, *out32;
    double *in64, *out64;
    CHK(hipMalloc(&in32, n * sizeof(float)));
    CHK(hipMalloc(&in64, n * sizeof(double)));
    CHK(hipMalloc(&out32, n * sizeof(float)));
    CHK(hipMalloc(&out64, n * sizeof(double)));
    {
        float* h32 = (float*)std::malloc(n * sizeof(float));
        double* h64 = (double*)std::malloc(n * sizeof(double));
        for (size_t i = 0; i < n; ++i) {
            h32[i] = 0.25f + 0.5f * (float)((i * 2654435761u) % 1000) / 1000.0f;   // (0.25, 0.75)
            h64[i] = 0.25 + 0.5 * (double)((i * 2654435761u) % 1000) / 1000.0;
        }
        CHK(hipMemcpy(in32, h32, n * sizeof(float), hipMemcpyHostToDevice));
        CHK(hipMemcpy(in64, h64, n * sizeof(double), hipMemcpyHostToDevice));
        std::free(h32);
        std::free(h64);
    }
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    std::printf("compute units %d, waves %d (%d per SIMD), %d chains x %d steps per lane\n", cus, waves,
                kWavesPerSimd, kChains, kSteps);
    std::printf("| instruction | launch ms (median of 5) | cycles per wave64 instruction per SIMD at 2.4 GHz |\n");
    std::printf("|---|---|---|\n");
    for (int k = 0; k < NKINDS; ++k) {
        float best[5];
        for (int rep = 0; rep < 6; ++rep) {
            CHK(hipEventRecord(e0, 0));
            switch (k) {
                case EXP_F32: hipLaunchKernelGGL(chains<EXP_F32>, dim3(blocks), dim3(kBlock), 0, 0, in32, in64, out32, out64); break;
                case RSQ_F32: hipLaunchKernelGGL(chains<RSQ_F32>, dim3(blocks), dim3(kBlock), 0, 0, in32, in64, out32, out64); break;
                case FMA_F32: hipLaunchKernelGGL(chains<FMA_F32>, dim3(blocks), dim3(kBlock), 0, 0, in32, in64, out32, out64); break;
                case MUL_F32: hipLaunchKernelGGL(chains<MUL_F32>, dim3(blocks), dim3(kBlock), 0, 0, in32, in64, out32, out64); break;
                case FMA_F64: hipLaunchKernelGGL(chains<FMA_F64>, dim3(blocks), dim3(kBlock), 0, 0, in32, in64, out32, out64); break;
                default: hipLaunchKernelGGL(chains<RSQ_F64>, dim3(blocks), dim3(kBlock), 0, 0, in32, in64, out32, out64); break;
            }
            CHK(hipGetLastError());
            CHK(hipEventRecord(e1, 0));
            CHK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best[rep - 1] = ms;   // first launch is the warm-up
        }
        for (int i = 0; i < 5; ++i)
            for (int j = i + 1; j < 5; ++j)
                if (best[j] < best[i]) { float t = best[i]; best[i] = best[j]; best[j] = t; }
        const double ms = best[2];
        const double insts_per_simd = (double)kWavesPerSimd * kChains * kSteps;
        const double cycles = ms * 1e-3 * 2.4e9 / insts_per_simd;
        std::printf("| %s | %.3f | %.2f |\n", kName[k], ms, cycles);
    }
    CHK(hipFree(in32));
    CHK(hipFree(in64));
    CHK(hipFree(out32));
    CHK(hipFree(out64));
    return 0;
}
