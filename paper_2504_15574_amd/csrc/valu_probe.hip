// VALU issue-rate probe for gfx950 (a measurement program, not part of the
// library).  Each kernel runs 8 independent chains of one instruction kind per
// thread, 64 of them per loop trip, in 8192 workgroups of 256 threads (8 waves
// per SIMD), so issue, not latency, limits it.  It prints the rate of the
// chained instruction kind in G wave-instructions/s and the cycles a wave64
// instruction of that kind occupies its SIMD at 2.4 GHz.  The stage kernel's
// instruction mix is weighted with these costs to tell how busy its VALU is.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                  \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(3);                                                      \
        }                                                                      \
    } while (0)

namespace {
constexpr int BLOCKS = 8192, THREADS = 256, ITERS = 4096, CHAINS = 8, UNROLL = 8;

__device__ inline float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return fma(a, b, c); }

// OP 0: mul, 1: add, 2: fma into the accumulator (fmac), 3: fma with three sources
template <class T, int OP>
__global__ __launch_bounds__(THREADS) void arith(T* out, T a, T b, int iters) {
    T x[CHAINS], y[CHAINS];
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) {
        x[j] = T(threadIdx.x) * T(1e-3) + T(j);
        y[j] = T(j) * T(0.5);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
            for (int j = 0; j < CHAINS; ++j) {
                if (OP == 0) x[j] = x[j] * a;
                else if (OP == 1) x[j] = x[j] + a;
                else if (OP == 2) x[j] = fma_t(a, b, x[j]);
                else x[j] = fma_t(x[j], a, y[j]);
            }
        }
    }
    T s = T(0);
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) s += x[j];
    out[blockIdx.x * THREADS + threadIdx.x] = s;
}

// OP 0: 32-bit integer add (chained across the chains, so it cannot fold);
// 1: compare + select + mul (three instructions per chained step);
// 2: FP32 multiply rounded to FP16 (one v_fma_mixlo_f16 per step)
template <int OP>
__global__ __launch_bounds__(THREADS) void other(unsigned* out, int iters) {
    unsigned x[CHAINS];
    float f[CHAINS];
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) {
        x[j] = threadIdx.x * 7u + j;
        f[j] = (float)x[j] * 1e-3f;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
#pragma unroll
            for (int j = 0; j < CHAINS; ++j) {
                if (OP == 0) x[j] = x[j] + x[(j + 1) % CHAINS];
                else if (OP == 1) f[j] = f[j] > 1.0f ? f[j] * 0.5f : f[j] * 1.0001f;
                else f[j] = __half2float(__float2half(f[j] * 1.0001f));
            }
        }
    }
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) s += x[j] + __float_as_uint(f[j]);
    out[blockIdx.x * THREADS + threadIdx.x] = s;
}

template <class K, class... Args>
double time_ms(K kernel, Args... args) {
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    hipLaunchKernelGGL(kernel, dim3(BLOCKS), dim3(THREADS), 0, 0, args...);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(kernel, dim3(BLOCKS), dim3(THREADS), 0, 0, args...);
    CK(hipGetLastError());
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
    return ms / 5.0;
}
}  // namespace

int main() {
    void* out = nullptr;
    CK(hipMalloc(&out, (size_t)BLOCKS * THREADS * sizeof(double)));   // one value per thread
    // chained steps per launch, counted per wave
    const double steps = (double)BLOCKS * (THREADS / 64) * ITERS * UNROLL * CHAINS;
    const double peak = 256 * 4 * 2.4;    // wave-instructions/s (G) at one per SIMD cycle
    struct Row { const char* name; int per_step; double ms; } rows[] = {
        {"f32 mul", 1, time_ms(arith<float, 0>, (float*)out, 0.999f, 1e-7f, ITERS)},
        {"f32 add", 1, time_ms(arith<float, 1>, (float*)out, 0.999f, 1e-7f, ITERS)},
        {"f32 fmac", 1, time_ms(arith<float, 2>, (float*)out, 0.999f, 1e-7f, ITERS)},
        {"f32 fma (3 sources)", 1, time_ms(arith<float, 3>, (float*)out, 0.999f, 1e-7f, ITERS)},
        {"f64 mul", 1, time_ms(arith<double, 0>, (double*)out, 0.999, 1e-7, ITERS)},
        {"f64 add", 1, time_ms(arith<double, 1>, (double*)out, 0.999, 1e-7, ITERS)},
        {"f64 fmac", 1, time_ms(arith<double, 2>, (double*)out, 0.999, 1e-7, ITERS)},
        {"f64 fma (3 sources)", 1, time_ms(arith<double, 3>, (double*)out, 0.999, 1e-7, ITERS)},
        {"u32 add", 1, time_ms(other<0>, (unsigned*)out, ITERS)},
        {"f32 cmp + cndmask + mul", 3, time_ms(other<1>, (unsigned*)out, ITERS)},
        {"f32 mul rounded to f16 (fma_mix)", 1, time_ms(other<2>, (unsigned*)out, ITERS)},
    };
    std::printf("%-34s %10s %22s %16s\n", "chained instructions", "ms/launch", "G wave-instructions/s",
                "cycles per inst");
    for (const Row& r : rows) {
        const double rate = steps * r.per_step / (r.ms * 1e-3) / 1e9;
        std::printf("%-34s %10.3f %22.1f %16.2f\n", r.name, r.ms, rate, peak / rate);
    }
    CK(hipFree(out));
    return 0;
}
