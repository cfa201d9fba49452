// valu_ceiling.hip -- measures the vector-ALU ceiling that code built like the
// distance kernels (packed-FP32 instruction selection disabled) can reach on
// this GPU: independent FMA chains per lane at full occupancy (FP32, FP64),
// the same with one reciprocal square root per eight FMAs, and the FP32 chains
// at 1, 2 and 4 waves per SIMD.  Prints one JSON object.
//
// Every launch writes exactly one element per lane of a buffer sized for the
// largest grid; the kernels have no data-dependent control flow.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));              \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

namespace {

constexpr int kThreads = 256;  // four waves per block

template <typename T, int CH>
__global__ __launch_bounds__(kThreads) void fma_chains(T *out, int iters, T a, T b) {
    T v[CH];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = T(gid + c) * T(1e-9);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CH; ++c) v[c] = v[c] * a + b;
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += v[c];
    out[gid] = s;
}

// Eight FMA chains; after each round of eight FMAs one chain goes through rsqrt.
__global__ __launch_bounds__(kThreads) void fma_rsq_chains(float *out, int iters, float a, float b) {
    float v[8];
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = 1.0f + float(gid + c) * 1e-9f;
    for (int i = 0; i < iters; i += 8) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = v[c] * a + b;
            v[t] = __builtin_amdgcn_rsqf(v[t]);
        }
    }
    float s = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += v[c];
    out[gid] = s;
}

template <typename L> float time_ms(L launch, int reps) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    launch();
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) launch();
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return ms / reps;
}

}  // namespace

int main() {
    int dev = 0, cus = 0, khz = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev));
    const double clk = 2.4e9;                      // peak engine clock used for the published peaks
    const int full_blocks = cus * 8;               // 8 four-wave blocks per CU = 8 waves per SIMD
    const long n = long(full_blocks) * kThreads;   // buffer: one element per lane of the largest grid
    const int iters = 4096;
    float *of = nullptr;
    double *od = nullptr;
    CHECK(hipMalloc(&of, n * sizeof(float)));
    CHECK(hipMalloc(&od, n * sizeof(double)));

    auto rate = [&](double ms, double wave_instr) { return wave_instr / (ms * 1e-3 * clk * cus); };
    std::printf("{\"cus\": %d, \"clock_khz_reported\": %d, \"clock_used_hz\": %.3g", cus, khz, clk);
    {
        float ms = time_ms([&] { fma_chains<float, 8><<<full_blocks, kThreads>>>(of, iters, 0.999f, 1e-3f); }, 5);
        double fma = 8.0 * iters * double(n);
        std::printf(", \"fp32_fma_tflops\": %.2f, \"fp32_fma_wave_instr_per_clk_per_cu\": %.3f", 2 * fma / ms * 1e-9,
                    rate(ms, fma / 64));
    }
    {
        float ms = time_ms([&] { fma_chains<double, 8><<<full_blocks, kThreads>>>(od, iters, 0.999, 1e-3); }, 5);
        double fma = 8.0 * iters * double(n);
        std::printf(", \"fp64_fma_tflops\": %.2f, \"fp64_fma_wave_instr_per_clk_per_cu\": %.3f", 2 * fma / ms * 1e-9,
                    rate(ms, fma / 64));
    }
    {
        float ms = time_ms([&] { fma_rsq_chains<<<full_blocks, kThreads>>>(of, iters, 0.999f, 1e-3f); }, 5);
        double fma = 8.0 * iters * double(n), rsq = iters * double(n);
        std::printf(", \"fp32_fma_plus_rsq_tflops_fma_only\": %.2f, \"fp32_fma_plus_rsq_wave_instr_per_clk_per_cu\": %.3f",
                    2 * fma / ms * 1e-9, rate(ms, (fma + rsq) / 64));
    }
    for (int waves : {1, 2, 4}) {
        const int blocks = cus * waves;  // four-wave blocks: `waves` waves per SIMD
        float ms = time_ms([&] { fma_chains<float, 8><<<blocks, kThreads>>>(of, 4 * iters, 0.999f, 1e-3f); }, 3);
        double fma = 8.0 * 4 * iters * double(blocks) * kThreads;
        std::printf(", \"fp32_fma_tflops_%d_waves_per_simd\": %.2f", waves, 2 * fma / ms * 1e-9);
    }
    std::printf("}\n");
    CHECK(hipFree(of));
    CHECK(hipFree(od));
    return 0;
}
