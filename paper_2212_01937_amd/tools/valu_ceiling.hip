// valu_ceiling.hip -- measures the vector-ALU ceiling that code built like the
// distance kernels (packed-FP32 instruction selection disabled) can reach on
// this GPU: independent FMA chains per lane at full occupancy (FP32, FP64),
// the same with one reciprocal square root per eight FMAs, and the FP32 chains
// at 1, 2 and 4 waves per SIMD.  Also the HBM write rate of the materialised
// Jacobian's store pattern without its arithmetic (five planes of 256 x 1e6 FP32,
// one redshift per lane and 16 cosmologies per lane, non-temporal stores) and of a
// plain streaming write of the same bytes.  Prints one JSON object.
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

// The Jacobian kernel's stores alone: lane i of a 256-lane block (grid x) writes
// element i of five planes for each of the ct cosmologies of its tile (grid y).
__global__ __launch_bounds__(kThreads) void jac_store_pattern(float *jac, long n_c, long n_z, int ct) {
    const long tile = blockIdx.y, i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n_z) return;
    const long plane = n_c * n_z;
    const long c0 = tile * ct, c1 = c0 + ct < n_c ? c0 + ct : n_c;
    for (long c = c0; c < c1; ++c) {
        float *row = jac + c * n_z;
        for (int q = 0; q < 5; ++q) __builtin_nontemporal_store(float(q + c) * 1e-3f + float(i), row + q * plane + i);
    }
}
// A plain streaming write: 16 bytes per lane, n a multiple of 4 * kThreads.
__global__ __launch_bounds__(kThreads) void stream_write(float *p, long n) {
    const long i = ((long)blockIdx.x * kThreads + threadIdx.x) * 4;
    if (i + 3 < n) *(float4 *)(p + i) = float4{1.f, 2.f, 3.f, 4.f};
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
    {
        const long n_c = 256, n_z = 1000000, n = 5 * n_c * n_z; // 5.12 GB
        float *jac = nullptr;
        CHECK(hipMalloc(&jac, n * sizeof(float)));
        const dim3 grid((unsigned)((n_z + kThreads - 1) / kThreads), 16);
        float ms = time_ms([&] { jac_store_pattern<<<grid, kThreads>>>(jac, n_c, n_z, 16); }, 10);
        std::printf(", \"hbm_write_jacobian_pattern_tbs\": %.2f, \"hbm_write_jacobian_pattern_ms\": %.3f", n * 4.0 / (ms * 1e-3) / 1e12, ms);
        ms = time_ms([&] { stream_write<<<(unsigned)(n / 4 / kThreads), kThreads>>>(jac, n); }, 10);
        std::printf(", \"hbm_write_stream_tbs\": %.2f", n * 4.0 / (ms * 1e-3) / 1e12);
        CHECK(hipFree(jac));
    }
    std::printf("}\n");
    CHECK(hipFree(of));
    CHECK(hipFree(od));
    return 0;
}
