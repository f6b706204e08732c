// Measured ceiling of the numeric product's accumulation: the rate of native
// LDS atomic adds of FP64 values (ds_add_f64) on one GPU, with each wave adding
// 64 consecutive columns of a 2048-column window (waves on different columns),
// and the same for FP32; then FP64 again with every lane adding at a
// pseudo-random column of the window (a product scatters its B entries into
// the window: its addresses lie between these two patterns).
// Prints one JSON line: lane-operations per second, per CU and clock, the
// clock and CU count used.
//
//   lds_atomic_rate [--iters N]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

constexpr int kThreads = 1024;
constexpr int kWindow = 2048;  // FP64 LDS accumulators per row of a window

template <typename T, bool kScatter>
__global__ __launch_bounds__(kThreads) void k_lds_add(T *out, int iters, T v) {
    __shared__ T acc[kWindow * (sizeof(double) / sizeof(T))];
    constexpr int kLen = kWindow * (sizeof(double) / sizeof(T));
    for (int s = threadIdx.x; s < kLen; s += kThreads) acc[s] = T(0);
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x & 63;
    int col = (wave * 128 + lane) & (kLen - 1);
    // scatter: 16 pseudo-random offsets per lane (a 32-bit LCG), reused with a
    // moving base, so the address arithmetic stays a few instructions
    int off[16];
    uint32_t x = 2654435761u * (uint32_t)(threadIdx.x + 1) + 12345u * blockIdx.x;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        x = 1664525u * x + 1013904223u;
        off[k] = (int)(x >> 16) & (kLen - 1);
    }
    for (int it = 0; it < iters; it += 16) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            atomicAdd(&acc[kScatter ? (off[k] + col) & (kLen - 1) : col], v);
            if (!kScatter) col = (col + 64 * 17) & (kLen - 1);  // next 64-column block
        }
        if (kScatter) col = (col + 64 * 17) & (kLen - 1);
    }
    __syncthreads();
    T t = T(0);
    for (int s = threadIdx.x; s < kLen; s += kThreads) t += acc[s];
    if (t == T(-1)) out[blockIdx.x] = t;  // never true; keeps the adds live
}

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
            std::exit(1);                                                         \
        }                                                                         \
    } while (0)

template <typename T, bool kScatter = false>
double rate(int blocks, int iters, float *ms_out) {
    iters = (iters + 15) / 16 * 16;  // the kernel adds in steps of 16
    T *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(T) * blocks));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    k_lds_add<T, kScatter><<<blocks, kThreads>>>(out, iters / 8, T(1));  // warm-up
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a));
    k_lds_add<T, kScatter><<<blocks, kThreads>>>(out, iters, T(1));
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipFree(out));
    *ms_out = ms;
    return (double)blocks * kThreads * (double)iters / (ms * 1e-3);
}

}  // namespace

int main(int argc, char **argv) {
    int iters = 4096;
    for (int i = 1; i + 1 < argc; ++i)
        if (!std::strcmp(argv[i], "--iters")) iters = std::atoi(argv[i + 1]);
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    int clk_khz = 0;
    CHECK(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, 0));
    const int cus = p.multiProcessorCount;
    const int blocks = cus * 8;
    float ms64 = 0.f, ms32 = 0.f, mss = 0.f;
    const double r64 = rate<double>(blocks, iters, &ms64);
    const double r32 = rate<float>(blocks, iters / 8, &ms32);
    const double rs = rate<double, true>(blocks, iters, &mss);
    const double hz = clk_khz * 1e3;
    std::printf("{\"lds_add_f64_per_s\": %.4e, \"lds_add_f64_per_cu_clk\": %.3f, "
                "\"lds_add_f32_per_s\": %.4e, \"lds_add_f32_per_cu_clk\": %.3f, "
                "\"lds_add_f64_scatter_per_s\": %.4e, \"lds_add_f64_scatter_per_cu_clk\": %.3f, "
                "\"cus\": %d, \"clock_mhz\": %.0f, \"ms_f64\": %.3f, \"ms_f32\": %.3f, "
                "\"ms_f64_scatter\": %.3f, \"device\": \"%s\"}\n",
                r64, r64 / (cus * hz), r32, r32 / (cus * hz), rs, rs / (cus * hz), cus, hz / 1e6,
                ms64, ms32, mss, p.gcnArchName);
    return 0;
}
