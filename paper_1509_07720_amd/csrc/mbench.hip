// Measured peaks of the two device resources the projection leans on, for
// the roofline figures: HBM bandwidth (a plain copy kernel of known size,
// also the calibration run for the FETCH_SIZE / WRITE_SIZE counters) and the
// rate of atomic adds to scattered addresses of a large grid (the deposit's
// access pattern).
//
//   mbench copy   <MiB> [reps]   stream MiB of float4 from one buffer to another
//   mbench atomic <MiB> [reps]   atomic adds to random cells of a MiB grid:
//                                FP32 plain, FP32 returning + compensated (as the
//                                FP32 deposit), FP64 plain (as the FP64 deposit)
//                                and 64-bit compare-and-swap
//   mbench lds    [reps]         atomic adds to random words of a 16 KiB LDS
//                                table per block, FP32 and FP64 (the set-up
//                                kernel's per-cell merge uses the FP64 form)
//
// Each mode prints one JSON line per measurement.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define CHECK(x)                                                                           \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) {                                                            \
            fprintf(stderr, "%s:%d: %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
            exit(1);                                                                       \
        }                                                                                  \
    } while (0)

__global__ void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) dst[i] = src[i];
}

// Integer hash (a 32-bit finaliser: xor-shift / odd multiply rounds) to
// spread the atomic targets over the grid.
__device__ inline uint32_t mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <bool COMPENSATED>
__global__ void k_atomic(float *hi, float *lo, uint32_t n, int iters)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        const uint32_t a = mix(t * 131u + (uint32_t)i * 7919u) % n;
        const float x = 1e-3f * (float)((t + i) & 7);
        if constexpr (COMPENSATED) {
            const float old = unsafeAtomicAdd(hi + a, x);
            const float s = old + x;
            const float bb = s - old;
            const float err = (old - (s - bb)) + (x - bb);
            if (err != 0.0f) unsafeAtomicAdd(lo + a, err);
        } else {
            unsafeAtomicAdd(hi + a, x);
        }
    }
}

__global__ void k_atomic64(double *g, uint32_t n, int iters)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        const uint32_t a = mix(t * 131u + (uint32_t)i * 7919u) % n;
        unsafeAtomicAdd(g + a, 1e-3 * (double)((t + i) & 7));
    }
}

__global__ void k_cas64(unsigned long long *g, uint32_t n, int iters)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        const uint32_t a = mix(t * 131u + (uint32_t)i * 7919u) % n;
        atomicCAS(g + a, (unsigned long long)i, (unsigned long long)t);
    }
}

template <typename F>
__global__ void k_lds(F *sink, int iters)
{
    constexpr int N = 16384 / sizeof(F);
    __shared__ F tab[N];
    for (int e = threadIdx.x; e < N; e += blockDim.x) tab[e] = F(0);
    __syncthreads();
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < iters; ++i) atomicAdd(&tab[mix(t * 131u + (uint32_t)i * 7919u) % N], F(1));
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = tab[0];
}

int main(int argc, char **argv)
{
    if (argc >= 2 && !strcmp(argv[1], "lds")) {
        const int reps = argc > 2 ? atoi(argv[2]) : 5;
        if (reps < 1 || reps > 1000) {
            fprintf(stderr, "reps must be in 1..1000\n");
            return 2;
        }
        hipDeviceProp_t prop;
        CHECK(hipGetDeviceProperties(&prop, 0));
        const int blocks = prop.multiProcessorCount * 8, iters = 1024;
        double *sink = nullptr;
        CHECK(hipMalloc(&sink, sizeof(double) * blocks));
        hipEvent_t e0, e1;
        CHECK(hipEventCreate(&e0));
        CHECK(hipEventCreate(&e1));
        const double ops = (double)blocks * 256 * iters;
        for (int f64 = 0; f64 < 2; ++f64) {
            for (int r = 0; r <= reps; ++r) {
                CHECK(hipEventRecord(e0, 0));
                if (f64)
                    hipLaunchKernelGGL(k_lds<double>, dim3(blocks), dim3(256), 0, 0, sink, iters);
                else
                    hipLaunchKernelGGL(k_lds<float>, dim3(blocks), dim3(256), 0, 0, (float *)sink, iters);
                CHECK(hipEventRecord(e1, 0));
                CHECK(hipEventSynchronize(e1));
                float ms = 0.f;
                CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (r > 0)
                    printf("{\"mode\": \"lds\", \"kind\": \"%s\", \"adds\": %.0f, \"ms\": %.4f, \"adds_per_s\": %.4e}\n",
                           f64 ? "f64" : "f32", ops, ms, ops / (ms * 1e-3));
            }
        }
        CHECK(hipFree(sink));
        return 0;
    }
    if (argc < 3) {
        fprintf(stderr, "usage: %s copy|atomic MiB [reps] | lds [reps]\n", argv[0]);
        return 2;
    }
    const size_t mib = strtoull(argv[2], nullptr, 10);
    const int reps = argc > 3 ? atoi(argv[3]) : 5;
    if (mib < 1 || mib > 65536 || reps < 1 || reps > 1000) {
        fprintf(stderr, "MiB must be in 1..65536 and reps in 1..1000\n");
        return 2;
    }
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const size_t bytes = mib << 20;
    if (!strcmp(argv[1], "copy")) {
        float4 *a = nullptr, *b = nullptr;
        CHECK(hipMalloc(&a, bytes));
        CHECK(hipMalloc(&b, bytes));
        CHECK(hipMemset(a, 0, bytes));
        const size_t n = bytes / sizeof(float4);
        const int blocks = prop.multiProcessorCount * 16;
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, 0, a, b, n);  // warm-up
        CHECK(hipDeviceSynchronize());
        for (int r = 0; r < reps; ++r) {
            CHECK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, 0, a, b, n);
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            printf("{\"mode\": \"copy\", \"bytes_read\": %zu, \"bytes_written\": %zu, \"ms\": %.4f, \"gbs\": %.1f}\n", bytes,
                   bytes, ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
        }
        CHECK(hipFree(a));
        CHECK(hipFree(b));
    } else if (!strcmp(argv[1], "atomic")) {
        float *hi = nullptr, *lo = nullptr;
        CHECK(hipMalloc(&hi, bytes));
        CHECK(hipMalloc(&lo, bytes));
        CHECK(hipMemset(hi, 0, bytes));
        CHECK(hipMemset(lo, 0, bytes));
        const uint32_t n = (uint32_t)(bytes / sizeof(float));
        const int blocks = prop.multiProcessorCount * 32, iters = 64;
        const double ops = (double)blocks * 256 * iters;
        const char *kinds[4] = {"plain", "returning+compensated", "f64", "cas64"};
        for (int comp = 0; comp < 4; ++comp) {
            for (int r = 0; r <= reps; ++r) {
                CHECK(hipEventRecord(e0, 0));
                if (comp == 3)  // 64-bit words over the same bytes
                    hipLaunchKernelGGL(k_cas64, dim3(blocks), dim3(256), 0, 0, (unsigned long long *)hi, n / 2, iters);
                else if (comp == 2)  // the same cells as doubles: the first half of both buffers' bytes
                    hipLaunchKernelGGL(k_atomic64, dim3(blocks), dim3(256), 0, 0, (double *)hi, n / 2, iters);
                else if (comp)
                    hipLaunchKernelGGL(k_atomic<true>, dim3(blocks), dim3(256), 0, 0, hi, lo, n, iters);
                else
                    hipLaunchKernelGGL(k_atomic<false>, dim3(blocks), dim3(256), 0, 0, hi, lo, n, iters);
                CHECK(hipEventRecord(e1, 0));
                CHECK(hipEventSynchronize(e1));
                float ms = 0.f;
                CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (r > 0)
                    printf("{\"mode\": \"atomic\", \"kind\": \"%s\", \"grid_bytes\": %zu, \"adds\": %.0f, \"ms\": %.4f, "
                           "\"adds_per_s\": %.4e}\n",
                           kinds[comp], bytes, ops, ms, ops / (ms * 1e-3));
            }
        }
        CHECK(hipFree(hi));
        CHECK(hipFree(lo));
    } else {
        fprintf(stderr, "unknown mode %s\n", argv[1]);
        return 2;
    }
    return 0;
}
