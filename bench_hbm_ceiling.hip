// bench_hbm_ceiling.hip -- the streaming bandwidth this GPU actually reaches,
// as the practical ceiling beside the vendor's 8 TB/s for the HBM-bound
// collide-stream kernel.  Plain kernels over device buffers of 64 MB to
// 2 GB, best of three grid sizes:
//   copy4:   b[i] = a[i] with 16-byte loads and stores, grid-stride loop;
//   stream7: 7 fields in, 7 fields out, one float per lane and field (the
//            collide kernel's traffic shape without its halo and ring);
//   stream7x2, stream7x4: the same with 2 or 4 consecutive floats per lane
//            and field (8- and 16-byte accesses).
// Bytes counted: everything read plus everything written.  Built next to
// bench.py by the package build; run as ./bench_hbm_ceiling.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define HIP_OK(call)                                                                                    \
    do {                                                                                                \
        const hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                         \
            std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));                      \
            std::exit(1);                                                                               \
        }                                                                                               \
    } while (0)

__global__ void copy4(const float4* __restrict__ a, float4* __restrict__ b, long n4)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) b[i] = a[i];
}

// a and b hold 7 fields of m floats each
__global__ void stream7(const float* __restrict__ a, float* __restrict__ b, long m)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        float v[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = a[k * m + i];
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < 7; ++k) s += v[k];
#pragma unroll
        for (int k = 0; k < 7; ++k) b[k * m + i] = v[k] + s * 1e-30f;
    }
}

// the same with V consecutive floats per lane and field (m a multiple of V)
template <int V>
__global__ void stream7v(const float* __restrict__ a, float* __restrict__ b, long m)
{
    typedef float vec __attribute__((ext_vector_type(V)));
    const long mv = m / V;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < mv; i += stride) {
        vec v[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = reinterpret_cast<const vec*>(a + k * m)[i];
        vec s = v[0];
#pragma unroll
        for (int k = 1; k < 7; ++k) s += v[k];
#pragma unroll
        for (int k = 0; k < 7; ++k) reinterpret_cast<vec*>(b + k * m)[i] = v[k] + s * 1e-30f;
    }
}

int main()
{
    const long sizes_mb[] = {64, 256, 1024, 2048};
    const int grids[] = {1024, 4096, 16384};
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    std::printf("%-9s %8s %12s %10s %8s\n", "kernel", "MB", "best us", "TB/s", "grid");
    for (const long mb : sizes_mb) {
        const long n = mb * 1024 * 1024 / 4;  // floats per buffer
        float *a = nullptr, *b = nullptr;
        HIP_OK(hipMalloc(&a, n * sizeof(float)));
        HIP_OK(hipMalloc(&b, n * sizeof(float)));
        HIP_OK(hipMemset(a, 0, n * sizeof(float)));
        const long m7 = (n / 7) / 4 * 4;  // floats per field, a multiple of 4
        for (int kind = 0; kind < 4; ++kind) {
            double best = 1e30;
            int best_grid = 0;
            for (const int grid : grids) {
                auto launch = [&]() {
                    if (kind == 0)
                        hipLaunchKernelGGL(copy4, dim3(grid), dim3(256), 0, 0, reinterpret_cast<const float4*>(a),
                                           reinterpret_cast<float4*>(b), n / 4);
                    else if (kind == 1)
                        hipLaunchKernelGGL(stream7, dim3(grid), dim3(256), 0, 0, a, b, m7);
                    else if (kind == 2)
                        hipLaunchKernelGGL(stream7v<2>, dim3(grid), dim3(256), 0, 0, a, b, m7);
                    else
                        hipLaunchKernelGGL(stream7v<4>, dim3(grid), dim3(256), 0, 0, a, b, m7);
                };
                for (int w = 0; w < 3; ++w) launch();
                HIP_OK(hipGetLastError());
                HIP_OK(hipDeviceSynchronize());
                const int reps = mb <= 256 ? 50 : 10;
                HIP_OK(hipEventRecord(e0, 0));
                for (int r = 0; r < reps; ++r) launch();
                HIP_OK(hipEventRecord(e1, 0));
                HIP_OK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, e0, e1));
                const double t = ms * 1e-3 / reps;
                if (t < best) {
                    best = t;
                    best_grid = grid;
                }
            }
            const double bytes = kind == 0 ? 2.0 * (n / 4) * 16 : 2.0 * 7 * m7 * 4;
            const char* names[] = {"copy4", "stream7", "stream7x2", "stream7x4"};
            std::printf("%-9s %8ld %12.2f %10.2f %8d\n", names[kind], mb, best * 1e6, bytes / best / 1e12,
                        best_grid);
            std::fflush(stdout);
        }
        HIP_OK(hipFree(a));
        HIP_OK(hipFree(b));
    }
    return 0;
}
