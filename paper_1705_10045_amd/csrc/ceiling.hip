// Bandwidth ceiling probe (libceiling.so, used by the benchmark's --ceiling mode only): how fast
// a kernel that reads and writes every population once can move the step's state on this GPU.
// Two access orders over a state of `planes` arrays of `n` floats (the step's SoA layout):
//   flat  - the state as one array, 16-byte loads and non-temporal 16-byte stores, grid-stride;
//   sweep - every workgroup takes a run of nodes and copies it in all planes, as the step reads
//           all populations of the same nodes together.
// Not part of the library's ABI; nothing of the method is computed here.
#include <hip/hip_runtime.h>

#include <cstddef>

namespace {

constexpr int kThreads = 256;
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kThreads)
k_copy_flat(const v4f* __restrict__ src, v4f* __restrict__ dst, size_t n4)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(src[i], dst + i);
}

// run of nodes per workgroup and plane: 4 floats per thread
constexpr int kRun = 4 * kThreads;

__global__ void __launch_bounds__(kThreads)
k_copy_sweep(const float* __restrict__ src, float* __restrict__ dst, size_t n, int planes)
{
    const size_t nruns = n / kRun;
    for (size_t r = blockIdx.x; r < nruns; r += gridDim.x) {
        const size_t i = r * kRun + 4 * (size_t)threadIdx.x;
#pragma unroll 4
        for (int k = 0; k < planes; ++k) {
            const v4f v = *(const v4f*)(src + (size_t)k * n + i);
            __builtin_nontemporal_store(v, (v4f*)(dst + (size_t)k * n + i));
        }
    }
}

}  // namespace

// Copies `planes` x `n` floats from src to dst `reps` times with the given order (0 flat,
// 1 sweep) and returns the mean milliseconds per copy in *ms (events on the null stream).
// n must be a multiple of 1024; returns a hipError_t value.
extern "C" int lbm_probe_copy(const void* src, void* dst, size_t n, int planes, int order, int reps,
                              int blocks, float* ms)
{
    if (n % kRun != 0 || planes < 1 || reps < 1 || blocks < 1 || !ms) return (int)hipErrorInvalidValue;
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return (int)e;
    auto launch = [&]() {
        if (order == 0)
            hipLaunchKernelGGL(k_copy_flat, dim3(blocks), dim3(kThreads), 0, 0, (const v4f*)src,
                               (v4f*)dst, n * (size_t)planes / 4);
        else
            hipLaunchKernelGGL(k_copy_sweep, dim3(blocks), dim3(kThreads), 0, 0, (const float*)src,
                               (float*)dst, n, planes);
    };
    launch();   // warm-up
    e = hipEventRecord(a, 0);
    for (int i = 0; i < reps && e == hipSuccess; ++i) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, 0);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    *ms = t / reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return (int)e;
}
