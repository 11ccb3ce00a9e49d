// ifa_calib.hip -- a plain device-to-device copy kernel of known size, used to
// calibrate the HBM byte counters (FETCH_SIZE / WRITE_SIZE) that profiling
// reads for the scan kernel. Not part of the scan path.
#include <hip/hip_runtime.h>
#include <stdint.h>

__global__ __launch_bounds__(256) void calib_copy_kernel(const uint4 *__restrict__ src,
                                                         uint4 *__restrict__ dst, uint64_t n)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

// Copy `bytes` (rounded down to 16) from one fresh device buffer to another,
// `reps` times, one kernel launch each. Returns 0 on success, else the HIP
// error code.
extern "C" int ifa_calib_copy(uint64_t bytes, int reps, double *ms_per_copy)
{
    const uint64_t n = bytes / 16;
    if (n == 0 || reps < 1) return (int)hipErrorInvalidValue;
    uint4 *src = nullptr, *dst = nullptr;
    hipError_t e = hipMalloc((void **)&src, n * 16);
    if (e != hipSuccess) return (int)e;
    e = hipMalloc((void **)&dst, n * 16);
    if (e != hipSuccess) {
        (void)hipFree(src);
        return (int)e;
    }
    (void)hipMemset(src, 1, n * 16);
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    const uint32_t grid = 256 * 8 * 4;   // 4 waves per SIMD-slot worth of workgroups per CU
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < reps; r++)
        hipLaunchKernelGGL(calib_copy_kernel, dim3(grid), dim3(256), 0, 0, src, dst, n);
    (void)hipEventRecord(b, 0);
    e = hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (ms_per_copy) *ms_per_copy = ms / reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(src);
    (void)hipFree(dst);
    return (int)e;
}
