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

// ---------------------------------------------------------------------------
// VALU issue-rate probes: each thread runs `iters` rounds of 16 independent
// dependency chains of one instruction kind, so the measured rate is the
// issue limit of that instruction, not its latency. The result is folded and
// stored once per thread so nothing is optimised away.
// ---------------------------------------------------------------------------

template <int OP>
__global__ __launch_bounds__(256) void calib_valu_kernel(uint32_t *out, uint32_t iters,
                                                         uint32_t seed)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[16];
#pragma unroll
    for (int j = 0; j < 16; j++) a[j] = gid * 2654435761u + (uint32_t)j * 40503u + seed;
    const uint32_t s2 = seed * 7u + 1u;
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const uint32_t b = a[(j + 1) & 15];
            if (OP == 0) a[j] = __builtin_amdgcn_bitop3_b32(a[j], b, seed, 0xBEu);
            if (OP == 1) a[j] = __builtin_amdgcn_alignbit(a[j], b, j + 1);
            if (OP == 2) a[j] = (uint32_t)__popc(a[j]) + b;   // v_bcnt_u32_b32, accumulating
            if (OP == 3) a[j] = min(min(a[j], b), seed ^ (uint32_t)j);  // v_min3_u32
            if (OP == 4) a[j] = a[j] ^ b;
            // chains that read only themselves and scalar operands
            if (OP == 5) a[j] = __builtin_amdgcn_bitop3_b32(a[j], seed, s2, 0xBEu);
            if (OP == 6) a[j] = (uint32_t)__popc(a[j] ^ seed);
        }
    }
    uint32_t x = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) x ^= a[j];
    out[gid] = x;
}

// Time `op` (0 bitop3, 1 alignbit, 2 bcnt, 3 min3, 4 xor; 5 bitop3 and 6
// xor + bcnt on self-only chains) over blocks x 256
// threads; returns the rate in giga lane-operations per second (16 chains x
// iters rounds x threads / time), or a negative HIP error code.
extern "C" double ifa_calib_valu(int op, uint32_t blocks, uint32_t iters)
{
    if (op < 0 || op > 6 || blocks == 0 || iters == 0) return -1.0;
    const uint64_t threads = (uint64_t)blocks * 256u;
    uint32_t *out = nullptr;
    hipError_t e = hipMalloc((void **)&out, threads * sizeof(uint32_t));
    if (e != hipSuccess) return -(double)e;
    void (*fns[7])(uint32_t *, uint32_t, uint32_t) = {
        calib_valu_kernel<0>, calib_valu_kernel<1>, calib_valu_kernel<2>, calib_valu_kernel<3>,
        calib_valu_kernel<4>, calib_valu_kernel<5>, calib_valu_kernel<6>};
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(fns[op], dim3(blocks), dim3(256), 0, 0, out, iters, 12345u);   // warm up
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL(fns[op], dim3(blocks), dim3(256), 0, 0, out, iters, 54321u);
    (void)hipEventRecord(b, 0);
    e = hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (e != hipSuccess) return -(double)e;
    return (double)threads * iters * 16.0 / (ms * 1e-3) / 1e9;
}

// ---------------------------------------------------------------------------
// Matrix-core probes for the fp4 (e2m1) MFMA of gfx950,
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales (E8M0 exponent 127):
// one wave's D for given A and B register contents (to read the operand
// lane layout), and the sustained rate with independent accumulators.
// ---------------------------------------------------------------------------

typedef int calib_v8i __attribute__((ext_vector_type(8)));
typedef float calib_v16f __attribute__((ext_vector_type(16)));
typedef float calib_v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64) void calib_mfma_layout_kernel(const uint32_t *a, const uint32_t *b,
                                                               float *d)
{
    const uint32_t l = threadIdx.x;
    calib_v8i va = {}, vb = {};
    for (int j = 0; j < 4; j++) {
        va[j] = (int)a[4 * l + j];
        vb[j] = (int)b[4 * l + j];
    }
    calib_v16f acc = {};
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, acc, 4, 4, 0, 127, 0, 127);
    for (int j = 0; j < 16; j++) d[16 * l + j] = acc[j];
}

// a, b: 64 lanes x 4 dwords of packed fp4 (host memory); d: 64 lanes x 16
// floats (host memory). Returns 0 or a HIP error code.
extern "C" int ifa_calib_mfma_layout(const uint32_t *a, const uint32_t *b, float *d)
{
    uint32_t *da = nullptr, *db = nullptr;
    float *dd = nullptr;
    hipError_t e = hipMalloc((void **)&da, 256 * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&db, 256 * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&dd, 1024 * 4);
    if (e == hipSuccess) e = hipMemcpy(da, a, 256 * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(db, b, 256 * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(calib_mfma_layout_kernel, dim3(1), dim3(64), 0, 0, da, db, dd);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(d, dd, 1024 * 4, hipMemcpyDeviceToHost);
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (dd) (void)hipFree(dd);
    return (int)e;
}

template <int SHAPE>
__global__ __launch_bounds__(256) void calib_mfma_rate_kernel(float *out, uint32_t iters,
                                                              uint32_t seed)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    calib_v8i va = {}, vb = {};
    for (int j = 0; j < 4; j++) {
        va[j] = (int)((gid * 2654435761u + seed * (uint32_t)(j + 1)) & 0x77777777u);
        vb[j] = (int)((gid * 40503u + seed + (uint32_t)j * 977u) & 0x77777777u);
    }
    float s = 0.f;
    if (SHAPE == 0) {
        calib_v16f c0 = {}, c1 = {}, c2 = {}, c3 = {};
        for (uint32_t i = 0; i < iters; i++) {
            c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, c0, 4, 4, 0, 127, 0, 127);
            c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(vb, va, c1, 4, 4, 0, 127, 0, 127);
            c2 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, va, c2, 4, 4, 0, 127, 0, 127);
            c3 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(vb, vb, c3, 4, 4, 0, 127, 0, 127);
        }
        for (int j = 0; j < 16; j++) s += c0[j] + c1[j] + c2[j] + c3[j];
    } else {
        calib_v4f c0 = {}, c1 = {}, c2 = {}, c3 = {};
        for (uint32_t i = 0; i < iters; i++) {
            c0 = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(va, vb, c0, 4, 4, 0, 127, 0, 127);
            c1 = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(vb, va, c1, 4, 4, 0, 127, 0, 127);
            c2 = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(va, va, c2, 4, 4, 0, 127, 0, 127);
            c3 = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(vb, vb, c3, 4, 4, 0, 127, 0, 127);
        }
        for (int j = 0; j < 4; j++) s += c0[j] + c1[j] + c2[j] + c3[j];
    }
    out[gid] = s;
}

// Rate of the fp4 MFMA (shape 0: 32x32x64, 1: 16x16x128) over blocks x 256
// threads, four independent accumulators per wave; returns dense TFLOP/s
// (2 x M x N x K per instruction), or a negative HIP error code.
extern "C" double ifa_calib_mfma(int shape, uint32_t blocks, uint32_t iters)
{
    if (shape < 0 || shape > 1 || blocks == 0 || iters == 0) return -1.0;
    const uint64_t threads = (uint64_t)blocks * 256u;
    float *out = nullptr;
    hipError_t e = hipMalloc((void **)&out, threads * sizeof(float));
    if (e != hipSuccess) return -(double)e;
    void (*fn)(float *, uint32_t, uint32_t) =
        shape == 0 ? calib_mfma_rate_kernel<0> : calib_mfma_rate_kernel<1>;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, 0, out, iters, 12345u);
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, 0, out, iters, 54321u);
    (void)hipEventRecord(b, 0);
    e = hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (e != hipSuccess) return -(double)e;
    const double waves = (double)threads / 64.0;
    const double flops = shape == 0 ? 2.0 * 32 * 32 * 64 : 2.0 * 16 * 16 * 128;
    return waves * iters * 4.0 * flops / (ms * 1e-3) / 1e12;
}

// Overlap probe: waves of one launch run either fp4 MFMA chains (four
// independent accumulators) or v_max3_u32 chains (16 independent), chosen by
// mode: 0 all MFMA, 1 all VALU, 2 even waves MFMA and odd waves VALU, 3 every
// wave both, interleaved one MFMA to four VALU instructions. Timing them
// shows whether the matrix core and the VALU run concurrently, across waves
// (2) and within one wave (3).
__global__ __launch_bounds__(256) void calib_mix_kernel(float *out, uint32_t iters, uint32_t mode,
                                                        uint32_t seed)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t wv = gid >> 6;
    const bool do_mfma = mode == 0 || (mode == 2 && (wv & 1u) == 0u);
    float s = 0.f;
    if (mode == 3) {
        calib_v8i va = {}, vb = {};
        for (int j = 0; j < 4; j++) {
            va[j] = (int)((gid * 2654435761u + seed * (uint32_t)(j + 1)) & 0x77777777u);
            vb[j] = (int)((gid * 40503u + seed + (uint32_t)j * 977u) & 0x77777777u);
        }
        calib_v16f c0 = {}, c1 = {}, c2 = {}, c3 = {};
        uint32_t a[16];
#pragma unroll
        for (int j = 0; j < 16; j++) a[j] = gid * 2654435761u + (uint32_t)j * 40503u + seed;
        for (uint32_t i = 0; i < iters; i++) {
            c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, c0, 4, 4, 0, 127, 0, 127);
            c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(vb, va, c1, 4, 4, 0, 127, 0, 127);
            c2 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, va, c2, 4, 4, 0, 127, 0, 127);
            c3 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(vb, vb, c3, 4, 4, 0, 127, 0, 127);
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int j = 0; j < 16; j++)
                    a[j] = max(max(a[j], a[(j + 1) & 15] ^ seed), a[(j + 5) & 15] + seed);
            for (int q = 0; q < 4; q++) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 24, 0);
            }
        }
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            s += c0[j] + c1[j] + c2[j] + c3[j];
            x ^= a[j];
        }
        s += (float)x;
    } else if (do_mfma) {
        calib_v8i va = {}, vb = {};
        for (int j = 0; j < 4; j++) {
            va[j] = (int)((gid * 2654435761u + seed * (uint32_t)(j + 1)) & 0x77777777u);
            vb[j] = (int)((gid * 40503u + seed + (uint32_t)j * 977u) & 0x77777777u);
        }
        calib_v16f c0 = {}, c1 = {}, c2 = {}, c3 = {};
        for (uint32_t i = 0; i < iters; i++) {
            c0 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, c0, 4, 4, 0, 127, 0, 127);
            c1 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(vb, va, c1, 4, 4, 0, 127, 0, 127);
            c2 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, va, c2, 4, 4, 0, 127, 0, 127);
            c3 = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(vb, vb, c3, 4, 4, 0, 127, 0, 127);
        }
        for (int j = 0; j < 16; j++) s += c0[j] + c1[j] + c2[j] + c3[j];
    } else {
        uint32_t a[16];
#pragma unroll
        for (int j = 0; j < 16; j++) a[j] = gid * 2654435761u + (uint32_t)j * 40503u + seed;
        // 8 x 16 max3 per iteration: as many VALU issue slots as 4 MFMAs
        // leave at one VALU instruction per 4 clocks
        for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int j = 0; j < 16; j++)
                    a[j] = max(max(a[j], a[(j + 1) & 15] ^ seed), a[(j + 5) & 15] + seed);
        }
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < 16; j++) x ^= a[j];
        s = (float)x;
    }
    out[gid] = s;
}

// Milliseconds of one calib_mix_kernel launch over blocks x 256 threads, or
// a negative HIP error code.
extern "C" double ifa_calib_mix(uint32_t mode, uint32_t blocks, uint32_t iters)
{
    if (mode > 3 || blocks == 0 || iters == 0) return -1.0;
    const uint64_t threads = (uint64_t)blocks * 256u;
    float *out = nullptr;
    hipError_t e = hipMalloc((void **)&out, threads * sizeof(float));
    if (e != hipSuccess) return -(double)e;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(calib_mix_kernel, dim3(blocks), dim3(256), 0, 0, out, iters, mode, 12345u);
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL(calib_mix_kernel, dim3(blocks), dim3(256), 0, 0, out, iters, mode, 54321u);
    (void)hipEventRecord(b, 0);
    e = hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (e != hipSuccess) return -(double)e;
    return ms;
}
